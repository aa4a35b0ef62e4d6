"""GPU parity: every entry point of the C ABI against the FP64 CPU oracle on the
same seeded inputs.  Tolerances: filtered block 1e-12 relative Frobenius,
Ritz values 1e-10 relative to max(|theta|, s) with s = max(|a0|, |b|),
orthonormality ||Yhat^T Yhat - I||_2 <= 1e-12."""
import numpy as np
import pytest

import oracle
import synth
from oracle import core

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def mkplan(lib, P):
    return lib.Plan(P.grid, P.stencil, P.J)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relf(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def ritz_rel(t_gpu, t_ora, s):
    return float(np.max(np.abs(t_gpu - t_ora) / np.maximum(np.abs(t_ora), s)))


def mixed_problem():
    J = np.array([8, 16, 24, 40, 64, 128, 72, 88, 104, 120, 56, 32], dtype=np.int32)
    return synth.make_blocks((4, 3, 1), 5, J)


def large_alb_problem():
    """ALB counts above 128 up to 256 (the paper's bulk system has 200 per
    element), mixed with small ones, on a 3 x 2 sheet."""
    J = np.array([200, 256, 129, 64, 144, 16], dtype=np.int32)
    return synth.make_blocks((3, 2, 1), 5, J)


PROBLEMS = {
    "tiny": lambda: synth.make_problem(synth.TINY),
    "len1_z_7pt": lambda: synth.make_blocks((3, 2, 1), 7, np.full(6, 24, dtype=np.int32)),
    "mixed_5pt": mixed_problem,
    "odd_3x3x3_nb40": lambda: synth.make_blocks((3, 3, 3), 7, np.full(27, 40, dtype=np.int32)),
    "large_alb_5pt": large_alb_problem,
    "alb200_2x2x2": lambda: synth.make_blocks((2, 2, 2), 7, np.full(8, 200, dtype=np.int32)),
}


# ---------------------------------------------------------------- filter
@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("ns,m", [(48, 10), (1, 3), (130, 7), (257, 2)])
def test_filter_f64_matches_oracle(lib, name, ns, m):
    P = PROBLEMS[name]()
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    X = synth.make_start_block(P.J, ns)
    a, b, a0 = 0.3, 5.5, -1.2
    ref = oracle.chebyshev_filter(oracle.DenseOperator(H), X, m, a, b, a0)
    plan = mkplan(lib, P)
    Y = plan.filter(dev(P.packed()), dev(X), m, a, b, a0)
    assert relf(host(Y), ref) <= 1e-12


def test_filter_degree_zero_one_and_strided(lib):
    P = synth.make_problem(synth.TINY)
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    plan = mkplan(lib, P)
    Hd = dev(P.packed())
    X = synth.make_start_block(P.J, 40)
    # strided views: leading dimensions larger than ns
    Xbig = dev(np.concatenate([X, np.zeros((P.N, 9))], axis=1))
    Xv = Xbig[:, :40]
    Ybig = torch.full((P.N, 57), 7.0, dtype=torch.float64, device="cuda")
    Yv = Ybig[:, 3:43]
    for m in (0, 1, 2):
        plan.filter(Hd, Xv, m, 0.1, 4.0, -0.9, out=Yv)
        ref = oracle.chebyshev_filter(oracle.DenseOperator(H), X, m, 0.1, 4.0, -0.9)
        assert relf(host(Yv), ref) <= 1e-12
    yb = host(Ybig)
    assert np.all(yb[:, :3] == 7.0) and np.all(yb[:, 43:] == 7.0)   # untouched outside the view


def test_filter_diff_workload_block_mode(lib):
    w = synth.DIFF
    P = synth.make_problem(w)
    X = synth.make_start_block(P.J, w.ns)
    a, b, a0 = 0.0, 5.8, -1.4
    bop = oracle.BlockOperator(P.grid, P.stencil, P.J, P.blocks)
    ref = oracle.chebyshev_filter(bop, X, w.m, a, b, a0)
    plan = mkplan(lib, P)
    Y = plan.filter(dev(P.packed()), dev(X), w.m, a, b, a0)
    assert relf(host(Y), ref) <= 1e-12


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("ns,m", [(64, 10), (1, 3), (130, 7), (257, 2), (9, 1)])
def test_filter_f32_shapes(lib, name, ns, m):
    """FP32 storage and MFMA over every grid shape and ragged column count: the
    error against the FP64 oracle is that of 24-bit mantissas."""
    P = PROBLEMS[name]()
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    X = synth.make_start_block(P.J, ns)
    a, b, a0 = 0.3, 5.5, -1.2
    ref = oracle.chebyshev_filter(oracle.DenseOperator(H), X, m, a, b, a0)
    plan = mkplan(lib, P)
    Y = plan.filter(dev(P.packed()), dev(X), m, a, b, a0, dtype=lib.F32)
    err = relf(host(Y), ref)
    assert 1e-10 < err <= 1e-5


def test_filter_f32_error_is_small(lib):
    P = synth.make_problem(synth.TINY)
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    X = synth.make_start_block(P.J, 64)
    a, b, a0 = 0.2, 5.0, -1.0
    ref = oracle.chebyshev_filter(oracle.DenseOperator(H), X, 10, a, b, a0)
    plan = mkplan(lib, P)
    Y = plan.filter(dev(P.packed()), dev(X), 10, a, b, a0, dtype=lib.F32)
    err = relf(host(Y), ref)
    print(f"FP32 filter relative error vs FP64 oracle: {err:.3e}")
    assert 1e-9 < err <= 1e-4


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("ns,m", [(64, 10), (1, 3), (130, 7), (257, 2), (9, 1)])
def test_filter_bf16_error_is_small(lib, name, ns, m):
    """BF16 storage of H and of the recurrence, FP32 accumulation: the error
    against the FP64 oracle is that of 8-bit mantissas (loose bound), and far
    above FP64 rounding (so the low-precision kernel really ran)."""
    P = PROBLEMS[name]()
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    X = synth.make_start_block(P.J, ns)
    a, b, a0 = 0.3, 5.5, -1.2
    ref = oracle.chebyshev_filter(oracle.DenseOperator(H), X, m, a, b, a0)
    plan = mkplan(lib, P)
    Y = plan.filter(dev(P.packed()), dev(X), m, a, b, a0, dtype=lib.BF16)
    err = relf(host(Y), ref)
    print(f"BF16 filter relative error vs FP64 oracle ({name}, ns={ns}, m={m}): {err:.3e}")
    assert 1e-6 < err <= 3e-2


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("ns,m", [(64, 10), (1, 3), (130, 7), (257, 2), (9, 1)])
def test_filter_split_bf16_error(lib, name, ns, m):
    """Split BF16 (hi + lo pairs, three BF16 MFMAs per product): the error
    against the FP64 oracle is that of ~16-bit mantissas -- far below plain
    BF16's on the same input and far above FP64 rounding."""
    P = PROBLEMS[name]()
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    X = synth.make_start_block(P.J, ns)
    a, b, a0 = 0.3, 5.5, -1.2
    ref = oracle.chebyshev_filter(oracle.DenseOperator(H), X, m, a, b, a0)
    plan = mkplan(lib, P)
    Hd, Xd = dev(P.packed()), dev(X)
    e3 = relf(host(plan.filter(Hd, Xd, m, a, b, a0, dtype=lib.BF16X3)), ref)
    e1 = relf(host(plan.filter(Hd, Xd, m, a, b, a0, dtype=lib.BF16)), ref)
    print(f"split-BF16 filter relative error ({name}, ns={ns}, m={m}): {e3:.3e} (plain BF16 {e1:.3e})")
    assert 1e-10 < e3 <= 2e-4
    assert e3 <= e1 / 30


def test_filter_rejects_bad_arguments(lib):
    P = synth.make_problem(synth.TINY)
    plan = mkplan(lib, P)
    Hd = dev(P.packed())
    X = dev(synth.make_start_block(P.J, 8))
    with pytest.raises(lib.ChefsiError) as e:
        plan.filter(Hd, X, 3, 1.0, 1.0, -1.0)
    assert e.value.code == lib.ERR_ARG
    with pytest.raises(lib.ChefsiError):
        plan.filter(Hd, X, 3, 1.0, 2.0, 1.5)
    with pytest.raises(lib.ChefsiError):
        plan.filter(Hd, X, -1, 0.0, 2.0, -1.5)
    with pytest.raises(lib.ChefsiError) as e:
        plan.filter(Hd, X, 3, 0.0, 2.0, -1.5, out=X)
    assert e.value.code == lib.ERR_ARG


# ---------------------------------------------------------------- Cholesky-QR
@pytest.mark.parametrize("n,ns,passes", [(256, 48, 2), (256, 48, 1), (3000, 200, 2), (10368, 512, 2), (700, 65, 2)])
def test_orthonormalize_matches_oracle(lib, n, ns, passes):
    g = np.random.default_rng(n + ns)
    Y = g.standard_normal((n, ns)) @ np.diag(np.logspace(0, 2, ns))
    Yh_o, U_o, _ = oracle.cholesky_qr(Y, passes)
    Yd = dev(Y)
    U = lib.orthonormalize(Yd, passes=passes, want_U=True)
    Yh = host(Yd)
    kappa = np.linalg.cond(Y)
    assert np.linalg.norm(Yh.T @ Yh - np.eye(ns), 2) <= (1e-12 if passes == 2 else 1e-15 * kappa ** 2 * 50)
    Uh = host(U)
    assert np.allclose(np.tril(Uh, -1), 0.0)
    assert np.linalg.norm(Uh - U_o) / np.linalg.norm(U_o) <= 1e-12 * kappa
    assert np.linalg.norm(Yh - Yh_o) / np.linalg.norm(Yh_o) <= 1e-13 * kappa ** (2 if passes == 1 else 1) * 10


@pytest.mark.parametrize("n,ns,cond", [(4000, 64, False), (3000, 200, True)])
def test_orthonormalize_auto_passes_match_oracle(lib, n, ns, cond):
    """passes = 0: a tall well-conditioned block keeps one pass, a block with
    two nearly parallel columns takes two, as the oracle decides; results
    match the oracle's and are orthonormal to 1e-12."""
    g = np.random.default_rng(n + 7)
    Y = g.standard_normal((n, ns)) * np.logspace(0, 3, ns)[None, :]
    if cond:
        Y[:, 11] = Y[:, 5] * 7.0 + 1e-5 * g.standard_normal(n)
    Yh_o, U_o, Us_o = oracle.cholesky_qr(Y, 0)
    assert len(Us_o) == (2 if cond else 1)
    Yd = dev(Y)
    U = lib.orthonormalize(Yd, passes=0, want_U=True)
    Yh = host(Yd)
    assert np.linalg.norm(Yh.T @ Yh - np.eye(ns), 2) <= 1e-12
    assert np.linalg.norm(host(U) - U_o) / np.linalg.norm(U_o) <= 1e-12 * np.linalg.cond(Y)
    assert np.linalg.norm(Yh - Yh_o) / np.linalg.norm(Yh_o) <= 1e-10


@pytest.mark.parametrize("passes", [0, 1, 2])
def test_orthonormalize_not_pd(lib, passes):
    g = np.random.default_rng(1)
    Y = g.standard_normal((300, 20))
    Y[:, 7] = 0.0
    with pytest.raises(lib.ChefsiError) as e:
        lib.orthonormalize(dev(Y), passes=passes)
    assert e.value.code == lib.ERR_NOT_PD


@pytest.mark.parametrize("passes", [0, 1, 2])
def test_orthonormalize_nonfinite_input(lib, passes):
    """A NaN or an Inf in Y reaches a Cholesky pivot as a non-finite value:
    CHEFSI_ERR_NONFINITE, not NOT_PD."""
    g = np.random.default_rng(2)
    for bad in (float("nan"), float("inf")):
        Y = g.standard_normal((300, 20))
        Y[123, 4] = bad
        with pytest.raises(lib.ChefsiError) as e:
            lib.orthonormalize(dev(Y), passes=passes)
        assert e.value.code == lib.ERR_NONFINITE, (bad, e.value)


def test_orthonormalize_workspace_too_small(lib):
    """A workspace one alignment unit short is refused before any work."""
    import ctypes
    n, ns = 300, 20
    Y = dev(np.random.default_rng(3).standard_normal((n, ns)))
    need = ctypes.c_size_t(0)
    assert lib.lib.chefsi_orthonormalize_workspace_bytes(n, ns, 2, ctypes.byref(need)) == 0
    ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    Y0 = host(Y).copy()
    rc = lib.lib.chefsi_orthonormalize(n, ns, ctypes.c_void_p(Y.data_ptr()), ns, 2, None,
                                       ctypes.c_void_p(ws.data_ptr()), need.value - 256, None)
    assert rc == lib.ERR_WORKSPACE
    assert b"workspace" in lib.lib.chefsi_last_error()
    assert np.array_equal(host(Y), Y0)


@pytest.mark.parametrize("passes", [0, 1, 2])
def test_sweep_nonfinite_x_leaves_x_unchanged(lib, passes):
    """A NaN in X propagates through the filter into the Gram matrix: the sweep
    returns CHEFSI_ERR_NONFINITE and leaves X as it was."""
    P = synth.make_problem(synth.TINY)
    plan = mkplan(lib, P)
    X0 = synth.make_start_block(P.J, 48)
    X0[17, 5] = float("nan")
    X = dev(X0)
    with pytest.raises(lib.ChefsiError) as e:
        plan.sweep(dev(P.packed()), X, 10, bounds=(0.5, 6.0, -1.5), passes=passes)
    assert e.value.code == lib.ERR_NONFINITE
    assert np.array_equal(host(X), X0, equal_nan=True)


@pytest.mark.parametrize("passes", [0, 1, 2])
def test_sweep_not_pd_leaves_x_unchanged(lib, passes):
    """A zero column makes the filtered block rank deficient: the sweep returns
    NOT_PD and X is untouched (the automatic pass count stops after the first
    factor; with 1 or 2 passes the final rotation sees the status word on the
    device and writes nothing)."""
    P = synth.make_problem(synth.TINY)
    plan = mkplan(lib, P)
    X0 = synth.make_start_block(P.J, 48)
    X0[:, 5] = 0.0
    X = dev(X0)
    with pytest.raises(lib.ChefsiError) as e:
        plan.sweep(dev(P.packed()), X, 10, bounds=(0.5, 6.0, -1.5), passes=passes)
    assert e.value.code == lib.ERR_NOT_PD
    assert np.array_equal(host(X), X0)


@pytest.mark.parametrize("passes", [0, 1, 2])
def test_sweep_rejects_warm_ritz_values_above_a_reused_bound(lib, passes):
    """Warm bounds whose reused upper bound lies below the previous top Ritz
    value (Ritz values of another H) would invert the filter; the sweep reports
    ERR_ARG and leaves X unchanged.  chefsi_bounds does the same on the host."""
    w = synth.TINY
    P = synth.make_problem(w)
    plan = mkplan(lib, P)
    Hd = dev(P.packed())
    X0 = synth.make_start_block(P.J, w.ns)
    X = dev(X0)
    ritz, _, bnd, _ = plan.sweep(Hd, X, w.m, v0=dev(synth.make_lanczos_start(P.N)), passes=2)
    top = float(host(ritz)[-1])
    Xs = host(X).copy()
    stale = torch.tensor([0.0, top - 0.25, -1.0], dtype=torch.float64, device="cuda")
    with pytest.raises(lib.ChefsiError) as e:
        plan.sweep(Hd, X, w.m, bounds=stale, ritz=ritz, warm=True, passes=passes)
    assert e.value.code == lib.ERR_ARG
    assert np.array_equal(host(X), Xs)
    # explicit bounds that are not finite
    with pytest.raises(lib.ChefsiError) as e:
        plan.sweep(Hd, X, w.m, bounds=(0.5, float("inf"), -1.0), passes=passes)
    assert e.value.code == lib.ERR_NONFINITE
    assert np.array_equal(host(X), Xs)


def test_binding_rejects_short_or_foreign_tensors_before_the_call(lib):
    P = synth.make_problem(synth.TINY)
    plan = mkplan(lib, P)
    Hd = dev(P.packed())
    X = dev(synth.make_start_block(P.J, 48))
    v0 = dev(synth.make_lanczos_start(P.N))
    bad = [
        lambda: plan.sweep(Hd, X, 10, v0=v0[:-1].clone()),                       # short v0
        lambda: plan.sweep(Hd, X, 10, v0=v0.cpu()),                               # host v0
        lambda: plan.sweep(Hd, X, 10, v0=v0, ritz=torch.zeros(48, device="cuda")),   # float32 ritz
        lambda: plan.sweep(Hd, X, 10, v0=v0, ritz=torch.zeros(47, dtype=torch.float64, device="cuda")),
        lambda: plan.sweep(Hd, X, 10, bounds=torch.zeros(2, dtype=torch.float64, device="cuda")),
        lambda: plan.sweep(Hd, X, 10, v0=v0, ws=torch.empty(1 << 20, dtype=torch.float64, device="cuda")),
        lambda: plan.sweep(Hd, X, 10, v0=v0, warm=True),                          # warm without ritz
        lambda: plan.sweep(Hd, X[:-8], 10, v0=v0),                                # too few rows
        lambda: plan.filter(Hd, X[:, ::2], 4, 0.0, 1.0, -1.0),                    # strided columns
    ]
    for f in bad:
        with pytest.raises(ValueError):
            f()


# ---------------------------------------------------------------- Rayleigh-Ritz
@pytest.mark.parametrize("name,ns", [("tiny", 48), ("mixed_5pt", 100), ("odd_3x3x3_nb40", 300),
                                     ("large_alb_5pt", 130), ("alb200_2x2x2", 260)])
def test_rayleigh_ritz_matches_oracle(lib, name, ns):
    P = PROBLEMS[name]()
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    op = oracle.DenseOperator(H)
    X = synth.make_start_block(P.J, ns)
    Yt = oracle.chebyshev_filter(op, X, 8, 0.5, 6.0, -1.5)
    Yh, _, _ = oracle.cholesky_qr(Yt, 2)
    Xn_o, th_o, r_o, Q_o, _ = oracle.rayleigh_ritz(op, Yh)
    plan = mkplan(lib, P)
    Xn, th, r, Q = plan.rayleigh_ritz(dev(P.packed()), dev(Yh), want_Q=True)
    th, r, Xn, Q = host(th), host(r), host(Xn), host(Q)
    s = 6.0
    assert ritz_rel(th, th_o, s) <= 1e-10
    assert np.max(np.abs(r - r_o)) <= 1e-10 * s
    # eigenvectors: compare columns whose eigenvalue is separated from its neighbours
    gaps = np.minimum(np.diff(th_o, prepend=-np.inf), np.diff(th_o, append=np.inf))
    ok = gaps > 1e-4 * s
    assert np.max(np.abs(Q[:, ok] - Q_o[:, ok])) <= 1e-8
    assert np.max(np.abs(Xn[:, ok] - Xn_o[:, ok])) <= 1e-8
    # clusters (neighbour gaps <= 1e-4 s): the spanned subspaces agree (all
    # principal angles near zero)
    start = 0
    for i in range(1, ns + 1):
        if i == ns or th_o[i] - th_o[i - 1] > 1e-4 * s:
            if i - start >= 2:
                sv = np.linalg.svd(Xn[:, start:i].T @ Xn_o[:, start:i], compute_uv=False)
                assert sv.min() >= 1 - 1e-8, (start, i, sv.min())
            start = i
    assert np.linalg.norm(Xn.T @ Xn - np.eye(ns), 2) <= 1e-12


@pytest.mark.parametrize("ns", [1, 2, 3, 63, 64, 65, 127, 128, 129, 256, 257, 258, 512, 513, 514])
def test_rayleigh_ritz_subspace_sizes(lib, ns):
    """Projected matrices of order 1 to 514: one and several 64 x 64 tiles of
    the tridiagonal reduction, panel boundaries at 64 and 128, ragged tails,
    and a ragged, a full, and a full plus a single-reflector block of the
    back-transformation (blocks of 512 reflectors)."""
    P = PROBLEMS["odd_3x3x3_nb40"]()
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    Yh, _ = np.linalg.qr(np.random.default_rng(ns).standard_normal((P.N, ns)))
    Xn_o, th_o, _, Q_o, _ = oracle.rayleigh_ritz(oracle.DenseOperator(H), Yh)
    Xn, th, _, Q = mkplan(lib, P).rayleigh_ritz(dev(P.packed()), dev(Yh), want_Q=True)
    th, Xn, Q = host(th), host(Xn), host(Q)
    s = float(np.max(np.abs(th_o)))
    assert ritz_rel(th, th_o, s) <= 1e-10
    gaps = np.minimum(np.diff(th_o, prepend=-np.inf), np.diff(th_o, append=np.inf))
    ok = gaps > 1e-4 * s
    assert np.max(np.abs(Q[:, ok] - Q_o[:, ok])) <= 1e-8
    assert np.linalg.norm(Q.T @ Q - np.eye(ns), 2) <= 1e-12
    assert np.linalg.norm(Xn.T @ Xn - np.eye(ns), 2) <= 1e-12


def test_rayleigh_ritz_diagonal_projection(lib):
    """One unit vector per element of an independent set of elements (no two
    are stencil neighbours): the projected matrix is exactly diagonal, so
    every Householder reflector of the reduction is the identity.  The Ritz
    values are the selected diagonal entries of H, sorted, and the Ritz
    vectors are the unit vectors in that order."""
    J = np.full(216, 8, dtype=np.int32)
    P = synth.make_blocks((6, 6, 6), 7, J)
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    rows = []
    for z in range(6):
        for y in range(6):
            for x in range(6):
                if (x + y + z) % 3 == 0:
                    K = x + 6 * (y + 6 * z)
                    rows.append(8 * K + (K % 8))
    rows = np.array(rows)
    ns = rows.size
    Yh = np.zeros((P.N, ns))
    Yh[rows, np.arange(ns)] = 1.0
    Hh = H[np.ix_(rows, rows)]
    assert np.count_nonzero(Hh - np.diag(np.diag(Hh))) == 0
    Xn, th, _, _ = mkplan(lib, P).rayleigh_ritz(dev(P.packed()), dev(Yh), want_Q=True)
    th, Xn = host(th), host(Xn)
    d = np.diag(Hh)
    order = np.argsort(d, kind="stable")
    assert np.min(np.diff(d[order])) > 1e-9
    assert np.max(np.abs(th - d[order])) <= 1e-15 * np.max(np.abs(d))
    assert np.max(np.abs(np.abs(Xn) - Yh[:, order])) <= 1e-15


# ---------------------------------------------------------------- bounds
@pytest.mark.parametrize("name", ["tiny", "mixed_5pt", "large_alb_5pt"])
def test_bounds_match_oracle(lib, name):
    P = PROBLEMS[name]()
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    op = oracle.DenseOperator(H)
    v0 = synth.make_lanczos_start(P.N)
    ns = 48
    b_o, th_l, tau = oracle.lanczos_upper_bound(op, v0, 20)
    a_o, _, a0_o = oracle.bounds_cold(b_o, th_l, tau, ns, P.N)
    plan = mkplan(lib, P)
    Hd = dev(P.packed())
    a, b, a0 = plan.bounds(Hd, dev(v0), 20, ns=ns)
    assert abs(b - b_o) <= 1e-12 * abs(b_o)
    assert abs(a - a_o) <= 1e-10 * abs(b_o) and abs(a0 - a0_o) <= 1e-10 * abs(b_o)
    assert b >= np.linalg.eigvalsh(H)[-1]
    ritz = np.sort(np.random.default_rng(0).uniform(-1, 2, ns))
    a, b, a0 = plan.bounds(Hd, dev(v0), 20, ritz_prev=dev(ritz))
    aw, bw, a0w = oracle.bounds_warm(ritz, b_o)
    assert (a, a0) == (aw, a0w) and abs(b - bw) <= 1e-12 * abs(bw)


# ---------------------------------------------------------------- full cycle
def test_sweep_tiny_external_bounds_match_oracle(lib):
    w = synth.TINY
    P = synth.make_problem(w)
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    op = oracle.DenseOperator(H)
    X0 = synth.make_start_block(P.J, w.ns)
    v0 = synth.make_lanczos_start(P.N)
    _, th_o, r_o, hist = core.run_sweeps(op, X0, v0, w.m, w.sweeps)
    plan = mkplan(lib, P)
    Hd = dev(P.packed())
    X = dev(X0)
    for (bnds, th_i, _) in hist:
        ritz, resid, _, _ = plan.sweep(Hd, X, w.m, bounds=bnds)
        s = max(abs(bnds[2]), abs(bnds[1]))
        assert ritz_rel(host(ritz), th_i, s) <= 1e-10
    k = 3 * w.ns // 4
    lam = np.linalg.eigvalsh(H)
    assert np.max(np.abs(host(ritz)[:k] - lam[:k])) <= 1e-8 * 6


def test_sweep_own_policy_converges_like_oracle(lib):
    w = synth.TINY
    P = synth.make_problem(w)
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    op = oracle.DenseOperator(H)
    X0 = synth.make_start_block(P.J, w.ns)
    v0 = synth.make_lanczos_start(P.N)
    _, th_o, _, hist = core.run_sweeps(op, X0, v0, w.m, w.sweeps)
    plan = mkplan(lib, P)
    Hd, X, v0d = dev(P.packed()), dev(X0), dev(v0)
    ritz = None
    for i in range(w.sweeps):
        ritz, resid, bused, st = plan.sweep(Hd, X, w.m, v0=v0d, ritz=ritz, warm=i > 0, stats=True)
        bo = hist[i][0]
        assert np.max(np.abs(host(bused) - np.array(bo))) <= 1e-9 * 6, (i, host(bused), bo)
        assert st["total_ms"] > 0
    assert ritz_rel(host(ritz), th_o, 6.0) <= 1e-10


@pytest.mark.parametrize("low", ["F32", "BF16", "BF16X3"])
def test_sweep_low_precision_filter_then_f64_finish(lib, low):
    w = synth.TINY
    P = synth.make_problem(w)
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    lam = np.linalg.eigvalsh(H)
    plan = mkplan(lib, P)
    Hd, X, v0d = dev(P.packed()), dev(synth.make_start_block(P.J, w.ns)), dev(synth.make_lanczos_start(P.N))
    ritz = None
    for i in range(6):
        dt = getattr(lib, low) if i < 3 else lib.F64
        ritz, resid, _, _ = plan.sweep(Hd, X, w.m, dtype=dt, v0=v0d, ritz=ritz, warm=i > 0)
    k = 3 * w.ns // 4
    assert np.max(np.abs(host(ritz)[:k] - lam[:k])) <= 1e-9 * 6


@pytest.mark.parametrize("name,ns,m", [("tiny", 48, 10), ("odd_3x3x3_nb40", 300, 12)])
def test_sweep_auto_passes_match_oracle(lib, name, ns, m):
    """passes = 0 with the oracle's bounds: every cycle takes the pass count
    the oracle takes (condition bound of the first factor within 1e-8), its
    Ritz values match the oracle's within 1e-10, and X stays orthonormal to
    1e-12.  passes = 1 (the folded single pass) matches the oracle's single
    pass, within the eps B^2 orthogonality loss of one pass."""
    P = PROBLEMS[name]()
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    op = oracle.DenseOperator(H)
    X0 = synth.make_start_block(P.J, ns)
    v0 = synth.make_lanczos_start(P.N)
    b, thl, tau = oracle.lanczos_upper_bound(op, v0, 20)
    plan = mkplan(lib, P)
    Hd = dev(P.packed())
    eps = np.finfo(np.float64).eps
    for passes in (0, 1):
        bounds = oracle.bounds_cold(b, thl, tau, ns, P.N)
        Xo, X = X0, dev(X0)
        taken = []
        for i in range(5):
            Yt = oracle.chebyshev_filter(op, Xo, m, *bounds)
            Yh, _, Us = oracle.cholesky_qr(Yt, passes)
            Xo, th_o, _, _, _ = oracle.rayleigh_ritz(op, Yh)
            ritz, resid, _, st = plan.sweep(Hd, X, m, bounds=bounds, passes=passes, stats=True)
            B = oracle.cholqr_condition_bound(Us[0])
            Bmax = B if i == 0 else max(Bmax, B)
            tol_orth = 1e-12 if len(Us) == 2 else max(1e-12, 50 * eps * B * B)
            s = max(abs(bounds[2]), abs(bounds[1]))
            assert ritz_rel(host(ritz), th_o, s) <= max(1e-10, 10 * tol_orth), (passes, i)
            Xh = host(X)
            assert np.linalg.norm(Xh.T @ Xh - np.eye(ns), 2) <= tol_orth, (passes, i, B)
            if passes == 1:
                # One pass loses orthogonality like eps B^2, but the span of
                # its output is that of the filtered block to about eps B, and
                # the filter of the next cycle depends only on that span: the
                # Ritz values of span(X) (orthonormalised twice here) match the
                # oracle's Ritz values of span(Y~) (two passes) to ~eps B.
                th_span = oracle.rayleigh_ritz(op, oracle.cholesky_qr(Xh, 2)[0])[1]
                th_ref = oracle.rayleigh_ritz(op, oracle.cholesky_qr(Yt, 2)[0])[1]
                tol_span = max(1e-10, 100 * eps * Bmax)
                assert ritz_rel(th_span, th_ref, s) <= tol_span, (i, B, ritz_rel(th_span, th_ref, s))
            assert st["cholqr_passes"] == len(Us), (passes, i)
            # the first factor of an ill-conditioned block is itself accurate
            # only to about eps B^2 in its small directions; after a lossy
            # single-pass cycle the two inputs differ, so passes = 1 compares
            # the bound of the first cycle only
            if passes == 0 or i == 0:
                assert abs(st["cholqr_cond_bound"] - B) <= (1e-8 + 1e-14 * B * B) * B, \
                    (passes, i, st["cholqr_cond_bound"], B)
            taken.append(int(st["cholqr_passes"]))
            bounds = oracle.bounds_warm(th_o, b)
        print(f"{name} passes={passes}: passes taken per cycle {taken}")


def test_sweep_warm_reuses_the_lanczos_bound(lib):
    """Warm cycles given the previous bounds take b from them and a, a0 from
    the Ritz values: bit-identical to recomputing the (deterministic) Lanczos
    bound every cycle."""
    w = synth.TINY
    P = synth.make_problem(w)
    plan = mkplan(lib, P)
    Hd = dev(P.packed())
    v0d = dev(synth.make_lanczos_start(P.N))
    X0 = synth.make_start_block(P.J, w.ns)
    XA, XB = dev(X0), dev(X0)
    rA = rB = bB = None
    for i in range(4):
        rA, _, bA, _ = plan.sweep(Hd, XA, w.m, v0=v0d, ritz=rA, warm=i > 0, passes=0)
        if i == 0:
            rB, _, bB, _ = plan.sweep(Hd, XB, w.m, v0=v0d, ritz=rB, warm=False, passes=0)
        else:
            rB, _, bB, _ = plan.sweep(Hd, XB, w.m, bounds=bB, ritz=rB, warm=True, passes=0)
        assert torch.equal(bA, bB), (i, host(bA), host(bB))
        assert torch.equal(rA, rB) and torch.equal(XA, XB)
