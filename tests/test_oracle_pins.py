"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, special cases that reduce to textbook or library routines,
invariants and brute force on small inputs.  Each check is chosen so that a
plausible slip (dropped term, wrong sign or index, transposed operand) fails.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import core

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def small_problem(grid=(2, 2, 2), stencil=7, nb=16, **kw):
    J = np.full(grid[0] * grid[1] * grid[2], nb, dtype=np.int32)
    return synth.make_blocks(grid, stencil, J, **kw)


def dense_of(P):
    return oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)


def p_closed(lam, m, a, b, a0):
    """p_m(t) = T_m(L(t)) / T_m(L(a0)) from the closed form of T_m."""
    c, e = (a + b) / 2, (b - a) / 2
    return core.chebyshev_T(m, (np.asarray(lam) - c) / e) / core.chebyshev_T(m, np.array([(a0 - c) / e]))[0]


# ---------------------------------------------------------------- T_m itself
def test_chebyshev_T_exact_rationals():
    """chebyshev_T (cos/cosh closed form) against T_k from the defining
    recurrence T_0 = 1, T_1 = x, T_{k+1} = 2x T_k - T_{k-1} in exact rationals."""
    for x in [Fraction(-7, 3), Fraction(-1), Fraction(-1, 2), Fraction(1, 3), Fraction(9, 10), Fraction(1), Fraction(5, 4), Fraction(3)]:
        T = [Fraction(1), x]
        for _ in range(2, 21):
            T.append(2 * x * T[-1] - T[-2])
        for m in (0, 1, 2, 5, 10, 16, 20):
            got = float(core.chebyshev_T(m, np.array([float(x)]))[0])
            ref = float(T[m])
            assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref)), (x, m, got, ref)


# ---------------------------------------------------------------- P1
def check_filter_diagonal(filter_fn):
    """Filter of a diagonal H against the closed form; returns max rel error."""
    grid, nb = (3, 2, 1), 8
    M = 6
    J = np.full(M, nb, dtype=np.int32)
    P = synth.make_blocks(grid, 7, J, lam_lo=-2.0, lam_hi=6.0, sigma_off=0.0, diag_kind="diag")
    H = dense_of(P)
    d = np.diag(H).copy()
    assert np.count_nonzero(H - np.diag(d)) == 0
    X = synth.make_start_block(J, 5)
    worst = 0.0
    for m, (a, b, a0) in [(10, (0.5, 5.0, -2.5)), (7, (-0.3, 6.5, -1.0)), (1, (1.0, 4.0, -1.0)), (16, (2.0, 5.5, -2.0))]:
        Y = filter_fn(oracle.DenseOperator(H), X, m, a, b, a0)
        ref = p_closed(d, m, a, b, a0)[:, None] * X
        worst = max(worst, float(np.max(np.abs(Y - ref) / (np.abs(ref) + 1e-300 + np.abs(X) * 1e-3))))
    return worst, d


def test_P1_filter_diagonal_closed_form():
    err, d = check_filter_diagonal(oracle.chebyshev_filter)
    # the spectrum straddles [a, b]: values inside and outside are both tested
    assert d.min() < 0.5 and d.max() > 5.0
    assert err <= 1e-12, err


def test_P1_detects_planted_mistakes():
    """Plant slips in a copy of the recurrence; the closed-form pin must fail."""
    def make(mutation):
        def f(op, X, m, a, b, a0):
            c, coefs = core.chebyshev_coefficients(m, a, b, a0)
            if mutation == "sign_c":
                c = -c
            Yp, Y = None, X
            for k, (al, be) in enumerate(coefs):
                if mutation == "drop_beta":
                    be = 0.0
                if mutation == "beta_index" and k > 0:
                    be = coefs[k - 1][1] if k > 1 else be * 1.01
                Yn = al * (op.apply(Y) - c * Y)
                if k > 0:
                    Yn -= be * Yp
                Yp, Y = Y, Yn
            return Y
        return f
    for mut in ("sign_c", "drop_beta", "beta_index"):
        err, _ = check_filter_diagonal(make(mut))
        assert err > 1e-3, mut


def test_filter_degree_zero_and_one():
    P = small_problem()
    H = dense_of(P)
    X = synth.make_start_block(P.J, 4)
    op = oracle.DenseOperator(H)
    assert np.array_equal(oracle.chebyshev_filter(op, X, 0, 0.0, 1.0, -1.0), X)
    a, b, a0 = 0.5, 4.0, -0.5
    c, e = (a + b) / 2, (b - a) / 2
    Y1 = oracle.chebyshev_filter(op, X, 1, a, b, a0)
    ref = (H @ X - c * X) / (a0 - c)    # T_1(L(H)) X / T_1(L(a0))
    assert np.max(np.abs(Y1 - ref)) <= 1e-13 * np.max(np.abs(ref))
    with pytest.raises(ValueError):
        oracle.chebyshev_filter(op, X, 3, 1.0, 1.0, 0.0)
    with pytest.raises(ValueError):
        oracle.chebyshev_filter(op, X, 3, 1.0, 2.0, 1.5)


# ---------------------------------------------------------------- P2
@pytest.mark.parametrize("m", [3, 10, 16])
def test_P2_filter_brute_force_eigendecomposition(m):
    """Y = V diag(p_m(lambda)) V^T X with the eigenpairs from LAPACK (N = 256)."""
    P = synth.make_problem(synth.TINY)
    H = dense_of(P)
    lam, V = np.linalg.eigh(H)
    X = synth.make_start_block(P.J, 12)
    a, b, a0 = 0.2, lam[-1] + 0.3, lam[0] - 0.05
    Y = oracle.chebyshev_filter(oracle.DenseOperator(H), X, m, a, b, a0)
    ref = V @ (p_closed(lam, m, a, b, a0)[:, None] * (V.T @ X))
    rel = np.linalg.norm(Y - ref) / np.linalg.norm(ref)
    assert rel <= 1e-12, rel


# ---------------------------------------------------------------- block mode == dense mode
def test_block_operator_matches_dense():
    for grid, stencil in [((2, 2, 2), 7), ((3, 2, 1), 7), ((4, 3, 1), 5), ((3, 3, 3), 7)]:
        P = small_problem(grid, stencil, nb=8)
        H = dense_of(P)
        # exact unless a length-1 dimension adds three terms onto a diagonal block
        assert np.max(np.abs(H - H.T)) <= 1e-15 * np.max(np.abs(H))
        if 1 not in grid:
            assert np.array_equal(H, H.T)
        bop = oracle.BlockOperator(P.grid, P.stencil, P.J, P.blocks)
        X = synth.make_start_block(P.J, 6)
        assert np.max(np.abs(bop.apply(X) - H @ X)) <= 1e-14 * np.max(np.abs(H @ X)) * 10
        assert np.max(np.abs(bop.apply_T(X) - H.T @ X)) <= 1e-13
    # mixed ALB counts
    J = np.array([8, 16, 24, 8, 16, 8], dtype=np.int32)
    P = synth.make_blocks((3, 2, 1), 5, J)
    H = dense_of(P)
    bop = oracle.BlockOperator(P.grid, P.stencil, P.J, P.blocks)
    X = synth.make_start_block(P.J, 3)
    assert np.max(np.abs(bop.apply(X) - H @ X)) <= 1e-13


def test_block_mode_filter_matches_dense_tiny():
    P = synth.make_problem(synth.TINY)
    H = dense_of(P)
    X = synth.make_start_block(P.J, synth.TINY.ns)
    args = (10, 0.2, 5.0, -1.0)
    Yd = oracle.chebyshev_filter(oracle.DenseOperator(H), X, *args)
    Yb = oracle.chebyshev_filter(oracle.BlockOperator(P.grid, P.stencil, P.J, P.blocks), X, *args)
    assert np.linalg.norm(Yd - Yb) / np.linalg.norm(Yd) <= 1e-13


# ---------------------------------------------------------------- P3
def test_P3_decoupled_blocks_reproduce_block_spectra():
    grid, nb, ns = (2, 2, 1), 12, 16
    J = np.full(4, nb, dtype=np.int32)
    P = synth.make_blocks(grid, 7, J, sigma_off=0.0)
    H = dense_of(P)
    # the off-diagonal blocks are exactly zero, so the spectrum is the union
    # of the drawn per-block spectra; the oracle's Jacobi recovers each one
    for K in range(4):
        w, _ = oracle.jacobi_eigh(P.blocks[K][0])
        assert np.max(np.abs(w - np.sort(P.eigs[K]))) <= 1e-13 * 4
    exact = np.sort(np.concatenate(P.eigs))
    op = oracle.DenseOperator(H)
    X0 = synth.make_start_block(J, ns)
    v0 = synth.make_lanczos_start(P.N)
    _, theta, resid, _ = core.run_sweeps(op, X0, v0, m=14, nsweeps=12)
    k = 3 * ns // 4
    s = max(abs(exact[0]), abs(exact[-1]))
    assert np.max(np.abs(theta[:k] - exact[:k])) <= 1e-12 * s


# ---------------------------------------------------------------- P4
def lattice_eigs(grid, stencil, nb, d, t):
    dims = [0, 1, 2] if stencil == 7 else [0, 1]
    vals = []
    for kx in range(grid[0]):
        for ky in range(grid[1]):
            for kz in range(grid[2]):
                ks = (kx, ky, kz)
                v = d + 2 * t * sum(math.cos(2 * math.pi * ks[i] / grid[i]) for i in dims)
                vals.extend([v] * nb)
    return np.sort(np.array(vals))


@pytest.mark.parametrize("grid,stencil", [((4, 3, 2), 7), ((3, 3, 1), 7), ((4, 4, 1), 5), ((2, 2, 2), 7), ((5, 1, 1), 7)])
def test_P4_scalar_lattice_cosine_band(grid, stencil):
    nb, d, t = 3, 0.7, -0.4
    P = synth.make_scalar_lattice(grid, stencil, nb, d, t)
    H = dense_of(P)
    got = np.linalg.eigvalsh(H)
    ref = lattice_eigs(grid, stencil, nb, d, t)
    assert np.max(np.abs(got - ref)) <= 1e-13
    # Lanczos bound is an upper bound of the analytic band
    b, _, _ = oracle.lanczos_upper_bound(oracle.DenseOperator(H), synth.make_lanczos_start(P.N), 20)
    assert b >= ref[-1] - 1e-12


def test_P4_scalar_lattice_chefsi_ritz_values():
    grid, stencil, nb, d, t = (4, 4, 2), 7, 2, 1.0, -0.5
    P = synth.make_scalar_lattice(grid, stencil, nb, d, t)
    H = dense_of(P)
    ref = lattice_eigs(grid, stencil, nb, d, t)
    # pick ns at a cluster boundary, with the wanted set 3/4 of it
    bounds = np.nonzero(np.diff(ref) > 1e-9)[0] + 1
    ns = int(bounds[bounds >= 24][0])
    X0 = synth.make_start_block(P.J, ns)
    _, theta, _, _ = core.run_sweeps(oracle.DenseOperator(H), X0, synth.make_lanczos_start(P.N), m=12, nsweeps=10)
    k = int(bounds[bounds <= 3 * ns // 4][-1])
    assert np.max(np.abs(theta[:k] - ref[:k])) <= 1e-11


# ---------------------------------------------------------------- P5
@pytest.mark.parametrize("n", [1, 2, 7, 40, 120])
def test_P5_jacobi_vs_lapack(n):
    g = np.random.default_rng(n)
    A = g.standard_normal((n, n))
    A = A + A.T
    w, V = oracle.jacobi_eigh(A)
    wl = np.linalg.eigvalsh(A)
    nrm = np.linalg.norm(A, 2)
    assert np.max(np.abs(w - wl)) <= 1e-13 * nrm * 4
    assert np.linalg.norm(A - (V * w) @ V.T) <= 1e-13 * nrm * n
    assert np.linalg.norm(V.T @ V - np.eye(n)) <= 1e-13 * n
    assert np.all(np.diff(w) >= 0)


# ---------------------------------------------------------------- P6
@pytest.mark.parametrize("passes", [1, 2])
def test_P6_cholesky_qr_equals_householder_qr(passes):
    g = np.random.default_rng(3)
    N, n = 300, 40
    Y = g.standard_normal((N, n)) @ np.diag(np.logspace(0, 3, n))   # cond ~ 1e3
    Yh, U, _ = oracle.cholesky_qr(Y, passes)
    Qh, R = np.linalg.qr(Y)
    sgn = np.sign(np.diag(R))
    Qh, R = Qh * sgn, R * sgn[:, None]
    kappa = np.linalg.cond(Y)
    assert np.allclose(np.triu(U), U) and np.all(np.diag(U) > 0)
    assert np.linalg.norm(Yh @ U - Y) <= 1e-14 * np.linalg.norm(Y) * 10
    tol_q = 1e-15 * kappa ** (2 if passes == 1 else 1) * 100
    assert np.linalg.norm(Yh - Qh) <= tol_q
    assert np.linalg.norm(U - R) / np.linalg.norm(R) <= tol_q
    orth = np.linalg.norm(Yh.T @ Yh - np.eye(n), 2)
    assert orth <= (1e-12 if passes == 2 else 1e-15 * kappa ** 2 * 100)


def test_P6_cholesky_upper_textbook_and_not_pd():
    g = np.random.default_rng(5)
    A = g.standard_normal((30, 30))
    S = A.T @ A + 0.1 * np.eye(30)
    U = oracle.cholesky_upper(S)
    assert np.max(np.abs(U - np.linalg.cholesky(S).T)) <= 1e-13 * np.max(np.abs(U))
    Y = g.standard_normal((50, 6))
    Y[:, 4] = 0.0       # rank deficient: the pivot of column 4 is exactly zero
    with pytest.raises(core.NotPositiveDefinite):
        oracle.cholesky_qr(Y, 1)
    Y[:, 4] = np.nan
    with pytest.raises(core.NotPositiveDefinite):
        oracle.cholesky_qr(Y, 1)


def test_P6_detects_transposed_solve():
    g = np.random.default_rng(9)
    Y = g.standard_normal((60, 8))
    U = oracle.cholesky_upper(Y.T @ Y)
    good = oracle.solve_right_upper(Y, U)
    bad = oracle.solve_right_upper(Y, U.T.copy())
    assert np.linalg.norm(good.T @ good - np.eye(8)) < 1e-12
    assert np.linalg.norm(bad.T @ bad - np.eye(8)) > 1e-3


# ---------------------------------------------------------------- P7
def test_P7_rayleigh_ritz_invariants():
    P = synth.make_problem(synth.TINY)
    H = dense_of(P)
    lam, V = np.linalg.eigh(H)
    op = oracle.DenseOperator(H)
    g = np.random.default_rng(1)
    ns = 20
    # interlacing: theta_i >= lambda_i for any orthonormal basis
    Yh, _, _ = oracle.cholesky_qr(g.standard_normal((P.N, ns)), 2)
    _, theta, _, _, _ = oracle.rayleigh_ritz(op, Yh)
    assert np.all(theta >= lam[:ns] - 1e-12)
    # exact invariant subspace: Ritz values are the eigenvalues, residuals ~ 0
    Yh, _, _ = oracle.cholesky_qr(V[:, :ns] @ g.standard_normal((ns, ns)), 2)
    Xn, theta, resid, _, _ = oracle.rayleigh_ritz(op, Yh)
    assert np.max(np.abs(theta - lam[:ns])) <= 1e-13 * 5
    assert np.max(resid) <= 1e-12
    # basis independence: RR(orth(X G)) = RR(orth(X))
    X = g.standard_normal((P.N, ns))
    G = g.standard_normal((ns, ns))
    t1 = oracle.rayleigh_ritz(op, oracle.cholesky_qr(X, 2)[0])[1]
    t2 = oracle.rayleigh_ritz(op, oracle.cholesky_qr(X @ G, 2)[0])[1]
    assert np.max(np.abs(t1 - t2)) <= 1e-11


def test_sign_normalize_rule():
    Q = np.array([[0.1, -0.5, 0.3], [-0.9, 0.5, -0.3], [0.2, 0.1, 0.0]])
    S = oracle.sign_normalize(Q)
    assert S[1, 0] > 0 and S[0, 1] > 0 and S[0, 2] > 0   # ties -> lowest index


# ---------------------------------------------------------------- P8
@pytest.mark.parametrize("w", ["tiny", "mixed"])
def test_P8_lanczos_upper_bound(w):
    if w == "tiny":
        P = synth.make_problem(synth.TINY)
    else:
        J = np.array([8, 16, 24, 8, 16, 8], dtype=np.int32)
        P = synth.make_blocks((3, 2, 1), 5, J)
    H = dense_of(P)
    lam = np.linalg.eigvalsh(H)
    b, theta, tau = oracle.lanczos_upper_bound(oracle.DenseOperator(H), synth.make_lanczos_start(P.N), 20)
    assert b >= lam[-1]
    assert b - lam[-1] <= 0.5 * (lam[-1] - lam[0])
    assert theta[0] >= lam[0] - 1e-12 and theta[-1] <= lam[-1] + 1e-12
    assert abs(np.sum(tau ** 2) - 1.0) <= 1e-12


# ---------------------------------------------------------------- P9
def test_P9_tiny_sweeps_converge_to_eigenvalues():
    w = synth.TINY
    P = synth.make_problem(w)
    H = dense_of(P)
    lam, _ = oracle.jacobi_eigh(H)
    assert np.max(np.abs(lam - np.linalg.eigvalsh(H))) < 1e-12
    op = oracle.DenseOperator(H)
    X0 = synth.make_start_block(P.J, w.ns)
    _, theta, resid, hist = core.run_sweeps(op, X0, synth.make_lanczos_start(P.N), w.m, w.sweeps)
    k = 3 * w.ns // 4
    s = max(abs(hist[0][0][2]), abs(hist[0][0][1]))
    assert np.max(np.abs(theta[:k] - lam[:k])) <= 1e-8 * s
    worst = [float(np.max(h[2][:k])) for h in hist]
    assert all(worst[i + 1] < worst[i] for i in range(len(worst) - 1)), worst


# ---------------------------------------------------------------- P10, P11, P12
def _mirror(P, K, s, i, j):
    Kp = core.slot_neighbour(K, s, P.grid)
    sm = 0 if s == 0 else (s + 1 if s % 2 == 1 else s - 1)
    return Kp, sm, j, i


def _small_grad_problem():
    grid, nb = (3, 3, 3), 8
    J = np.full(27, nb, dtype=np.int32)
    P = synth.make_blocks(grid, 7, J)
    H = dense_of(P)
    op = oracle.DenseOperator(H)
    ns, m, k = 24, 6, 16
    # a well-conditioned start: output of three cold sweeps
    X, theta, _, hist = core.run_sweeps(op, synth.make_start_block(J, ns), synth.make_lanczos_start(P.N), m, 3)
    b = hist[0][0][1]
    bounds = core.bounds_warm(theta, b)
    return P, op, X, m, k, bounds


def test_P10_gradient_matches_central_differences():
    P, op, X, m, k, bounds = _small_grad_problem()
    L, cache = oracle.loss_forward(op, X, m, bounds, k)
    Gd, Xbar = oracle.loss_backward(op, cache)
    Gb = oracle.restrict_to_pattern(Gd, P.grid, P.stencil, P.J)
    h = 1e-6
    ents = synth.fd_entries(P, 16)
    errs, mags = [], []
    for (K, s, i, j) in ents:
        K2, s2, i2, j2 = _mirror(P, K, s, i, j)
        vals = []
        for sgn in (+1, -1):
            blocks = [[B.copy() for B in row] for row in P.blocks]
            blocks[K][s][i, j] += sgn * h
            if (K2, s2, i2, j2) != (K, s, i, j):
                blocks[K2][s2][i2, j2] += sgn * h
            Hp = oracle.assemble_dense(P.grid, P.stencil, P.J, blocks)
            vals.append(oracle.loss_forward(oracle.DenseOperator(Hp), X, m, bounds, k)[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        an = Gb[K][s][i, j] + (Gb[K2][s2][i2, j2] if (K2, s2, i2, j2) != (K, s, i, j) else 0.0)
        errs.append(fd - an)
        mags.append(an)
    errs, mags = np.array(errs), np.array(mags)
    assert np.linalg.norm(errs) <= 1e-6 * max(1.0, np.linalg.norm(mags)), (errs, mags)
    # X gradient by finite differences along a random direction
    D = np.random.default_rng(2).standard_normal(X.shape)
    lp = oracle.loss_forward(op, X + h * D, m, bounds, k)[0]
    lm = oracle.loss_forward(op, X - h * D, m, bounds, k)[0]
    assert abs((lp - lm) / (2 * h) - np.sum(Xbar * D)) <= 1e-6 * max(1.0, abs(np.sum(Xbar * D)))


def test_P10_block_mode_gradient_matches_dense():
    P, op, X, m, k, bounds = _small_grad_problem()
    L, cache = oracle.loss_forward(op, X, m, bounds, k)
    Gd, Xbar = oracle.loss_backward(op, cache)
    bop = oracle.BlockOperator(P.grid, P.stencil, P.J, P.blocks)
    L2, cache2 = oracle.loss_forward(bop, X, m, bounds, k)
    Gb2, Xbar2 = oracle.loss_backward(bop, cache2)
    Gb = oracle.restrict_to_pattern(Gd, P.grid, P.stencil, P.J)
    assert abs(L - L2) <= 1e-12 * abs(L)
    num = sum(np.sum((Gb[K][s] - Gb2[K][s]) ** 2) for K in range(P.M) for s in range(P.stencil))
    den = sum(np.sum(Gb[K][s] ** 2) for K in range(P.M) for s in range(P.stencil))
    assert math.sqrt(num / den) <= 1e-11
    assert np.linalg.norm(Xbar - Xbar2) <= 1e-11 * np.linalg.norm(Xbar)


def test_P11_hellmann_feynman_at_invariant_subspace():
    P = synth.make_problem(synth.TINY)
    H = dense_of(P)
    lam, V = np.linalg.eigh(H)
    op = oracle.DenseOperator(H)
    ns, k, m = 24, 16, 5
    X = V[:, :ns]
    bounds = (lam[ns + 5], lam[-1] + 0.5, lam[0] - 0.1)
    L, cache = oracle.loss_forward(op, X, m, bounds, k)
    assert abs(L - np.sum(lam[:k])) <= 1e-12 * abs(L) * 10
    Gd, Xbar = oracle.loss_backward(op, cache)
    ref = V[:, :k] @ V[:, :k].T
    assert np.max(np.abs(Gd - ref)) <= 1e-10
    assert np.linalg.norm(Xbar) <= 1e-9


def test_P12_x_gradient_is_filter_of_ytilde_bar():
    P = synth.make_problem(synth.TINY)
    H = dense_of(P)
    op = oracle.DenseOperator(H)
    X = synth.make_start_block(P.J, 10)
    m, (a, b, a0) = 9, (0.3, 5.0, -1.0)
    _, Ys = oracle.chebyshev_filter(op, X, m, a, b, a0, return_all=True)
    Ybar = np.random.default_rng(4).standard_normal(X.shape)
    acc = oracle.adjoint._PatternAccumulator(op)
    Xbar = oracle.filter_backward(op, Ys, m, a, b, a0, Ybar, acc)
    ref = oracle.chebyshev_filter(op, Ybar, m, a, b, a0)     # p_m(H) symmetric
    assert np.linalg.norm(Xbar - ref) <= 1e-12 * np.linalg.norm(ref)


def test_P10_detects_planted_adjoint_mistakes(monkeypatch):
    """Planted slips in the adjoint must break agreement with a directional
    finite difference of the loss."""
    P, op, X, m, k, bounds = _small_grad_problem()
    D = np.random.default_rng(8).standard_normal(X.shape)
    h = 1e-6
    fd = (oracle.loss_forward(op, X + h * D, m, bounds, k)[0]
          - oracle.loss_forward(op, X - h * D, m, bounds, k)[0]) / (2 * h)

    def xdir():
        L, cache = oracle.loss_forward(op, X, m, bounds, k)
        return float(np.sum(oracle.loss_backward(op, cache)[1] * D))

    assert abs(xdir() - fd) <= 1e-6 * max(1.0, abs(fd))
    with monkeypatch.context() as mp:
        # (for this loss M is symmetric, so only dropping the term is visible)
        mp.setattr(oracle.adjoint, "_copyltu", lambda M: 0.0 * M)
        assert abs(xdir() - fd) > 1e-4 * max(1.0, abs(fd))
    # forward unchanged (cached); only the reverse sweep loses its beta term
    L, cache = oracle.loss_forward(op, X, m, bounds, k)
    with monkeypatch.context() as mp:
        orig = core.chebyshev_coefficients

        def no_beta(m_, a, b, a0):
            c, coefs = orig(m_, a, b, a0)
            return c, [(al, 0.0) for al, _ in coefs]
        mp.setattr(oracle.adjoint.core, "chebyshev_coefficients", no_beta)
        bad = float(np.sum(oracle.loss_backward(op, cache)[1] * D))
    assert abs(bad - fd) > 1e-4 * max(1.0, abs(fd))


# ------------------------------------------------ Cholesky-QR condition bound
def test_cholqr_condition_bound_is_an_upper_bound():
    """sqrt(kappa_1 kappa_inf) of the equilibrated factor is >= the 2-norm
    condition number of the column-equilibrated block (LAPACK SVD), equals 1
    for orthogonal columns of any scale, and tracks ill-conditioning."""
    g = np.random.default_rng(21)
    for N, n, spread in ((200, 30, 0.0), (300, 60, 3.0), (500, 40, 6.0)):
        Y = g.standard_normal((N, n)) * 10.0 ** g.uniform(-spread, spread, n)[None, :]
        U = np.linalg.cholesky(Y.T @ Y).T
        Ye = Y / np.linalg.norm(Y, axis=0)[None, :]
        s = np.linalg.svd(Ye, compute_uv=False)
        k2 = s[0] / s[-1]
        b = oracle.cholqr_condition_bound(U)
        assert b >= k2 * (1 - 1e-12)
        assert b <= n * k2
    Q, _ = np.linalg.qr(g.standard_normal((100, 20)))
    Ys = Q * 10.0 ** g.uniform(-5, 5, 20)[None, :]
    assert abs(oracle.cholqr_condition_bound(np.linalg.cholesky(Ys.T @ Ys).T) - 1.0) <= 1e-10
    # two nearly parallel columns: the bound grows like 1/angle
    Y = g.standard_normal((100, 5))
    Y[:, 4] = Y[:, 3] + 1e-6 * g.standard_normal(100)
    assert oracle.cholqr_condition_bound(np.linalg.cholesky(Y.T @ Y).T) > 1e5


def test_cholesky_qr_auto_passes():
    """passes = 0 keeps one pass for a well-conditioned block (the result is
    the one-pass result) and takes the second pass for an ill-conditioned one
    (orthonormal to rounding either way)."""
    g = np.random.default_rng(22)
    Y = g.standard_normal((3000, 20)) * 10.0 ** g.uniform(-4, 4, 20)[None, :]
    Yh0, _, Us0 = oracle.cholesky_qr(Y, 0)
    Yh1, _, _ = oracle.cholesky_qr(Y, 1)
    assert len(Us0) == 1 and np.array_equal(Yh0, Yh1)
    assert np.linalg.norm(Yh0.T @ Yh0 - np.eye(20), 2) <= 1e-13
    Z = g.standard_normal((300, 40))
    Z[:, 7] = Z[:, 3] + 1e-5 * g.standard_normal(300)
    Zh, _, Usz = oracle.cholesky_qr(Z, 0)
    assert len(Usz) == 2
    assert np.linalg.norm(Zh.T @ Zh - np.eye(40), 2) <= 1e-13
