"""GPU adjoint of one filter + Cholesky-QR + Rayleigh-Ritz pass (loss = sum of
the k lowest Ritz values, bounds held constant) against the oracle's adjoint,
against central finite differences of the GPU forward, and through
torch.autograd."""
import numpy as np
import pytest

import oracle
import synth
from oracle import core

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def blocks_rel(Gb, Go):
    num = sum(np.sum((a - b) ** 2) for ra, rb in zip(Gb, Go) for a, b in zip(ra, rb))
    den = sum(np.sum(b ** 2) for rb in Go for b in rb)
    return float(np.sqrt(num / den))


def mirror(P, K, s, i, j):
    Kp = core.slot_neighbour(K, s, P.grid)
    sm = 0 if s == 0 else (s + 1 if s % 2 == 1 else s - 1)
    return Kp, sm, j, i


def oracle_case(grid, nb, ns, m, k):
    J = np.full(grid[0] * grid[1] * grid[2], nb, dtype=np.int32)
    P = synth.make_blocks(grid, 7, J)
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    op = oracle.DenseOperator(H)
    X, theta, _, hist = core.run_sweeps(op, synth.make_start_block(J, ns), synth.make_lanczos_start(P.N), m, 3)
    bounds = core.bounds_warm(theta, hist[0][0][1])
    return P, op, X, bounds


@pytest.mark.parametrize("grid,nb,ns,m,k,passes,cs", [
    ((3, 3, 3), 8, 24, 6, 16, 2, 4),
    ((4, 4, 4), 16, 64, 12, 48, 2, 4),
    ((3, 3, 3), 8, 24, 6, 16, 1, 6),
    ((2, 3, 2), 12, 30, 5, 20, 2, 2),
    ((2, 2, 1), 200, 40, 5, 30, 2, 2),     # blocks above 128 x 128 (gradient tiles)
])
def test_loss_backward_matches_oracle(lib, grid, nb, ns, m, k, passes, cs):
    P, op, X, bounds = oracle_case(grid, nb, ns, m, k)
    L_o, cache = oracle.loss_forward(op, X, m, bounds, k, passes)
    Gd, Xbar_o = oracle.loss_backward(op, cache)
    Gb_o = oracle.restrict_to_pattern(Gd, P.grid, P.stencil, P.J)
    plan = lib.Plan(P.grid, P.stencil, P.J)
    L, Hbar, Xbar = plan.loss_backward(dev(P.packed()), dev(X), m, *bounds, k, passes, cs)
    assert abs(L - L_o) <= 1e-12 * abs(L_o)
    Gb = synth.BlockProblem.from_packed(P.grid, P.stencil, P.J, host(Hbar)).blocks
    assert blocks_rel(Gb, Gb_o) <= 1e-9
    assert np.linalg.norm(host(Xbar) - Xbar_o) <= 1e-9 * np.linalg.norm(Xbar_o)


def test_checkpoint_stride_does_not_change_the_gradient(lib):
    P, op, X, bounds = oracle_case((3, 3, 3), 8, 24, 7, 16)
    plan = lib.Plan(P.grid, P.stencil, P.J)
    Hd, Xd = dev(P.packed()), dev(X)
    ref = None
    for cs in (1, 2, 3, 7):
        L, Hbar, Xbar = plan.loss_backward(Hd, Xd, 7, *bounds, 16, 2, cs)
        cur = (L, host(Hbar), host(Xbar))
        if ref is None:
            ref = cur
        else:
            assert cur[0] == ref[0]
            assert np.max(np.abs(cur[1] - ref[1])) <= 1e-14 * np.max(np.abs(ref[1]))
            assert np.max(np.abs(cur[2] - ref[2])) <= 1e-14 * np.max(np.abs(ref[2]))


@pytest.mark.parametrize("m,cs", [(9, 4), (9, 9), (1, 1), (4, 3)])
def test_filter_backward_matches_oracle(lib, m, cs):
    P = synth.make_problem(synth.TINY)
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    op = oracle.DenseOperator(H)
    X = synth.make_start_block(P.J, 10)
    a, b, a0 = 0.3, 5.0, -1.0
    _, Ys = oracle.chebyshev_filter(op, X, m, a, b, a0, return_all=True)
    Ybar = np.random.default_rng(4).standard_normal(X.shape)
    acc = oracle.adjoint._PatternAccumulator(op)
    Xbar_o = oracle.filter_backward(op, Ys, m, a, b, a0, Ybar, acc)
    Gb_o = oracle.restrict_to_pattern(acc.result(), P.grid, P.stencil, P.J)
    plan = lib.Plan(P.grid, P.stencil, P.J)
    Hbar0 = np.random.default_rng(5).standard_normal(P.packed_size())   # accumulated onto
    Hbar, Xbar = plan.filter_backward(dev(P.packed()), dev(X), dev(Ybar), m, a, b, a0, cs, Hbar=dev(Hbar0))
    Gb = synth.BlockProblem.from_packed(P.grid, P.stencil, P.J, host(Hbar) - Hbar0).blocks
    assert blocks_rel(Gb, Gb_o) <= 1e-11
    assert np.linalg.norm(host(Xbar) - Xbar_o) <= 1e-11 * np.linalg.norm(Xbar_o)


def test_diff_workload_gradient_against_finite_differences(lib):
    """Differentiation workload: 6x6x6 elements, 48 ALBs, N_s = 512, m = 12,
    loss over the lowest 384 Ritz values, checkpoints every 4 steps; X is the
    output of 3 cold FP64 cycles; central differences with h = 1e-6 on 32
    random stored entries (each perturbed together with its mirror entry)."""
    w = synth.DIFF
    P = synth.make_problem(w)
    plan = lib.Plan(P.grid, P.stencil, P.J)
    Hh = P.packed()
    Hd = dev(Hh)
    X = dev(synth.make_start_block(P.J, w.ns))
    v0 = dev(synth.make_lanczos_start(P.N))
    ritz = None
    for i in range(3):
        ritz, resid, bused, _ = plan.sweep(Hd, X, w.m, v0=v0, ritz=ritz, warm=i > 0)
    bh = host(bused)
    r = host(ritz)
    a, b = float(r[-1]), float(bh[1])
    a0 = float(r[0])
    k = 384
    assert r[k] - r[k - 1] > 1e-8 * b
    L, Hbar, Xbar = plan.loss_backward(Hd, X, w.m, a, b, a0, k, 2, 4)
    G = host(Hbar)
    # offsets of the stored blocks in the packed layout
    offs, pos = {}, 0
    for K in range(P.M):
        for s in range(P.stencil):
            offs[(K, s)] = pos
            pos += P.blocks[K][s].size
    h = 1e-6
    fd, an = [], []
    for (K, s, i, j) in synth.fd_entries(P, 32):
        K2, s2, i2, j2 = mirror(P, K, s, i, j)
        idx1 = offs[(K, s)] + i * P.blocks[K][s].shape[1] + j
        idx2 = offs[(K2, s2)] + i2 * P.blocks[K2][s2].shape[1] + j2
        vals = []
        for sgn in (1, -1):
            Hp = Hh.copy()
            Hp[idx1] += sgn * h
            if idx2 != idx1:
                Hp[idx2] += sgn * h
            vals.append(plan.loss_backward(dev(Hp), X, w.m, a, b, a0, k, 2, 4)[0])
        fd.append((vals[0] - vals[1]) / (2 * h))
        an.append(G[idx1] + (G[idx2] if idx2 != idx1 else 0.0))
    fd, an = np.array(fd), np.array(an)
    rel = np.linalg.norm(fd - an) / np.linalg.norm(an)
    print(f"diff workload: FD vs adjoint relative 2-norm error over 32 entries: {rel:.3e}")
    assert rel <= 1e-4
    # directional derivative in X
    D = torch.randn(X.shape, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    lp = plan.loss_backward(Hd, X + h * D, w.m, a, b, a0, k, 2, 4)[0]
    lm = plan.loss_backward(Hd, X - h * D, w.m, a, b, a0, k, 2, 4)[0]
    dd = float(torch.sum(Xbar * D).item())
    assert abs((lp - lm) / (2 * h) - dd) <= 1e-4 * max(abs(dd), 1e-8)


def test_diff_workload_gradient_matches_oracle(lib):
    """Differentiation workload against the oracle's block-mode adjoint: X is
    the output of 3 cold oracle cycles (the oracle's own Lanczos bound and
    policy), bounds from its last Ritz values; loss over the lowest 384 Ritz
    values, two Cholesky-QR passes, checkpoints every 4 steps."""
    w = synth.DIFF
    P = synth.make_problem(w)
    op = oracle.BlockOperator(P.grid, P.stencil, P.J, P.blocks)
    X, theta, _, hist = core.run_sweeps(op, synth.make_start_block(P.J, w.ns), synth.make_lanczos_start(P.N),
                                        w.m, 3)
    bounds = core.bounds_warm(theta, hist[0][0][1])
    k = 384
    L_o, cache = oracle.loss_forward(op, X, w.m, bounds, k, 2)
    Gb_o, Xbar_o = oracle.loss_backward(op, cache)
    plan = lib.Plan(P.grid, P.stencil, P.J)
    L, Hbar, Xbar = plan.loss_backward(dev(P.packed()), dev(X), w.m, *bounds, k, 2, 4)
    Gb = synth.BlockProblem.from_packed(P.grid, P.stencil, P.J, host(Hbar)).blocks
    eH, eX = blocks_rel(Gb, Gb_o), float(np.linalg.norm(host(Xbar) - Xbar_o) / np.linalg.norm(Xbar_o))
    print(f"diff workload vs oracle adjoint: loss {abs(L - L_o) / abs(L_o):.2e}, Hbar {eH:.2e}, Xbar {eX:.2e}")
    assert abs(L - L_o) <= 1e-12 * abs(L_o)
    assert eH <= 1e-10 and eX <= 1e-10


@pytest.mark.parametrize("n,ns,inplace", [(300, 20, False), (2000, 130, True), (10368, 257, False)])
def test_orthonormalize_backward_matches_oracle(lib, n, ns, inplace):
    """chefsi_orthonormalize_backward on the oracle's own QR factors (two
    passes, combined factor) against the oracle's QR adjoint."""
    g = np.random.default_rng(n + ns)
    Y = g.standard_normal((n, ns)) * 10.0 ** g.uniform(-2, 2, ns)[None, :]
    Yh, U, _ = oracle.cholesky_qr(Y, 2)
    Gbar = g.standard_normal((n, ns))
    ref = oracle.cholesky_qr_backward([Yh], [U], Gbar)
    Gd = dev(Gbar)
    out = lib.orthonormalize_backward(dev(Yh), dev(U), Gd, out=Gd if inplace else None)
    if inplace:
        assert out.data_ptr() == Gd.data_ptr()
    assert np.linalg.norm(host(out) - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("name,ns", [("tiny", 48), ("mixed", 100)])
def test_rayleigh_ritz_backward_matches_oracle(lib, name, ns):
    """chefsi_rayleigh_ritz_backward on the oracle's orthonormal block and
    eigenvectors, random Ritz-value cotangent, against the oracle's rule; and
    accumulation onto an existing gradient."""
    if name == "tiny":
        P = synth.make_problem(synth.TINY)
    else:
        J = np.array([8, 16, 24, 40, 64, 128, 72, 88, 104, 120, 56, 32], dtype=np.int32)
        P = synth.make_blocks((4, 3, 1), 5, J)
    H = oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks)
    op = oracle.DenseOperator(H)
    g = np.random.default_rng(ns)
    Yh = oracle.cholesky_qr(g.standard_normal((P.N, ns)), 2)[0]
    _, theta, _, Q, _ = oracle.rayleigh_ritz(op, Yh)
    tb = g.standard_normal(ns)
    acc = oracle.adjoint._PatternAccumulator(op)
    Yb_o = oracle.rayleigh_ritz_backward(op, Yh, Q, tb, acc)
    Gb_o = oracle.restrict_to_pattern(acc.result(), P.grid, P.stencil, P.J)
    plan = lib.Plan(P.grid, P.stencil, P.J)
    Hd = dev(P.packed())
    Yb, Hbar = plan.rayleigh_ritz_backward(Hd, dev(Yh), dev(Q), dev(tb))
    assert np.linalg.norm(host(Yb) - Yb_o) <= 1e-12 * np.linalg.norm(Yb_o)
    Gb = synth.BlockProblem.from_packed(P.grid, P.stencil, P.J, host(Hbar)).blocks
    assert blocks_rel(Gb, Gb_o) <= 1e-12
    H0 = g.standard_normal(P.packed_size())
    _, Hacc = plan.rayleigh_ritz_backward(Hd, dev(Yh), dev(Q), dev(tb), Hbar=dev(H0), accumulate=True)
    Gb2 = synth.BlockProblem.from_packed(P.grid, P.stencil, P.J, host(Hacc) - H0).blocks
    assert blocks_rel(Gb2, Gb_o) <= 1e-12


def test_loss_forward_alone_matches_the_adjoint_forward(lib):
    """chefsi_loss runs only the forward and returns exactly the loss that
    chefsi_loss_backward reports (same arithmetic)."""
    P, op, X, bounds = oracle_case((3, 3, 3), 8, 24, 6, 16)
    plan = lib.Plan(P.grid, P.stencil, P.J)
    Hd, Xd = dev(P.packed()), dev(X)
    for passes in (1, 2):
        L0 = plan.loss(Hd, Xd, 6, *bounds, 16, passes)
        L1 = plan.loss_backward(Hd, Xd, 6, *bounds, 16, passes, 2)[0]
        assert L0 == L1
        L_o = oracle.loss_forward(op, X, 6, bounds, 16, passes)[0]
        assert abs(L0 - L_o) <= 1e-12 * abs(L_o)


def test_autograd_functions(lib):
    P, op, X, bounds = oracle_case((3, 3, 3), 8, 24, 6, 16)
    plan = lib.Plan(P.grid, P.stencil, P.J)
    Hd = dev(P.packed()).requires_grad_(True)
    Xd = dev(X).requires_grad_(True)
    L = lib.ChefsiLoss.apply(Hd, Xd, plan, 6, bounds, 16, 2, 4)
    gH, gX = torch.autograd.grad(L, (Hd, Xd))
    L1, Hbar, Xbar = plan.loss_backward(Hd.detach(), Xd.detach(), 6, *bounds, 16, 2, 4)
    assert float(L.detach()) == L1
    assert torch.equal(gH, Hbar) and torch.equal(gX, Xbar)
    # without gradients the forward is chefsi_loss alone
    with torch.no_grad():
        L2 = lib.ChefsiLoss.apply(Hd, Xd, plan, 6, bounds, 16, 2, 4)
    assert float(L2) == plan.loss(Hd.detach(), Xd.detach(), 6, *bounds, 16, 2)
    a, b, a0 = 0.3, 5.0, -1.0
    Y = lib.ChebFilter.apply(Hd, Xd, plan, 5, a, b, a0, 2)
    Ybar = torch.ones_like(Y)
    gH2, gX2 = torch.autograd.grad(Y, (Hd, Xd), Ybar)
    Hb, Xb = plan.filter_backward(Hd.detach(), Xd.detach(), Ybar, 5, a, b, a0, 2)
    assert torch.equal(gH2, Hb) and torch.equal(gX2, Xb)
