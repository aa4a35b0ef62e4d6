"""Full-size GPU checks on the bulk (12x12x12 elements, 64 ALBs, N_s = 4,096,
m = 16) and sheet (48x40x1 elements, 5-block stencil, ALB counts drawn from
{64, 72, ..., 128}, N_s = 8,192, m = 20) workloads, in the launch configuration
the benchmark times (whole multivector, automatic Cholesky-QR pass count, 20
Lanczos steps).

The oracle cannot filter or diagonalise at these sizes, so the checks are:
* the filter is column-separable, so a 32-column slice across a column-tile
  boundary and sampled columns of the GPU result are compared with the
  block-mode oracle filter of the same columns of X;
* after a sweep, properties that hold at any size: orthonormality of X, the
  Ritz values equal the Rayleigh quotients x_i^T H x_i of the returned vectors
  (recomputed by the oracle's block operator on sampled columns), the reported
  residuals equal ||H x_i - theta_i x_i||, and the Ritz values ascend."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SAMPLE_SEED = 88


def sample_columns(ns, count=6):
    g = np.random.default_rng(SAMPLE_SEED)
    cols = set(g.choice(ns, size=count, replace=False).tolist()) | {0, ns - 1}
    return np.array(sorted(cols))


def filter_columns(ns, width=32):
    """A contiguous slice of `width` columns across a 128-column tile boundary
    of the step kernel (at a seeded tile), plus the sampled columns (first and
    last included).  The block-mode oracle needs about a second per column at
    these sizes, which bounds the slice."""
    t = int(np.random.default_rng(SAMPLE_SEED + 1).integers(1, ns // 128))
    c0 = 128 * t - width // 2
    return np.array(sorted(set(range(c0, c0 + width)) | set(sample_columns(ns).tolist())))


def relf(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module", params=["bulk", "sheet"])
def case(request, lib):
    w = {"bulk": synth.BULK, "sheet": synth.SHEET}[request.param]
    P = synth.make_problem(w)
    X0 = synth.make_start_block(P.J, w.ns)
    v0 = synth.make_lanczos_start(P.N)
    plan = lib.Plan(P.grid, P.stencil, P.J)
    dev = torch.device("cuda", 0)
    H = torch.from_numpy(P.packed()).to(dev)
    ws = torch.empty(max(plan.workspace_bytes(lib.OP_SWEEP, w.ns, dt, 2, w.lanczos_steps)
                         for dt in (lib.F64, lib.F32, lib.BF16, lib.BF16X3)), dtype=torch.uint8, device=dev)
    bop = oracle.BlockOperator(P.grid, P.stencil, P.J, P.blocks)
    print(f"\n[{w.name}] N={P.N} ns={w.ns} m={w.m}", flush=True)
    yield w, P, X0, v0, plan, H, ws, bop
    del H, ws
    torch.cuda.empty_cache()


def test_filter_sampled_columns_match_oracle(case, lib):
    w, P, X0, v0, plan, H, ws, bop = case
    a, b, a0 = 0.5, 7.0, -1.5
    Xd = torch.from_numpy(X0).cuda()
    Y = plan.filter(H, Xd, w.m, a, b, a0)
    cols = filter_columns(w.ns)
    Yc = Y[:, torch.from_numpy(cols).cuda()].cpu().numpy()
    ref = oracle.chebyshev_filter(bop, np.ascontiguousarray(X0[:, cols]), w.m, a, b, a0)
    err = relf(Yc, ref)
    colerr = np.max(np.linalg.norm(Yc - ref, axis=0) / np.linalg.norm(ref, axis=0))
    print(f"[{w.name}] FP64 filter, {len(cols)} columns: rel Frobenius error {err:.3e}, "
          f"worst column {colerr:.3e}")
    assert err <= 1e-12
    Y32 = plan.filter(H, Xd, w.m, a, b, a0, dtype=lib.F32)
    err32 = relf(Y32[:, torch.from_numpy(cols).cuda()].cpu().numpy(), ref)
    print(f"[{w.name}] FP32 filter, same columns: rel error {err32:.3e}")
    assert err32 <= 1e-4
    del Y, Y32, Xd


def rayleigh_checks(name, P, bop, X, ritz, resid, s):
    ns = X.shape[1]
    G = X.T @ X
    G.diagonal().sub_(1.0)
    orth = float(torch.linalg.eigvalsh(G).abs().max().item())
    print(f"[{name}] ||X^T X - I||_2 = {orth:.3e}")
    assert orth <= 1e-12
    del G
    th = ritz.cpu().numpy()
    assert np.all(np.isfinite(th)) and np.all(np.diff(th) >= 0)
    cols = sample_columns(ns)
    Xc = X[:, torch.from_numpy(cols).cuda()].cpu().numpy()
    HX = bop.apply(Xc)
    rq = np.einsum("ij,ij->j", Xc, HX) / np.einsum("ij,ij->j", Xc, Xc)
    rel = np.max(np.abs(rq - th[cols]) / np.maximum(np.abs(th[cols]), s))
    print(f"[{name}] sampled Rayleigh quotients vs Ritz values: max rel {rel:.3e}")
    assert rel <= 1e-10
    r_o = np.linalg.norm(HX - Xc * th[cols], axis=0)
    r_g = resid.cpu().numpy()[cols]
    dr = np.max(np.abs(r_o - r_g))
    print(f"[{name}] sampled residual norms: max abs difference {dr:.3e} (largest {r_o.max():.3e})")
    assert dr <= 1e-10 * s


def test_sweeps_full_size_properties(case, lib):
    """Four FP64 sweeps (cold bounds, then warm) with the automatic
    Cholesky-QR pass count, as the benchmark runs them; on the bulk workload
    the fourth takes a single pass, so both forms end in the checks."""
    w, P, X0, v0, plan, H, ws, bop = case
    X = torch.from_numpy(X0).cuda()
    v0d = torch.from_numpy(v0).cuda()
    ritz = None
    taken = []
    for i in range(4):
        ritz, resid, bnd, st = plan.sweep(H, X, w.m, passes=0, lanczos_steps=w.lanczos_steps, v0=v0d,
                                          ritz=ritz, warm=i > 0, ws=ws, stats=True)
        taken.append((int(st["cholqr_passes"]), round(st["cholqr_cond_bound"], 2)))
    print(f"[{w.name}] (passes, condition bound) per sweep: {taken}")
    bh = bnd.cpu().numpy()
    s = float(max(abs(bh[1]), abs(bh[2])))
    assert bh[2] < bh[0] < bh[1]
    rayleigh_checks(w.name, P, bop, X, ritz, resid, s)
    del X


def test_mixed_sweeps_reach_the_fp64_ritz_error(case, lib):
    """Low-precision-filter sweeps then FP64 sweeps from the same start as four
    FP64 sweeps; "the same final Ritz error" is read as a worst wanted (lowest
    3/4) residual within 5 % of the FP64 run's.
    * FP32 and split BF16 (BF16X3): two low + two FP64 sweeps reach it, and the
      wanted Ritz values agree with the FP64 run's to 1e-8.
    * BF16 (8-bit mantissas): two low + two FP64 sweeps, then FP64 sweeps until
      the residual reaches the FP64 run's (at most three more; measured: none on
      the bulk workload (1.04x), one on the sheet, whose slowest wanted states
      need more FP64 cycles to wash out the BF16 rounding)."""
    w, P, X0, v0, plan, H, ws, bop = case
    v0d = torch.from_numpy(v0).cuda()
    k = 3 * w.ns // 4

    def run(dts, target=None, extra=0):
        X = torch.from_numpy(X0).cuda()
        ritz = None
        n = 0
        for i, dt in enumerate(dts + [lib.F64] * extra):
            ritz, resid, bnd, _ = plan.sweep(H, X, w.m, dtype=dt, passes=0, lanczos_steps=w.lanczos_steps,
                                             v0=v0d, ritz=ritz, warm=i > 0, ws=ws)
            n += 1
            if i >= len(dts) - 1 and target is not None and float(resid[:k].max().item()) <= target:
                break
        return X, ritz, resid, bnd.cpu().numpy(), n

    X, t64, r64, b64, _ = run([lib.F64] * 4)
    t64, r64 = t64.cpu().numpy(), float(r64[:k].max().item())
    del X
    s = float(max(abs(b64[1]), abs(b64[2])))
    for name, low, extra, ttol in (("FP32", lib.F32, 0, 1e-8), ("BF16X3", lib.BF16X3, 0, 1e-8),
                                   ("BF16", lib.BF16, 3, 1e-6)):
        X, tmx, rmx, bmx, n = run([low] * 2 + [lib.F64] * 2, target=1.05 * r64, extra=extra)
        rayleigh_checks(f"{w.name} {name} mixed", P, bop, X, tmx, rmx,
                        float(max(abs(bmx[1]), abs(bmx[2]))))
        tmx, rmx = tmx.cpu().numpy(), float(rmx[:k].max().item())
        dth = np.max(np.abs(tmx[:k] - t64[:k]) / np.maximum(np.abs(t64[:k]), s))
        print(f"[{w.name}] max wanted residual: FP64 {r64:.3e}, {name} mixed {rmx:.3e} after {n} sweeps "
              f"({n - 4} extra FP64); Ritz rel diff {dth:.3e}")
        assert rmx <= 1.05 * r64
        assert dth <= ttol
        del X
