"""GPU parity of the steps around the cycle, through the C ABI, against the
oracle: Fermi level and occupations, diagonal density-matrix blocks (eq.
densitymatrix), and the re-alignment to a new ALB basis (eq.
basis_rotation_3).  Small cases cover every row-block class (ALB counts 1 to
128, ragged tiles), odd and strided leading dimensions and ragged column
counts; the bulk and sheet cases run at full size in the benchmark's launch
configuration and are compared element by element on sampled elements."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KT = synth.KT_300K


def relf(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def spectrum(ns, seed):
    g = np.random.default_rng(seed)
    return np.sort(g.uniform(-0.8, -0.2, size=ns))


# ---------------------------------------------------------------- occupations
@pytest.mark.parametrize("ns", [1, 2, 48, 130, 1000, 4096, 8192])
def test_occupations_match_oracle(lib, ns):
    th = spectrum(ns, ns)
    n_occ = 0.5 if ns == 1 else synth.occupied_count(ns)
    mu_o, f_o = oracle.occupations(th, n_occ, KT)
    f, mu = lib.occupations(torch.from_numpy(th).cuda(), n_occ, KT)
    mu_g, f_g = float(mu.item()), f.cpu().numpy()
    print(f"ns={ns}: mu gpu-oracle {mu_g - mu_o:.2e}, max |df| {np.max(np.abs(f_g - f_o)):.2e}")
    assert abs(mu_g - mu_o) <= 1e-12
    assert np.max(np.abs(f_g - f_o)) <= 1e-12
    assert abs(f_g.sum() - n_occ) <= 1e-9 * max(1.0, n_occ)


def test_occupations_in_place_degenerate_and_nonfinite(lib):
    th = torch.full((10,), 0.123, dtype=torch.float64, device="cuda")
    f, mu = lib.occupations(th, 7.5, KT, out=th)
    assert f.data_ptr() == th.data_ptr()
    assert abs(mu.item() - (0.123 + KT * np.log(7.5 / 2.5))) <= 1e-14
    assert np.max(np.abs(th.cpu().numpy() - 0.75)) <= 1e-14
    bad = torch.from_numpy(spectrum(64, 3)).cuda()
    bad[17] = float("nan")
    f, mu = lib.occupations(bad, 10.0, KT)
    assert np.isnan(mu.item()) and torch.isnan(f).all().item()
    with pytest.raises(lib.ChefsiError):
        lib.occupations(bad, 64.0, KT)


# ---------------------------------------------------- density-matrix blocks
PLANS = {
    "uniform64": ((3, 2, 2), 7, np.full(12, 64)),
    "ragged": ((4, 3, 1), 5, np.array([1, 7, 16, 17, 33, 48, 64, 65, 100, 127, 128, 5])),
    "small": ((2, 1, 1), 7, np.array([3, 9])),
}


def make_plan(lib, name):
    grid, stencil, J = PLANS[name]
    return lib.Plan(grid, stencil, J.astype(np.int32)), J.astype(np.int64)


def random_block(N, ns, seed, ld=None):
    g = np.random.default_rng(seed)
    X = g.standard_normal((N, ns))
    if ld is None or ld == ns:
        return X, torch.from_numpy(X).cuda()
    buf = torch.zeros((N, ld), dtype=torch.float64, device="cuda")
    buf[:, :ns] = torch.from_numpy(X).cuda()
    return X, buf[:, :ns]


@pytest.mark.parametrize("name", list(PLANS))
@pytest.mark.parametrize("ns,ld", [(1, None), (31, None), (48, 51), (130, None), (257, 300), (1000, None)])
def test_density_blocks_match_oracle(lib, name, ns, ld):
    plan, J = make_plan(lib, name)
    X, Xd = random_block(plan.N, ns, 100 + ns, ld)
    f = np.random.default_rng(7).uniform(0, 1, ns)
    P = plan.density_blocks(Xd, torch.from_numpy(f).cuda())
    blocks = plan.split_blocks(P)
    ref = oracle.density_diag_blocks(J, X, f)
    err = max(relf(b.cpu().numpy(), r) for b, r in zip(blocks, ref))
    print(f"{name} ns={ns} ld={ld}: worst block rel error {err:.2e}")
    assert err <= 1e-13
    for b in blocks:
        assert torch.equal(b, b.T)


def test_density_blocks_trace_identity_after_sweeps(lib):
    """After CheFSI cycles (orthonormal Ritz vectors) with the GPU's own
    occupations, sum_K tr P_KK = n_occ and every block has eigenvalues in
    [0, 1]."""
    w = synth.TINY
    P_ = synth.make_problem(w)
    plan = lib.Plan(P_.grid, P_.stencil, P_.J)
    H = torch.from_numpy(P_.packed()).cuda()
    X = torch.from_numpy(synth.make_start_block(P_.J, w.ns)).cuda()
    v0 = torch.from_numpy(synth.make_lanczos_start(P_.N)).cuda()
    ritz = None
    for i in range(3):
        ritz, resid, _, _ = plan.sweep(H, X, w.m, v0=v0, ritz=ritz, warm=i > 0)
    n_occ = synth.occupied_count(w.ns)
    f, mu = lib.occupations(ritz, n_occ, KT)
    Pd = plan.density_blocks(X, f)
    tr = sum(float(torch.trace(b)) for b in plan.split_blocks(Pd))
    assert abs(tr - n_occ) <= 1e-10
    for b in plan.split_blocks(Pd):
        ev = np.linalg.eigvalsh(b.cpu().numpy())
        assert ev.min() >= -1e-13 and ev.max() <= 1 + 1e-13
    ref = oracle.density_diag_blocks(P_.J, X.cpu().numpy(), oracle.fermi_dirac(ritz.cpu().numpy(), float(mu), KT))
    assert max(relf(b.cpu().numpy(), r) for b, r in zip(plan.split_blocks(Pd), ref)) <= 1e-13


def test_density_blocks_no_columns_gives_zero(lib):
    plan, _ = make_plan(lib, "small")
    X = torch.empty((plan.N, 0), dtype=torch.float64, device="cuda")
    P = torch.full((plan.block_elems,), 5.0, dtype=torch.float64, device="cuda")
    plan.density_blocks(X, torch.empty(1, dtype=torch.float64, device="cuda"), out=P)
    assert torch.count_nonzero(P).item() == 0


# ------------------------------------------------------------- re-alignment
@pytest.mark.parametrize("name", list(PLANS))
@pytest.mark.parametrize("ns,ld,nr", [(1, None, 128), (63, None, 130), (64, 70, 200), (65, None, 512),
                                      (200, 201, 129)])
def test_realign_matches_oracle(lib, name, ns, ld, nr):
    plan, J = make_plan(lib, name)
    V = synth.make_alb_samples(J, nr)
    Vn = synth.make_next_alb_samples(J, V, nr, delta=0.2)
    X, Xd = random_block(plan.N, ns, 300 + ns, ld)
    out = plan.realign(Xd, torch.from_numpy(Vn).cuda(), torch.from_numpy(V).cuda(), nr)
    assert out.data_ptr() == Xd.data_ptr()
    ref = oracle.realign(J, nr, Vn, V, X)
    err = relf(Xd.cpu().numpy(), ref)
    print(f"{name} ns={ns} ld={ld} nr={nr}: rel Frobenius error {err:.2e}")
    assert err <= 1e-13


def test_realign_unchanged_basis_is_identity(lib):
    plan, J = make_plan(lib, "ragged")
    nr = 160
    V = torch.from_numpy(synth.make_alb_samples(J, nr)).cuda()
    X, Xd = random_block(plan.N, 77, 9)
    plan.realign(Xd, V, V, nr)
    assert np.max(np.abs(Xd.cpu().numpy() - X)) <= 1e-13


# ---------------------------------------------------------------- full size
def sample_elements(M, count=8, seed=5):
    g = np.random.default_rng(seed)
    return np.array(sorted(set(g.choice(M, size=count, replace=False).tolist()) | {0, M - 1}))


def sub_rows(J, Ks):
    off = np.concatenate([[0], np.cumsum(J)])
    return np.concatenate([np.arange(off[K], off[K + 1]) for K in Ks])


@pytest.mark.parametrize("wname", ["bulk", "sheet"])
def test_full_size_density_and_realign_sampled_elements(lib, wname):
    """Bulk (12^3 elements, 64 ALBs, N_s = 4,096) and sheet (48 x 40
    elements, 64-128 ALBs, N_s = 8,192) workloads with n_r = 512: GPU density
    blocks and re-aligned rows of sampled elements against the oracle's
    element-local definitions."""
    w = {"bulk": synth.BULK, "sheet": synth.SHEET}[wname]
    J = synth.draw_alb_counts(w).astype(np.int64)
    plan = lib.Plan(w.grid, w.stencil, J.astype(np.int32))
    X0 = synth.make_start_block(J, w.ns)
    Xd = torch.from_numpy(X0).cuda()
    f = oracle.fermi_dirac(spectrum(w.ns, 1), -0.5, KT)
    P = plan.density_blocks(Xd, torch.from_numpy(f).cuda())
    Ks = sample_elements(plan.J.size)
    rows = sub_rows(J, Ks)
    ref = oracle.density_diag_blocks(J[Ks], X0[rows], f)
    blocks = plan.split_blocks(P)
    err = max(relf(blocks[K].cpu().numpy(), r) for K, r in zip(Ks, ref))
    print(f"{wname} density blocks, {len(Ks)} sampled elements: worst rel error {err:.2e}")
    assert err <= 1e-13
    del P
    nr = synth.NR_PER_ELEMENT
    V = synth.make_alb_samples(J, nr)
    Vn = synth.make_next_alb_samples(J, V, nr)
    plan.realign(Xd, torch.from_numpy(Vn).cuda(), torch.from_numpy(V).cuda(), nr)
    vrows = np.concatenate([np.arange(nr * r0, nr * (r0 + n)) for r0, n in
                            zip(np.concatenate([[0], np.cumsum(J)])[Ks], J[Ks])])
    ref = oracle.realign(J[Ks], nr, Vn[vrows], V[vrows], X0[rows])
    got = Xd[torch.from_numpy(rows).cuda()].cpu().numpy()
    err = relf(got, ref)
    print(f"{wname} realign, {len(Ks)} sampled elements: rel Frobenius error {err:.2e}")
    assert err <= 1e-13
    del Xd
    torch.cuda.empty_cache()


def test_post_cycle_kernels_report_unsupported_above_128_albs(lib):
    """Density-matrix blocks and re-alignment are built for ALB counts up to
    128; larger plans are refused on the host before any launch."""
    J = np.array([200, 64, 32, 129], dtype=np.int32)
    P = synth.make_blocks((2, 2, 1), 5, J)
    plan = lib.Plan(P.grid, P.stencil, P.J)
    X = torch.zeros((P.N, 8), dtype=torch.float64, device="cuda")
    f = torch.ones(8, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.ChefsiError) as e:
        plan.density_blocks(X, f)
    assert e.value.code == lib.ERR_UNSUPPORTED
    V = torch.zeros(P.N * 256, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.ChefsiError) as e:
        plan.realign(X, V, V, 256)
    assert e.value.code == lib.ERR_UNSUPPORTED
