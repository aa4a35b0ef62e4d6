"""The allocation-free filter entry point (chefsi_filter_noalloc) against
chefsi_filter on the same inputs: two calls in a row on one GPU, the second
smaller (the shared scratch keeps the first call's contents), in FP64, FP32
and BF16, and a request larger than the static scratch rejected on the host."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("dtype", [0, 1, 2])
def test_noalloc_filter_matches_the_workspace_filter(lib, dtype):
    w = synth.DIFF
    P = synth.make_problem(w)
    plan = lib.Plan(P.grid, P.stencil, P.J)
    Hd = dev(P.packed())
    a, b, a0 = 0.4, 5.6, -1.3
    X = synth.make_start_block(P.J, w.ns)
    cases = [(dev(X), w.m), (dev(X[:, :130]), 7)]   # second call smaller: fewer columns, lower degree
    for Xd, m in cases:
        ref = plan.filter(Hd, Xd, m, a, b, a0, dtype)
        out = torch.full_like(ref, float("nan"))
        got = plan.filter_noalloc(Hd, Xd, m, a, b, a0, dtype, out=out)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        rel = float(torch.linalg.norm(got - ref) / torch.linalg.norm(ref))
        assert rel <= 1e-12, (dtype, Xd.shape, m, rel)
    # a smaller plan on the same GPU after the larger calls
    T = synth.make_problem(synth.TINY)
    tplan = lib.Plan(T.grid, T.stencil, T.J)
    Td = dev(T.packed())
    Xt = dev(synth.make_start_block(T.J, 48))
    ref = tplan.filter(Td, Xt, 10, a, b, a0, dtype)
    got = tplan.filter_noalloc(Td, Xt, 10, a, b, a0, dtype)
    torch.cuda.synchronize()
    assert float(torch.linalg.norm(got - ref) / torch.linalg.norm(ref)) <= 1e-12


def test_noalloc_filter_rejects_requests_beyond_its_scratch(lib):
    w = synth.DIFF
    P = synth.make_problem(w)
    plan = lib.Plan(P.grid, P.stencil, P.J)
    Hd = dev(P.packed())
    ns = 4096   # N * ns * 8 = 340 MB > 256 MiB
    X = torch.zeros((P.N, ns), dtype=torch.float64, device="cuda")
    Y = torch.zeros_like(X)
    with pytest.raises(lib.ChefsiError) as e:
        plan.filter_noalloc(Hd, X, 4, 0.4, 5.6, -1.3, out=Y)
    assert e.value.code == lib.ERR_WORKSPACE
    assert "256" in str(e.value) or "268435456" in str(e.value)
