"""A CheFSI run resumed from a saved state reproduces the uninterrupted run
bit for bit (every reduction in the library has a fixed order): three cycles
straight against one cycle, save, load in fresh tensors, two more cycles."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def test_resumed_run_is_bit_identical(lib, tmp_path):
    from paper_1606_03416_amd.state import SweepState, run_cycles
    w = synth.TINY
    P = synth.make_problem(w)
    plan = lib.Plan(P.grid, P.stencil, P.J)
    Hd = torch.from_numpy(P.packed()).cuda()
    X0 = synth.make_start_block(P.J, w.ns)
    v0 = torch.from_numpy(synth.make_lanczos_start(P.N)).cuda()

    a = SweepState(torch.from_numpy(X0).cuda(), v0.clone())
    ra = run_cycles(plan, Hd, a, 3, w.m)

    b = SweepState(torch.from_numpy(X0).cuda(), v0.clone())
    run_cycles(plan, Hd, b, 1, w.m)
    path = str(tmp_path / "state.npz")
    b.save(path, plan)
    del b
    c = SweepState.load(path, plan)
    assert c.cycle == 1 and c.X.is_cuda
    rc = run_cycles(plan, Hd, c, 2, w.m)
    torch.cuda.synchronize()
    assert c.cycle == 3
    assert torch.equal(a.X, c.X)
    assert torch.equal(a.ritz, c.ritz)
    assert torch.equal(a.bounds, c.bounds)
    assert torch.equal(ra, rc)
    # the resumed run did converge somewhere sensible (not a trivially equal failure)
    assert np.all(np.isfinite(rc.cpu().numpy()))
    # the same ALB counts on another element grid: refused
    other = lib.Plan((2, 4, 1), 5, P.J)
    with pytest.raises(ValueError, match="another plan"):
        SweepState.load(path, other)
