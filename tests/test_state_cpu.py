"""Saving and loading a CheFSI run's state: the arrays come back exactly, the
file holds no pickled objects, and a state saved for one discretisation is
refused by another.  Host tensors only; no library call."""
import json

import numpy as np
import pytest
import torch

from paper_1606_03416_amd.state import FORMAT, SweepState, plan_fingerprint


class FakePlan:
    def __init__(self, grid=(2, 2, 1), stencil=5, J=(8, 8, 12, 8)):
        self.grid, self.stencil = grid, stencil
        self.J = np.asarray(J, dtype=np.int32)
        self.N = int(self.J.sum())
        self.device = torch.device("cpu")


def state(plan, ns=6, cycle=2, seed=3):
    g = torch.Generator().manual_seed(seed)
    X = torch.randn(plan.N, ns, dtype=torch.float64, generator=g)
    v0 = torch.randn(plan.N, dtype=torch.float64, generator=g)
    ritz = torch.sort(torch.randn(ns, dtype=torch.float64, generator=g)).values if cycle else None
    bounds = torch.tensor([0.5, 3.0, -1.0], dtype=torch.float64) if cycle else None
    return SweepState(X, v0, ritz, bounds, cycle)


def test_round_trip_is_exact(tmp_path):
    plan = FakePlan()
    s = state(plan)
    s.save(str(tmp_path / "s.npz"), plan)
    r = SweepState.load(str(tmp_path / "s.npz"), plan, device="cpu")
    assert r.cycle == 2
    for a, b in ((s.X, r.X), (s.v0, r.v0), (s.ritz, r.ritz), (s.bounds, r.bounds)):
        assert torch.equal(a, b) and b.is_contiguous()
    # the file is plain arrays: it loads with pickles refused
    with np.load(str(tmp_path / "s.npz"), allow_pickle=False) as z:
        assert set(z.files) == {"meta", "X", "v0", "ritz", "bounds"}
        assert json.loads(str(z["meta"]))["format"] == FORMAT


def test_fresh_state_has_no_ritz_values(tmp_path):
    plan = FakePlan()
    s = state(plan, cycle=0)
    s.save(str(tmp_path / "s.npz"), plan)
    r = SweepState.load(str(tmp_path / "s.npz"), plan, device="cpu")
    assert r.cycle == 0 and r.ritz is None and r.bounds is None


@pytest.mark.parametrize("other", [
    dict(grid=(2, 1, 2)),
    dict(stencil=7),
    dict(J=(8, 8, 8, 12)),          # same N, other counts
])
def test_state_of_another_plan_is_refused(tmp_path, other):
    plan = FakePlan()
    state(plan).save(str(tmp_path / "s.npz"), plan)
    with pytest.raises(ValueError, match="another plan"):
        SweepState.load(str(tmp_path / "s.npz"), FakePlan(**other), device="cpu")


def test_bad_states_are_refused(tmp_path):
    plan = FakePlan()
    s = state(plan)
    with pytest.raises(ValueError):
        SweepState(s.X, s.v0, s.ritz, s.bounds, cycle=0)        # Ritz values but no cycle done
    with pytest.raises(ValueError):
        SweepState(s.X, s.v0, None, None, cycle=1)              # a cycle done but no Ritz values
    with pytest.raises(ValueError):
        SweepState(s.X.float(), s.v0)
    with pytest.raises(ValueError):
        SweepState(s.X, s.v0[:-1])
    p = tmp_path / "x.npz"
    np.savez(str(p), meta=np.array(json.dumps({"format": "something else"})), X=np.zeros((2, 2)))
    with pytest.raises(ValueError, match="not a"):
        SweepState.load(str(p), plan, device="cpu")


def test_fingerprint_names_the_discretisation():
    a, b = FakePlan(), FakePlan(J=(8, 8, 8, 12))
    fa, fb = plan_fingerprint(a, 6), plan_fingerprint(b, 6)
    assert fa["N"] == fb["N"] and fa["J_sha256"] != fb["J_sha256"]
