"""The Python binding rejects unusable tensors before it calls the library:
host tensors, wrong dtypes, short vectors or a foreign workspace never reach a
kernel.  Runs without a GPU (the plan object is built without the library, so
any library call would fail with a ChefsiError, not a ValueError)."""
import numpy as np
import pytest
import torch

import paper_1606_03416_amd as chefsi
from paper_1606_03416_amd import _binding


def fake_plan(N=256, h_elems=7 * 8 * 32 * 32, ns=48):
    p = object.__new__(chefsi.Plan)
    p._h = None
    p.N, p.h_elems, p.block_elems = N, h_elems, 8 * 32 * 32
    p.J = np.full(8, 32, dtype=np.int32)
    p.device = torch.device("cuda", 0)
    return p


def cpu(*shape, dtype=torch.float64):
    return torch.zeros(*shape, dtype=dtype)


def test_sweep_rejects_host_tensors_before_any_library_call():
    p = fake_plan()
    H, X = cpu(p.h_elems), cpu(p.N, 48)
    with pytest.raises(ValueError, match="H must be"):
        p.sweep(H, X, 10, v0=cpu(p.N))


def test_multivector_checks():
    with pytest.raises(ValueError, match="CUDA"):
        _binding._mv(cpu(256, 48), "X", 256)
    with pytest.raises(ValueError, match="CUDA"):
        _binding._mv(np.zeros((256, 48)), "X", 256)
    with pytest.raises(ValueError):
        _binding._vec(cpu(255), "v0", 256)
    with pytest.raises(ValueError):
        _binding._vec(cpu(256, dtype=torch.float32), "ritz", 256)
    with pytest.raises(ValueError, match="uint8"):
        _binding._user_ws(cpu(1024, dtype=torch.uint8), None)
    with pytest.raises(ValueError, match="uint8"):
        _binding._user_ws(cpu(1024, dtype=torch.float64), None)


def test_every_plan_method_checks_first():
    p = fake_plan()
    H, X = cpu(p.h_elems), cpu(p.N, 48)
    calls = [
        lambda: p.bounds(H, cpu(p.N), ns=48),
        lambda: p.filter(H, X, 4, 0.0, 1.0, -1.0),
        lambda: p.rayleigh_ritz(H, X),
        lambda: p.sweep(H, X, 4, bounds=(0.0, 1.0, -1.0)),
        lambda: p.loss_backward(H, X, 4, 0.0, 1.0, -1.0, 8),
        lambda: p.filter_backward(H, X, X, 4, 0.0, 1.0, -1.0),
        lambda: p.density_blocks(X, cpu(48)),
        lambda: p.realign(X, cpu(p.N * 16), cpu(p.N * 16), 16),
        lambda: chefsi.orthonormalize(X),
        lambda: chefsi.orthonormalize_backward(X, cpu(48, 48), X),
        lambda: p.loss(H, X, 4, 0.0, 1.0, -1.0, 8),
        lambda: p.rayleigh_ritz_backward(H, X, cpu(48, 48), cpu(48)),
        lambda: chefsi.occupations(cpu(48), 10.0, 1e-3),
    ]
    for c in calls:
        with pytest.raises(ValueError):
            c()
