"""Resumable CheFSI state (host-side plumbing, no arithmetic of the method).

A CheFSI run carries from one cycle of Algorithm 1 (steps 1-5) to the next:
the block X, the previous cycle's Ritz values (where the warm lower bounds a
and a0 come from), the Lanczos start vector v0 of the upper-bound estimate,
the bounds used last and the number of cycles done.  SweepState holds them as
device tensors, writes them to an .npz file (plain arrays and a JSON header, no
pickled objects) together with a fingerprint of the plan, and reads them back
onto a device.  Every reduction in the library runs in a fixed order, so a run
resumed from a saved state reproduces the uninterrupted run bit for bit.

    st = SweepState(X, v0)
    run_cycles(plan, H, st, 2, m)            # cycles 1-2 (cold, then warm)
    st.save("run.npz", plan)
    st = SweepState.load("run.npz", plan)    # later, in another process
    run_cycles(plan, H, st, 2, m)            # cycles 3-4
"""
import hashlib
import json
from typing import Optional

import numpy as np
import torch

from ._binding import F64

FORMAT = "chefsi-sweep-state/1"
_PLAN_KEYS = ("grid", "stencil", "N", "ns", "J_sha256")


def plan_fingerprint(plan, ns: int) -> dict:
    """What a saved state must agree with before it can resume on `plan`."""
    J = np.ascontiguousarray(np.asarray(plan.J), dtype=np.int32)
    return {"format": FORMAT, "grid": [int(v) for v in plan.grid], "stencil": int(plan.stencil),
            "N": int(plan.N), "ns": int(ns), "J_sha256": hashlib.sha256(J.tobytes()).hexdigest()}


def _f64(t, name, shape):
    if not torch.is_tensor(t) or t.dtype != torch.float64 or tuple(t.shape) != shape:
        raise ValueError(f"{name} must be a float64 tensor of shape {shape}")
    return t


class SweepState:
    """X (N x ns, updated in place by the cycles), v0 (N), the last Ritz values
    (ns, None before the first cycle), the last bounds (a, b, a0) and the
    number of cycles done."""

    def __init__(self, X: torch.Tensor, v0: torch.Tensor, ritz: Optional[torch.Tensor] = None,
                 bounds: Optional[torch.Tensor] = None, cycle: int = 0):
        if not torch.is_tensor(X) or X.dim() != 2:
            raise ValueError("X must be an N x ns tensor")
        N, ns = X.shape
        self.X = _f64(X, "X", (N, ns))
        self.v0 = _f64(v0, "v0", (N,))
        self.ritz = None if ritz is None else _f64(ritz, "ritz", (ns,))
        self.bounds = None if bounds is None else _f64(bounds, "bounds", (3,))
        if int(cycle) < 0 or (int(cycle) > 0) != (ritz is not None):
            raise ValueError("cycle counts the cycles done: ritz is given exactly when cycle > 0")
        self.cycle = int(cycle)

    def save(self, path: str, plan) -> None:
        """Write the state and the plan's fingerprint to `path` (.npz)."""
        meta = plan_fingerprint(plan, self.X.shape[1])
        if tuple(self.X.shape) != (meta["N"], meta["ns"]):
            raise ValueError("X does not belong to this plan")
        meta["cycle"] = self.cycle
        arrays = {"meta": np.array(json.dumps(meta, sort_keys=True)),
                  "X": self.X.detach().cpu().numpy(), "v0": self.v0.detach().cpu().numpy()}
        if self.ritz is not None:
            arrays["ritz"] = self.ritz.detach().cpu().numpy()
        if self.bounds is not None:
            arrays["bounds"] = self.bounds.detach().cpu().numpy()
        with open(path, "wb") as f:
            np.savez(f, **arrays)

    @classmethod
    def load(cls, path: str, plan, device=None) -> "SweepState":
        """Read a state written by save(); it must have been saved for the same
        grid, stencil and ALB counts (and column count)."""
        with np.load(path, allow_pickle=False) as z:
            meta = json.loads(str(z["meta"]))
            if meta.get("format") != FORMAT:
                raise ValueError(f"{path}: not a {FORMAT} file")
            expect = plan_fingerprint(plan, int(meta.get("ns", -1)))
            for k in _PLAN_KEYS:
                if meta.get(k) != expect[k]:
                    raise ValueError(f"{path}: the state was saved for another plan ({k} differs)")
            if z["X"].shape != (meta["N"], meta["ns"]) or z["X"].dtype != np.float64:
                raise ValueError(f"{path}: X has the wrong shape or type")
            dev = torch.device(device) if device is not None else plan.device

            def put(name):
                return torch.from_numpy(np.ascontiguousarray(z[name])).to(dev) if name in z.files else None

            return cls(put("X"), put("v0"), put("ritz"), put("bounds"), int(meta["cycle"]))


def run_cycles(plan, H, state: SweepState, n: int, m: int, *, dtype: int = F64, passes: int = 0,
               lanczos_steps: int = 20, ws: Optional[torch.Tensor] = None):
    """n more CheFSI cycles from `state` (X updated in place): the first cycle
    of a fresh state takes cold bounds, every later one the warm bounds from the
    previous Ritz values.  Returns the last cycle's residual norms."""
    resid = None
    for _ in range(int(n)):
        ritz, resid, bnd, _ = plan.sweep(H, state.X, m, dtype=dtype, passes=passes, lanczos_steps=lanczos_steps,
                                         v0=state.v0, ritz=state.ritz, warm=state.ritz is not None, ws=ws)
        state.ritz, state.bounds = ritz, bnd
        state.cycle += 1
    return resid
