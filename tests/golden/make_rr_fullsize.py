"""Writes the stored expected values of the full-size Rayleigh-Ritz parity test
(tests/test_gpu_rr_fullsize.py) from the CPU oracle alone.

For the bulk (12 x 12 x 12 elements, 64 ALBs, N = 110,592, N_s = 4,096) and
sheet (48 x 40 elements, 64..128 ALBs, N = 184,584, N_s = 8,192) workloads:
the input is synth.make_orthonormal_block(N, N_s), a dense block with
orthonormal columns; the oracle's Rayleigh-Ritz (Algorithm 1 steps 4-5, H
applied block by block, LAPACK eigensolver) gives every Ritz value, every
residual norm and a sample of eigenvector columns of the projected matrix.

    python tests/golden/make_rr_fullsize.py [bulk] [sheet]

Output: tests/golden/rr_fullsize_<workload>.npz (theta, resid, q_idx, q_cols,
hh_fro).  Takes minutes and ~40 GB of host memory for the sheet.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

WORKLOADS = {"bulk": synth.BULK, "sheet": synth.SHEET}
SAMPLES = 12


def sample_indices(ns: int) -> np.ndarray:
    """Eigenvector columns kept: both ends, the wanted-set edge, and evenly
    spread interior ones."""
    k = 3 * ns // 4
    idx = {0, 1, k - 1, k, ns - 2, ns - 1}
    idx.update(int(v) for v in np.linspace(2, ns - 3, SAMPLES - len(idx)))
    return np.array(sorted(idx), dtype=np.int64)


def make(name: str) -> str:
    w = WORKLOADS[name]
    t0 = time.time()
    P = synth.make_problem(w)
    op = oracle.BlockOperator(P.grid, P.stencil, P.J, P.blocks)
    Yh = synth.make_orthonormal_block(P.N, w.ns)
    print(f"[{name}] N={P.N} ns={w.ns}: inputs in {time.time() - t0:.1f} s", flush=True)
    Xn, theta, resid, Q, Hh = oracle.rayleigh_ritz(op, Yh, col_chunk=512)
    del Xn, Yh
    idx = sample_indices(w.ns)
    out = os.path.join(HERE, f"rr_fullsize_{name}.npz")
    np.savez_compressed(out, theta=theta, resid=resid, q_idx=idx, q_cols=Q[:, idx].copy(),
                        hh_fro=np.array(np.linalg.norm(Hh)))
    print(f"[{name}] wrote {out} after {time.time() - t0:.1f} s", flush=True)
    return out


if __name__ == "__main__":
    for n in (sys.argv[1:] or ["bulk", "sheet"]):
        make(n)
