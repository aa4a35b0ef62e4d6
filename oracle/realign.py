"""Re-alignment of the eigenvector coefficients to a new ALB basis, in plain
float64 NumPy.

Test infrastructure: part of the CPU oracle, never imported by the product path.

Sec. II B 3 of the paper: the basis changes between SCF steps, so the
coefficients X^(i) (N_b x N_s) of the previous step are carried over by l2
projection onto the new basis, X^(i+1) = (V^{i+1})^T V^i X^(i) (eq.
basis_rotation_1), where V^i (N_r x N_b) samples the ALBs on the real-space
grid.  Because ALBs of different elements have disjoint supports, this splits
into one small product per element, X^(i+1)_K = (V^{i+1}_K)^T V^i_K X^(i)_K
(eqs. basis_rotation_2-3), with V_K the n_r x J_K samples of element K's ALBs
on its own n_r grid points.

Layout of the ALB samples (the library's): element-major; element K holds
V_K^T, i.e. J_K rows of n_r samples (row j = ALB j on the element's grid),
row-major, starting at n_r * rowoff[K].  The grid of every element has the same
n_r points.
"""
from __future__ import annotations

import numpy as np


def _row_offsets(J) -> np.ndarray:
    off = np.zeros(len(J) + 1, dtype=np.int64)
    off[1:] = np.cumsum(np.asarray(J, dtype=np.int64))
    return off


def element_samples(J, nr: int, V_packed: np.ndarray, K: int) -> np.ndarray:
    """V_K (n_r x J_K) of element K from the packed layout."""
    off = _row_offsets(J)
    flat = np.asarray(V_packed, dtype=np.float64)
    return flat[nr * off[K]:nr * off[K + 1]].reshape(int(J[K]), nr).T


def overlap_blocks(J, nr: int, V_new: np.ndarray, V_old: np.ndarray) -> list:
    """R_K = (V^{i+1}_K)^T V^i_K, J_K x J_K, for every element."""
    return [element_samples(J, nr, V_new, K).T @ element_samples(J, nr, V_old, K)
            for K in range(len(J))]


def realign(J, nr: int, V_new: np.ndarray, V_old: np.ndarray, X: np.ndarray) -> np.ndarray:
    """X^(i+1)_K = R_K X^(i)_K element by element (eq. basis_rotation_3)."""
    X = np.asarray(X, dtype=np.float64)
    off = _row_offsets(J)
    out = np.empty_like(X)
    for K, R in enumerate(overlap_blocks(J, nr, V_new, V_old)):
        out[off[K]:off[K + 1]] = R @ X[off[K]:off[K + 1]]
    return out


def assemble_samples(J, nr: int, V_packed: np.ndarray) -> np.ndarray:
    """The whole N_r x N_b sample matrix V (N_r = M n_r): element K's grid
    points are rows K n_r .. (K+1) n_r - 1 and its ALBs are columns
    rowoff[K] .. rowoff[K+1] - 1; all other entries are zero (disjoint
    supports)."""
    off = _row_offsets(J)
    M = len(J)
    V = np.zeros((M * nr, int(off[-1])))
    for K in range(M):
        V[K * nr:(K + 1) * nr, off[K]:off[K + 1]] = element_samples(J, nr, V_packed, K)
    return V


def realign_dense(J, nr: int, V_new: np.ndarray, V_old: np.ndarray, X: np.ndarray) -> np.ndarray:
    """X^(i+1) = (V^{i+1})^T V^i X^(i) with the whole sample matrices (eq.
    basis_rotation_1); only for small sizes."""
    Vn = assemble_samples(J, nr, V_new)
    Vo = assemble_samples(J, nr, V_old)
    return Vn.T @ (Vo @ np.asarray(X, dtype=np.float64))
