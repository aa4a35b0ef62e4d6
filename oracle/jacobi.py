"""Cyclic two-sided Jacobi eigensolver for small dense symmetric matrices.

Test infrastructure (part of the CPU oracle).  Textbook cyclic-by-row Jacobi
(Golub & Van Loan, "Matrix Computations", the symmetric Schur 2x2 rotation
and the cyclic Jacobi sweep): every off-diagonal pair (p, q) is annihilated in
turn by a plane rotation until the off-diagonal Frobenius norm is below a
relative tolerance.  Used by the oracle for the Lanczos tridiagonal T_k and for
projected matrices of order <= 256, where a Python loop over pairs is fast
enough; its output is pinned against numpy.linalg.eigh in the tests.
"""
from __future__ import annotations

import numpy as np


def _schur2(app: float, aqq: float, apq: float):
    """Rotation (c, s) that zeroes the (p, q) entry of a symmetric 2x2 block."""
    if apq == 0.0:
        return 1.0, 0.0
    tau = (aqq - app) / (2.0 * apq)
    if tau >= 0.0:
        t = 1.0 / (tau + np.sqrt(1.0 + tau * tau))
    else:
        t = -1.0 / (-tau + np.sqrt(1.0 + tau * tau))
    c = 1.0 / np.sqrt(1.0 + t * t)
    return c, t * c


def jacobi_eigh(A: np.ndarray, rtol: float = 1e-15, max_sweeps: int = 60):
    """Eigenvalues (ascending) and orthonormal eigenvectors (columns) of symmetric A."""
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    assert A.shape == (n, n)
    V = np.eye(n)
    if n == 1:
        return A.diagonal().copy(), V
    fro = np.linalg.norm(A)
    if fro == 0.0:
        return np.zeros(n), V
    for _ in range(max_sweeps):
        off = np.linalg.norm(A - np.diag(A.diagonal()))
        if off <= rtol * fro:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = A[p, q]
                if abs(apq) <= 1e-300:
                    continue
                c, s = _schur2(A[p, p], A[q, q], apq)
                cp = A[:, p].copy()
                cq = A[:, q].copy()
                A[:, p] = c * cp - s * cq
                A[:, q] = s * cp + c * cq
                rp = A[p, :].copy()
                rq = A[q, :].copy()
                A[p, :] = c * rp - s * rq
                A[q, :] = s * rp + c * rq
                A[p, q] = 0.0
                A[q, p] = 0.0
                vp = V[:, p].copy()
                vq = V[:, q].copy()
                V[:, p] = c * vp - s * vq
                V[:, q] = s * vp + c * vq
    w = A.diagonal().copy()
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order]
