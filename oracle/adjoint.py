"""Reverse-mode gradient of one filter + Cholesky-QR + Rayleigh-Ritz pass.

Test infrastructure: part of the CPU oracle.  The paper does not
differentiate the CheFSI cycle; these are the textbook reverse-mode rules for
each step of Algorithm 1 (steps 2-4) with the filter bounds held constant:

* loss L = sum of the k lowest Ritz values;
* eigenvalues:  dtheta_i = q_i^T dHhat q_i, so Hhat_bar = Q diag(theta_bar) Q^T;
* projection Hhat = sym(Yhat^T H Yhat):
      Yhat_bar = H Yhat Hhat_bar + H^T Yhat Hhat_bar,  H_bar += Yhat Hhat_bar Yhat^T;
* thin QR Y = Yhat U with U unused downstream (the QR backward rule with
  R_bar = 0):  M = -Yhat_bar^T Yhat,
      Y_bar = (Yhat_bar + Yhat copyltu(M)) U^{-T},  copyltu(M) = tril(M) + tril(M,-1)^T;
  with two passes the rule is applied to each pass in reverse order;
* three-term recurrence Y_{j+1} = alpha_j (H - cI) Y_j - beta_j Y_{j-1}:
      Lambda_m = Y~_bar, Lambda_{m+1} = 0,
      Lambda_j = alpha_j (H^T - cI) Lambda_{j+1} - beta_{j+1} Lambda_{j+2}  (beta_m := 0),
      H_bar += sum_j alpha_j Lambda_{j+1} Y_j^T,   X_bar = Lambda_0.

H_bar is the gradient with respect to the *stored* blocks: the dense gradient
restricted to the block pattern (not symmetrised).  Two stored blocks that
land on the same dense block (duplicate neighbours) both receive it.
"""
from __future__ import annotations

import numpy as np

from . import core


def restrict_to_pattern(Gd: np.ndarray, grid, stencil: int, J):
    """Stored-block view [K][s] of a dense N x N gradient."""
    off = core._row_offsets(J)
    out = []
    for K in range(len(J)):
        row = []
        for s in range(stencil):
            Kp = core.slot_neighbour(K, s, grid)
            row.append(Gd[off[K]:off[K + 1], off[Kp]:off[Kp + 1]].copy())
        out.append(row)
    return out


class _PatternAccumulator:
    """Accumulates sum_j A_j B_j^T either densely or block by block."""

    def __init__(self, op):
        self.op = op
        if isinstance(op, core.DenseOperator):
            self.dense = np.zeros((op.N, op.N))
            self.blocks = None
        else:
            self.dense = None
            self.blocks = [[np.zeros_like(B) for B in row] for row in op.blocks]

    def add_outer(self, A: np.ndarray, B: np.ndarray, scale: float = 1.0):
        if self.dense is not None:
            self.dense += scale * (A @ B.T)
            return
        op = self.op
        off = op.off
        for K in range(len(op.J)):
            for s in range(op.stencil):
                Kp = op.nbr[K][s]
                self.blocks[K][s] += scale * (A[off[K]:off[K + 1]] @ B[off[Kp]:off[Kp + 1]].T)

    def result(self, grid=None, stencil=None, J=None):
        if self.dense is not None:
            return self.dense
        return self.blocks


def _copyltu(M: np.ndarray) -> np.ndarray:
    L = np.tril(M)
    return L + np.tril(M, -1).T


def _solve_right_upper_T(B: np.ndarray, U: np.ndarray) -> np.ndarray:
    """X with X U^T = B (U upper), by back substitution over columns."""
    n = U.shape[0]
    X = np.empty_like(B, dtype=np.float64)
    for j in range(n - 1, -1, -1):
        X[:, j] = (B[:, j] - X[:, j + 1:] @ U[j, j + 1:]) / U[j, j]
    return X


def cholesky_qr_backward(Yh_passes, Us, Yh_bar):
    """Adjoint of the (one- or two-pass) Cholesky-QR.

    Yh_passes[p] is the output of pass p and Us[p] its triangular factor.
    """
    G = Yh_bar
    for p in range(len(Us) - 1, -1, -1):
        Q, U = Yh_passes[p], Us[p]
        M = -(G.T @ Q)
        G = _solve_right_upper_T(G + Q @ _copyltu(M), U)
    return G


def rayleigh_ritz_backward(op, Yh: np.ndarray, Q: np.ndarray, theta_bar: np.ndarray, acc):
    Hh_bar = (Q * theta_bar[None, :]) @ Q.T
    YH = Yh @ Hh_bar
    Yh_bar = op.apply(YH) + op.apply_T(YH)
    acc.add_outer(YH, Yh)          # H_bar += Yhat Hhat_bar Yhat^T
    return Yh_bar


def filter_backward(op, Ys, m: int, a: float, b: float, a0: float, Yt_bar: np.ndarray, acc):
    """Reverse three-term sweep; Ys = [Y_0 .. Y_m] from the forward filter."""
    if m == 0:
        return Yt_bar.copy()
    c, coefs = core.chebyshev_coefficients(m, a, b, a0)
    lam_next = Yt_bar               # Lambda_{j+1}
    lam_next2 = np.zeros_like(Yt_bar)  # Lambda_{j+2}
    for j in range(m - 1, -1, -1):
        alpha_j = coefs[j][0]
        beta_next = coefs[j + 1][1] if j + 1 < m else 0.0
        acc.add_outer(lam_next, Ys[j], alpha_j)
        lam = alpha_j * (op.apply_T(lam_next) - c * lam_next) - beta_next * lam_next2
        lam_next2, lam_next = lam_next, lam
    return lam_next


def loss_forward(op, X: np.ndarray, m: int, bounds, k: int, passes: int = 2):
    """L = sum of the k lowest Ritz values after one filter + Cholesky-QR + RR."""
    a, b, a0 = bounds
    Yt, Ys = core.chebyshev_filter(op, X, m, a, b, a0, return_all=True)
    Yh = Yt
    Yh_passes, Us = [], []
    for _ in range(passes):
        Yh, U, _ = core.cholesky_qr(Yh, 1)
        Yh_passes.append(Yh)
        Us.append(U)
    W = op.apply(Yh)
    Hh = Yh.T @ W
    Hh = 0.5 * (Hh + Hh.T)
    theta, Q = core.symmetric_eig(Hh)
    L = float(np.sum(theta[:k]))
    cache = dict(X=X, m=m, bounds=bounds, k=k, Ys=Ys, Yh_passes=Yh_passes, Us=Us,
                 Yh=Yh, Q=Q, theta=theta)
    return L, cache


def loss_backward(op, cache):
    """(H_bar, X_bar): H_bar dense N x N for a DenseOperator, else stored blocks."""
    k, theta = cache["k"], cache["theta"]
    theta_bar = np.zeros_like(theta)
    theta_bar[:k] = 1.0
    acc = _PatternAccumulator(op)
    Yh_bar = rayleigh_ritz_backward(op, cache["Yh"], cache["Q"], theta_bar, acc)
    Yt_bar = cholesky_qr_backward(cache["Yh_passes"], cache["Us"], Yh_bar)
    a, b, a0 = cache["bounds"]
    X_bar = filter_backward(op, cache["Ys"], cache["m"], a, b, a0, Yt_bar, acc)
    return acc.result(), X_bar
