"""CheFSI cycle (Algorithm 1 of the paper) in plain float64 NumPy.

Test infrastructure: part of the CPU oracle, never imported by the product path.

Each function states the passage of the paper it follows.  Where the paper is
silent the reading taken is stated in the docstring; the same readings bind
the GPU library.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

from .jacobi import jacobi_eigh

# Slot order of the stored blocks of one element: self, -x, +x, -y, +y, -z, +z.
_DIRS = ((0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))


# ----------------------------------------------------------------------------
# Block structure of H^DG (Sec. II A, block partition of H^DG; eqs. matvec_1-3)
# ----------------------------------------------------------------------------
def slot_neighbour(K: int, s: int, grid: Sequence[int]) -> int:
    """Element reached from element K through stencil slot s on a periodic grid."""
    nx, ny, nz = grid
    ix, iy, iz = K % nx, (K // nx) % ny, K // (nx * ny)
    dx, dy, dz = _DIRS[s]
    return ((ix + dx) % nx) + nx * (((iy + dy) % ny) + ny * ((iz + dz) % nz))


def _row_offsets(J) -> np.ndarray:
    off = np.zeros(len(J) + 1, dtype=np.int64)
    off[1:] = np.cumsum(np.asarray(J, dtype=np.int64))
    return off


def assemble_dense(grid, stencil: int, J, blocks) -> np.ndarray:
    """Dense H from its stored nonzero blocks: H[K rows, K' cols] += H_{K;K'}.

    Blocks that reach the same neighbour through two slots (a periodic
    dimension of length 2) or the element itself (length 1) add.
    """
    off = _row_offsets(J)
    N = int(off[-1])
    H = np.zeros((N, N))
    for K in range(len(J)):
        for s in range(stencil):
            Kp = slot_neighbour(K, s, grid)
            B = blocks[K][s]
            assert B.shape == (J[K], J[Kp])
            H[off[K]:off[K + 1], off[Kp]:off[Kp + 1]] += B
    return H


class DenseOperator:
    """H applied as a dense matrix product (the parity authority)."""

    def __init__(self, H: np.ndarray):
        self.H = np.asarray(H, dtype=np.float64)
        self.N = self.H.shape[0]

    def apply(self, Y):
        return self.H @ Y

    def apply_T(self, Y):
        return self.H.T @ Y


class BlockOperator:
    """H applied element by element from its stored blocks (eq. matvec_3):
    y_K = sum over the stencil slots s of H_{K;K'_s} x_{K'_s}."""

    def __init__(self, grid, stencil: int, J, blocks):
        self.grid, self.stencil = tuple(grid), stencil
        self.J = np.asarray(J)
        self.blocks = blocks
        self.off = _row_offsets(J)
        self.N = int(self.off[-1])
        self.nbr = [[slot_neighbour(K, s, grid) for s in range(stencil)] for K in range(len(J))]

    def apply(self, Y):
        off = self.off
        out = np.zeros((self.N,) + Y.shape[1:])
        for K in range(len(self.J)):
            acc = out[off[K]:off[K + 1]]
            for s in range(self.stencil):
                Kp = self.nbr[K][s]
                acc += self.blocks[K][s] @ Y[off[Kp]:off[Kp + 1]]
        return out

    def apply_T(self, Y):
        off = self.off
        out = np.zeros((self.N,) + Y.shape[1:])
        for K in range(len(self.J)):
            for s in range(self.stencil):
                Kp = self.nbr[K][s]
                out[off[Kp]:off[Kp + 1]] += self.blocks[K][s].T @ Y[off[K]:off[K + 1]]
        return out


# ----------------------------------------------------------------------------
# Chebyshev filter (Algorithm 1 step 2; three-term recurrence)
# ----------------------------------------------------------------------------
def chebyshev_T(m: int, t):
    """T_m(t) from its closed form (cos / cosh branches)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    inside = np.abs(t) <= 1.0
    out[inside] = np.cos(m * np.arccos(t[inside]))
    hi = t > 1.0
    out[hi] = np.cosh(m * np.arccosh(t[hi]))
    lo = t < -1.0
    out[lo] = (-1.0) ** m * np.cosh(m * np.arccosh(-t[lo]))
    return out


def chebyshev_coefficients(m: int, a: float, b: float, a0: float):
    """Coefficients of the scaled recurrence Y_{k+1} = alpha_k (H - c I) Y_k - beta_k Y_{k-1}.

    The filter maps the damped interval [a, b] = [b_low, b_up] onto [-1, 1]
    (Algorithm 1 step 2) with L(t) = (t - c)/e, c = (a+b)/2, e = (b-a)/2, and
    is normalised so that p_m(a0) = 1 (scaled form, rho_k = T_k(L(a0))):
        sigma_1 = e/(a0 - c), sigma_{k+1} = 1/(2/sigma_1 - sigma_k),
        alpha_0 = sigma_1/e, beta_0 = 0,
        alpha_k = 2 sigma_{k+1}/e, beta_k = sigma_k sigma_{k+1} (k >= 1).
    Returns (c, [(alpha_k, beta_k) for k = 0..m-1]).
    """
    e = (b - a) / 2.0
    c = (b + a) / 2.0
    sigma1 = e / (a0 - c)
    tau = 2.0 / sigma1
    coefs = [(sigma1 / e, 0.0)]
    sigma = sigma1
    for _ in range(1, m):
        sigma_next = 1.0 / (tau - sigma)
        coefs.append((2.0 * sigma_next / e, sigma * sigma_next))
        sigma = sigma_next
    return c, coefs[:m]


def chebyshev_filter(op, X: np.ndarray, m: int, a: float, b: float, a0: float, return_all=False):
    """Y~ = p_m(H) X with p_m(t) = T_m(L(t)) / T_m(L(a0)) (Algorithm 1 step 2)."""
    if not (a0 < a < b):
        raise ValueError("filter bounds must satisfy a0 < a < b")
    if m < 0:
        raise ValueError("filter degree must be >= 0")
    X = np.asarray(X, dtype=np.float64)
    if m == 0:
        return (X.copy(), [X.copy()]) if return_all else X.copy()
    c, coefs = chebyshev_coefficients(m, a, b, a0)
    Ys = [X]
    Yprev, Y = None, X
    for k, (alpha, beta) in enumerate(coefs):
        Ynew = alpha * (op.apply(Y) - c * Y)
        if k > 0:
            Ynew -= beta * Yprev
        Yprev, Y = Y, Ynew
        Ys.append(Y)
    return (Y, Ys) if return_all else Y


# ----------------------------------------------------------------------------
# Bounds (Algorithm 1 step 1)
# ----------------------------------------------------------------------------
def lanczos(op, v0: np.ndarray, k: int):
    """k steps of Lanczos with full reorthogonalisation (two classical
    Gram-Schmidt passes per step) from start vector v0.

    Returns (alpha[0..j-1], beta[0..j-1]) where j <= k is the number of steps
    taken; the run stops early when beta_j <= 1e-14 * |alpha_1| (an invariant
    subspace has been found).
    """
    v = np.asarray(v0, dtype=np.float64)
    v = v / np.linalg.norm(v)
    V = [v]
    alphas, betas = [], []
    beta_prev = 0.0
    v_prev = np.zeros_like(v)
    for j in range(k):
        w = op.apply(V[j][:, None])[:, 0]
        alpha = float(V[j] @ w)
        w = w - alpha * V[j] - beta_prev * v_prev
        B = np.stack(V, axis=1)
        for _ in range(2):
            w = w - B @ (B.T @ w)
        beta = float(np.linalg.norm(w))
        alphas.append(alpha)
        betas.append(beta)
        if beta <= 1e-14 * abs(alphas[0]):
            break
        v_prev = V[j]
        beta_prev = beta
        V.append(w / beta)
    return np.array(alphas), np.array(betas)


def lanczos_upper_bound(op, v0: np.ndarray, k: int):
    """Upper bound b_up of the spectrum from a few Lanczos steps (Algorithm 1
    step 1): b = theta_max(T_j) + beta_j, together with the Ritz values theta
    of T_j (ascending) and the first components tau of its eigenvectors."""
    alpha, beta = lanczos(op, v0, k)
    j = len(alpha)
    T = np.diag(alpha)
    if j > 1:
        T += np.diag(beta[:j - 1], 1) + np.diag(beta[:j - 1], -1)
    theta, S = jacobi_eigh(T)
    b = float(theta[-1] + beta[j - 1])
    return b, theta, S[0, :].copy()


def _separate(a: float, a0: float, b: float) -> float:
    if a0 >= a - 1e-12 * abs(b):
        a0 = a - 1e-3 * (b - a)
    return a0


def bounds_cold(b: float, theta: np.ndarray, tau: np.ndarray, ns: int, N: int):
    """First-sweep bounds from the Lanczos run (no Ritz values yet).

    The paper takes b_low from previous Ritz values, which a random start
    does not have.  Reading: a0 = smallest Lanczos Ritz value, and a = the
    smallest Lanczos Ritz value theta_j whose cumulative quadrature weight
    sum_{i<=j} tau_i^2 reaches ns/N (an estimate of the spectral point below
    which ns eigenvalues lie).
    """
    w = np.cumsum(np.asarray(tau) ** 2)
    target = ns / float(N)
    j = int(np.searchsorted(w, target, side="left"))
    j = min(j, len(theta) - 1)
    a = float(theta[j])
    a0 = _separate(a, float(theta[0]), b)
    return a, b, a0


def bounds_warm(ritz: np.ndarray, b: float):
    """Bounds from the previous Ritz values (Algorithm 1 step 1):
    a = b_low = largest Ritz value, a0 = smallest Ritz value."""
    a = float(np.max(ritz))
    a0 = _separate(a, float(np.min(ritz)), b)
    return a, b, a0


# ----------------------------------------------------------------------------
# Cholesky-QR (Algorithm 1 step 3; Sec. II B 2)
# ----------------------------------------------------------------------------
class NotPositiveDefinite(ArithmeticError):
    pass


def cholesky_upper(S: np.ndarray) -> np.ndarray:
    """U upper triangular with positive diagonal and U^T U = S (row-oriented
    textbook algorithm); raises NotPositiveDefinite at the first pivot <= 0."""
    S = np.asarray(S, dtype=np.float64)
    n = S.shape[0]
    U = np.zeros_like(S)
    for j in range(n):
        d = S[j, j] - U[:j, j] @ U[:j, j]
        if not (d > 0.0) or not np.isfinite(d):
            raise NotPositiveDefinite(f"pivot {j} is {d}")
        U[j, j] = math.sqrt(d)
        U[j, j + 1:] = (S[j, j + 1:] - U[:j, j] @ U[:j, j + 1:]) / U[j, j]
    return U


def solve_right_upper(Y: np.ndarray, U: np.ndarray) -> np.ndarray:
    """Solve Yhat U = Y for Yhat by substitution over columns (no inverse)."""
    n = U.shape[0]
    Yh = np.empty_like(Y, dtype=np.float64)
    for j in range(n):
        Yh[:, j] = (Y[:, j] - Yh[:, :j] @ U[:j, j]) / U[j, j]
    return Yh


# One pass is kept when 10 eps B^2 <= 1e-12 for the condition bound B of the
# first factor: the predicted orthogonality loss, with a factor 10 over the
# observed eps kappa^2 behaviour, stays within the 1e-12 target (B >= kappa).
AUTO_LOSS_LIMIT = 1e-12
AUTO_LOSS_FACTOR = 10.0


def auto_passes(U1: np.ndarray) -> int:
    """Passes chosen by passes = 0 (auto): 1 if 10 eps B^2 <= 1e-12 for
    B = cholqr_condition_bound(U1), else 2."""
    B = cholqr_condition_bound(U1)
    return 1 if AUTO_LOSS_FACTOR * np.finfo(np.float64).eps * B * B <= AUTO_LOSS_LIMIT else 2


def cholesky_qr(Y: np.ndarray, passes: int = 2):
    """S = Y^T Y, U^T U = S, solve Yhat U = Y (Algorithm 1 step 3).

    passes = 2 repeats the three steps on Yhat (CholeskyQR2, Fukaya et al.
    2014): one pass loses orthogonality like eps * cond(Y)^2.  passes = 0
    factors once and repeats only if auto_passes says so.  Returns Yhat, the
    combined factor U = U_2 U_1 and the per-pass factors.
    """
    if passes not in (0, 1, 2):
        raise ValueError("passes must be 0 (auto), 1 or 2")
    Yh = np.asarray(Y, dtype=np.float64)
    Us = []
    npass = passes if passes else 2
    for i in range(npass):
        S = Yh.T @ Yh
        S = 0.5 * (S + S.T)
        U = cholesky_upper(S)
        Yh = solve_right_upper(Yh, U)
        Us.append(U)
        if passes == 0 and i == 0 and auto_passes(U) == 1:
            break
    Utot = Us[0] if len(Us) == 1 else Us[1] @ Us[0]
    return Yh, Utot, Us


def cholqr_condition_bound(U: np.ndarray) -> float:
    """Upper bound on the 2-norm condition number of the column-equilibrated
    block Y D^{-1} (D = column norms of Y) from its Cholesky factor U:
    with U_e = U D^{-1} (D_j = norm of column j of U, which is ||y_j||) and
    T_e = U_e^{-1}, kappa_2 <= sqrt(kappa_1 kappa_inf), where kappa_1 and
    kappa_inf are the exact 1- and inf-norm condition numbers of U_e
    (||A||_2^2 <= ||A||_1 ||A||_inf).  One Cholesky-QR pass loses
    orthogonality like eps kappa_2^2 (Sec. II B 2 uses one pass); the bound
    decides whether a second pass is needed."""
    U = np.triu(np.asarray(U, dtype=np.float64))
    d = np.sqrt(np.sum(U * U, axis=0))
    Ue = U / d[None, :]
    Te = np.linalg.inv(Ue)
    k1 = np.abs(Ue).sum(axis=0).max() * np.abs(Te).sum(axis=0).max()
    ki = np.abs(Ue).sum(axis=1).max() * np.abs(Te).sum(axis=1).max()
    return float(math.sqrt(k1 * ki))


# ----------------------------------------------------------------------------
# Rayleigh-Ritz and subspace rotation (Algorithm 1 steps 4 and 5)
# ----------------------------------------------------------------------------
def sign_normalize(Q: np.ndarray) -> np.ndarray:
    """Flip each column so that its largest-magnitude entry (lowest index on
    ties) is positive."""
    Q = np.array(Q, copy=True)
    idx = np.argmax(np.abs(Q), axis=0)
    sgn = np.sign(Q[idx, np.arange(Q.shape[1])])
    sgn[sgn == 0] = 1.0
    return Q * sgn[None, :]


def symmetric_eig(A: np.ndarray):
    """Ascending eigenpairs: the oracle's own Jacobi up to order 256, the
    LAPACK driver above that."""
    if A.shape[0] <= 256:
        return jacobi_eigh(A)
    return np.linalg.eigh(A)


def rayleigh_ritz(op, Yh: np.ndarray, col_chunk: int = 0):
    """Hhat = Yhat^T (H Yhat), Hhat Q = Q D, X_new = Yhat Q, residuals
    r_i = ||H x_i - theta_i x_i||_2 (Algorithm 1 steps 4-5).

    col_chunk > 0 forms the columns of H Yhat (and of Hhat) and the residual
    columns that many at a time, to bound the memory of very tall blocks;
    every column is the same product as without it."""
    N, ns = Yh.shape
    step = col_chunk if col_chunk > 0 else ns
    Hh = np.empty((ns, ns))
    for c0 in range(0, ns, step):
        W = op.apply(Yh[:, c0:c0 + step])
        Hh[:, c0:c0 + step] = Yh.T @ W
        del W
    Hh = 0.5 * (Hh + Hh.T)
    theta, Q = symmetric_eig(Hh)
    Q = sign_normalize(Q)
    Xn = Yh @ Q
    resid = np.empty(ns)
    for c0 in range(0, ns, step):
        Xc = Xn[:, c0:c0 + step]
        R = op.apply(Xc) - Xc * theta[None, c0:c0 + step]
        resid[c0:c0 + step] = np.sqrt(np.sum(R * R, axis=0))
        del R
    return Xn, theta, resid, Q, Hh


def sweep(op, X: np.ndarray, m: int, bounds: Tuple[float, float, float], passes: int = 2):
    """One CheFSI cycle with explicit filter bounds (a, b, a0)."""
    a, b, a0 = bounds
    Yt = chebyshev_filter(op, X, m, a, b, a0)
    Yh, U, _ = cholesky_qr(Yt, passes)
    Xn, theta, resid, Q, Hh = rayleigh_ritz(op, Yh)
    return Xn, theta, resid


def run_sweeps(op, X0: np.ndarray, v0: np.ndarray, m: int, nsweeps: int,
               lanczos_steps: int = 20, passes: int = 2):
    """nsweeps CheFSI cycles from a random start: Lanczos bound once, cold
    bounds for the first cycle, Ritz-value bounds afterwards."""
    b, theta_l, tau = lanczos_upper_bound(op, v0, lanczos_steps)
    N, ns = X0.shape
    bounds = bounds_cold(b, theta_l, tau, ns, N)
    X = X0
    history = []
    for _ in range(nsweeps):
        X, theta, resid = sweep(op, X, m, bounds, passes)
        history.append((bounds, theta, resid))
        bounds = bounds_warm(theta, b)
    return X, theta, resid, history
