"""Occupations and diagonal density-matrix blocks after a CheFSI cycle, in
plain float64 NumPy.

Test infrastructure: part of the CPU oracle, never imported by the product path.

The paper computes, once a cycle has produced Ritz pairs (theta_i, x_i):
  * occupation numbers f_i in [0, 1] by Fermi-Dirac smearing at electronic
    temperature T (Sec. II A, the free-energy functional and the paragraph
    after it; Sec. II B 2, the Ritz values give the Fermi energy and the
    occupations; Sec. III, 300 K);
  * the diagonal blocks of the density matrix (eq. densitymatrix with K = K'):
    P_{K;K}[j, j'] = sum_i f_i x_i[K, j] x_i[K, j'], one J_K x J_K block per
    element, which is all the electron density needs (eq.
    electron_density_from_DM) and is local to each element.

Readings (the paper does not spell these out):
  * f_i = 1 / (1 + exp((theta_i - mu)/kT)) per spatial orbital, with the spin
    factor 2 kept outside (it multiplies the density); the Fermi level mu is
    fixed by sum_i f_i = n_occ, the number of occupied orbital pairs N_e / 2.
  * mu is found by bisection on g(mu) = sum_i f_i(mu) - n_occ, which is
    continuous and strictly increasing in mu, from the bracket
    [theta_min - 50 kT, theta_max + 50 kT] (there g < 0 < g for
    0 < n_occ < ns), halving until the midpoint is no longer strictly inside
    the bracket (the interval is exhausted in float64) or 200 halvings; mu is
    the midpoint of the final bracket.
"""
from __future__ import annotations

import numpy as np

BISECTION_MAX = 200
BRACKET_KT = 50.0


def fermi_dirac(theta, mu: float, kT: float) -> np.ndarray:
    """Fermi-Dirac occupation 1 / (1 + exp((theta - mu)/kT)) of each level
    (exp overflow gives occupation 0, as the limit says)."""
    x = (np.asarray(theta, dtype=np.float64) - mu) / kT
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(x))


def fermi_level(theta, n_occ: float, kT: float) -> float:
    """Fermi level mu with sum_i f_i(mu) = n_occ, by bisection (module
    docstring gives the bracket and the stopping rule)."""
    theta = np.asarray(theta, dtype=np.float64)
    ns = theta.size
    if not (kT > 0.0 and np.isfinite(kT)):
        raise ValueError("kT must be positive and finite")
    if not (0.0 < n_occ < ns):
        raise ValueError("n_occ must lie strictly between 0 and the number of levels")
    if not np.all(np.isfinite(theta)):
        raise ValueError("Ritz values must be finite")
    lo = float(theta.min()) - BRACKET_KT * kT
    hi = float(theta.max()) + BRACKET_KT * kT
    for _ in range(BISECTION_MAX):
        mid = 0.5 * (lo + hi)
        if not (lo < mid < hi):
            break
        if float(np.sum(fermi_dirac(theta, mid, kT))) < n_occ:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def occupations(theta, n_occ: float, kT: float):
    """(mu, f): the Fermi level and the occupation of every Ritz value."""
    mu = fermi_level(theta, n_occ, kT)
    return mu, fermi_dirac(theta, mu, kT)


def _row_offsets(J) -> np.ndarray:
    off = np.zeros(len(J) + 1, dtype=np.int64)
    off[1:] = np.cumsum(np.asarray(J, dtype=np.int64))
    return off


def density_diag_blocks(J, X: np.ndarray, f) -> list:
    """P_{K;K} = X_K diag(f) X_K^T for every element K (eq. densitymatrix with
    K = K'), X_K the J_K rows of element K of the N x ns Ritz vectors."""
    X = np.asarray(X, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    off = _row_offsets(J)
    out = []
    for K in range(len(J)):
        XK = X[off[K]:off[K + 1]]
        out.append((XK * f[None, :]) @ XK.T)
    return out


def density_dense(X: np.ndarray, f) -> np.ndarray:
    """The whole N x N density matrix P = X diag(f) X^T (eq. densitymatrix);
    only for small N, to check the element blocks against."""
    X = np.asarray(X, dtype=np.float64)
    return (X * np.asarray(f, dtype=np.float64)[None, :]) @ X.T


def pack_blocks(blocks) -> np.ndarray:
    """Element blocks back to back, each row-major (the library's layout)."""
    return np.concatenate([np.asarray(b, dtype=np.float64).ravel() for b in blocks])
