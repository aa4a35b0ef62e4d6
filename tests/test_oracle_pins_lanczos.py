"""Pins of the oracle's Lanczos run (Algorithm 1 step 1: the upper bound b_up
from a few Lanczos steps; the first-cycle bounds from its quadrature weights)
against facts that do not come from the oracle:

* the Lanczos vectors are the orthonormalised Krylov sequence, so T_k is
  Q^T H Q for Q from a Householder QR (LAPACK) of any nested basis of the
  Krylov space (here the Chebyshev vectors T_p(L(H)) v, which stay well
  conditioned);
* Gauss quadrature: sum_i tau_i^2 f(theta_i) = v^T f(H) v exactly for every
  polynomial f of degree <= 2k - 1;
* a run of N steps reproduces the whole spectrum of H and the squared
  components of v along its eigenvectors (LAPACK eigh);
* with prescribed spectral weights of the start vector, the first-cycle rule
  picks a known eigenvalue (exact rational arithmetic).

Planted slips (weights from the wrong axis of T_k's eigenvector matrix,
beta_{k-1} in place of beta_k, T_k without its off-diagonal, tau in place of
tau^2) must fail.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import core


def tiny_h():
    P = synth.make_problem(synth.TINY)
    return oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks), synth.make_lanczos_start(P.N)


def mixed_h():
    J = np.array([8, 16, 24, 8, 16, 8], dtype=np.int32)
    P = synth.make_blocks((3, 2, 1), 5, J)
    return oracle.assemble_dense(P.grid, P.stencil, P.J, P.blocks), synth.make_lanczos_start(P.N)


def cheb_vectors(H, v, count):
    """T_p(L(H)) v for p < count, L mapping the spectrum into [-1, 1]."""
    lam = np.linalg.eigvalsh(H)
    c, r = 0.5 * (lam[-1] + lam[0]), 0.505 * (lam[-1] - lam[0])
    Ls = (H - c * np.eye(H.shape[0])) / r
    out = [v, Ls @ v]
    for _ in range(2, count):
        out.append(2.0 * (Ls @ out[-1]) - out[-2])
    return out[:count], (lambda t: (np.asarray(t) - c) / r)


def krylov_tridiagonal(H, v0, k):
    """T_{k+1} = Q^T H Q, Q the Householder-QR basis of K_{k+1}(H, v) with the
    sign of every column chosen so that the subdiagonal is positive."""
    v = v0 / np.linalg.norm(v0)
    K, _ = cheb_vectors(H, v, k + 1)
    Q, R = np.linalg.qr(np.stack(K, axis=1))
    Q = Q * np.sign(np.diag(R))[None, :]
    return Q.T @ H @ Q


# ------------------------------------------------------------- pin checks
def tridiagonal_error(lanczos_fn, H, v0, k):
    alpha, beta = lanczos_fn(oracle.DenseOperator(H), v0, k)
    T = krylov_tridiagonal(H, v0, k)
    a_ref = np.diag(T)[:k]
    b_ref = np.array([T[j + 1, j] for j in range(k)])
    return max(np.max(np.abs(alpha - a_ref)), np.max(np.abs(beta - b_ref)))


def upper_bound_error(ub_fn, H, v0, k):
    b, _, _ = ub_fn(oracle.DenseOperator(H), v0, k)
    T = krylov_tridiagonal(H, v0, k)
    b_ref = float(np.linalg.eigvalsh(T[:k, :k])[-1] + T[k, k - 1])
    return abs(b - b_ref)


def quadrature_error(ub_fn, H, v0, k):
    """max_p |sum_i tau_i^2 T_p(L(theta_i)) - v^T T_p(L(H)) v|, p < 2k."""
    _, theta, tau = ub_fn(oracle.DenseOperator(H), v0, k)
    v = v0 / np.linalg.norm(v0)
    vecs, L = cheb_vectors(H, v, 2 * k)
    mom = np.array([v @ x for x in vecs])
    t = L(theta)
    Tq = [np.ones_like(t), t]
    for _ in range(2, 2 * k):
        Tq.append(2.0 * t * Tq[-1] - Tq[-2])
    quad = np.array([np.sum(tau ** 2 * x) for x in Tq])
    return float(np.max(np.abs(quad - mom)))


def full_run_errors(ub_fn, N=30, seed=41):
    """k = N: Ritz values = eig(H), tau_i^2 = (u_i^T v)^2."""
    g = np.random.default_rng(seed)
    A = g.standard_normal((N, N))
    H = 0.5 * (A + A.T) / np.sqrt(N) + 3.0 * np.eye(N)   # spectrum inside [1, 5]
    v0 = g.standard_normal(N)
    _, theta, tau = ub_fn(oracle.DenseOperator(H), v0, N)
    lam, U = np.linalg.eigh(H)
    w = (U.T @ (v0 / np.linalg.norm(v0))) ** 2
    return float(np.max(np.abs(theta - lam))), float(np.max(np.abs(tau ** 2 - w)))


def cold_bound_case(cold_fn, ub_fn):
    """H = U diag(lam) U^T with a start vector whose squared components along
    the eigenvectors are w_i = (i+1)/S (S = N(N+1)/2).  A full run gives
    tau_i^2 = w_i, so the first-cycle rule must return a = lam_{j*}, j* the
    smallest j with (j+1)(j+2)/2 >= ns/N * S (exact rationals), and a0 = lam_0.
    Returns |a - expected| + |a0 - lam_0| summed over several ns."""
    N = 40
    g = np.random.default_rng(17)
    lam = np.sort(g.uniform(-1.0, 4.0, N))
    U, _ = np.linalg.qr(g.standard_normal((N, N)))
    H = (U * lam[None, :]) @ U.T
    H = 0.5 * (H + H.T)
    S = N * (N + 1) // 2
    v0 = U @ np.sqrt(np.arange(1, N + 1) / S)
    b, theta, tau = ub_fn(oracle.DenseOperator(H), v0, N)
    err = 0.0
    for ns in (1, 3, 7, 10, 19, 25, 33):
        target = Fraction(ns, N) * S
        jstar = next(j for j in range(N) if Fraction((j + 1) * (j + 2), 2) >= target)
        # keep away from exact ties, where rounding could pick either side
        assert Fraction((jstar + 1) * (jstar + 2), 2) != target
        a, b2, a0 = cold_fn(b, theta, tau, ns, N)
        err += abs(a - lam[jstar]) + abs(a0 - lam[0]) + abs(b2 - b)
    return err


# ------------------------------------------------------------------ tests
@pytest.mark.parametrize("k", [8, 12, 20])
@pytest.mark.parametrize("which", ["tiny", "mixed"])
def test_lanczos_tridiagonal_equals_krylov_qr(which, k):
    H, v0 = tiny_h() if which == "tiny" else mixed_h()
    assert tridiagonal_error(core.lanczos, H, v0, k) <= 1e-12


@pytest.mark.parametrize("k", [8, 20])
def test_upper_bound_is_top_ritz_value_plus_last_beta(k):
    H, v0 = tiny_h()
    assert upper_bound_error(core.lanczos_upper_bound, H, v0, k) <= 1e-12


@pytest.mark.parametrize("k", [5, 12, 20])
@pytest.mark.parametrize("which", ["tiny", "mixed"])
def test_quadrature_weights_integrate_moments_exactly(which, k):
    H, v0 = tiny_h() if which == "tiny" else mixed_h()
    assert quadrature_error(core.lanczos_upper_bound, H, v0, k) <= 1e-12


def test_full_run_reproduces_spectrum_and_weights():
    e_theta, e_tau = full_run_errors(core.lanczos_upper_bound)
    assert e_theta <= 1e-12 and e_tau <= 1e-12, (e_theta, e_tau)


def test_cold_bounds_pick_the_known_eigenvalue():
    assert cold_bound_case(core.bounds_cold, core.lanczos_upper_bound) <= 1e-11


# ------------------------------------------------------------ planted slips
def _ub_variant(mutation):
    def f(op, v0, k):
        alpha, beta = core.lanczos(op, v0, k)
        j = len(alpha)
        T = np.diag(alpha)
        if j > 1 and mutation != "no_offdiag":
            T += np.diag(beta[:j - 1], 1) + np.diag(beta[:j - 1], -1)
        theta, S = core.jacobi_eigh(T)
        bj = beta[j - 2] if (mutation == "beta_prev" and j > 1) else beta[j - 1]
        tau = S[:, 0].copy() if mutation == "tau_axis" else S[0, :].copy()
        return float(theta[-1] + bj), theta, tau
    return f


def _cold_tau_not_squared(b, theta, tau, ns, N):
    w = np.cumsum(np.abs(tau))
    j = min(int(np.searchsorted(w, ns / float(N), side="left")), len(theta) - 1)
    a = float(theta[j])
    return a, b, core._separate(a, float(theta[0]), b)


def test_planted_lanczos_slips_fail():
    H, v0 = tiny_h()
    ref = _ub_variant("none")
    assert upper_bound_error(ref, H, v0, 20) <= 1e-12
    assert quadrature_error(ref, H, v0, 20) <= 1e-12
    # weights from the first eigenvector instead of the first components
    assert quadrature_error(_ub_variant("tau_axis"), H, v0, 20) > 1e-3
    assert full_run_errors(_ub_variant("tau_axis"))[1] > 1e-3
    assert cold_bound_case(core.bounds_cold, _ub_variant("tau_axis")) > 1e-3
    # beta_{k-1} in place of beta_k in the bound
    assert upper_bound_error(_ub_variant("beta_prev"), H, v0, 20) > 1e-3
    # T_k without its off-diagonal
    assert upper_bound_error(_ub_variant("no_offdiag"), H, v0, 20) > 1e-3
    assert quadrature_error(_ub_variant("no_offdiag"), H, v0, 20) > 1e-3
    # cumulative weight of tau instead of tau^2
    assert cold_bound_case(_cold_tau_not_squared, core.lanczos_upper_bound) > 1e-3
