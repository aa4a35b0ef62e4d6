"""Pins of the oracle's post-cycle steps against facts that do not come from
the oracle itself: Fermi-Dirac closed forms and symmetries, a library root
finder, the completeness relation and the trace identity of the density
matrix, the paper's whole-matrix form of the basis re-alignment, least
squares (the l2 projection the paper names) and closed forms for a rotated
basis.  Each check is chosen so that a plausible slip (sign, scale, offset,
transposed operand, squared weight) fails."""
import math

import numpy as np
import pytest
from scipy import optimize, special

import oracle
import synth

KT = synth.KT_300K


def spectrum(ns, seed=3, lo=-0.8, hi=-0.2):
    g = np.random.default_rng(seed)
    return np.sort(g.uniform(lo, hi, size=ns))


# ------------------------------------------------------------ Fermi-Dirac
def fermi_closed_forms_hold(fd):
    """f(mu) = 1/2, f(mu + kT ln 3) = 1/4, f(mu - kT ln 3) = 3/4,
    f(mu - x) + f(mu + x) = 1, and the far tails are exactly 0 and 1."""
    mu = -0.37
    f = fd(np.array([mu, mu + KT * math.log(3.0), mu - KT * math.log(3.0)]), mu, KT)
    ok = abs(f[0] - 0.5) <= 1e-16
    # (theta - mu) loses ~ulp(mu)/kT relative accuracy in the subtraction
    ok &= abs(f[1] - 0.25) <= 1e-13 and abs(f[2] - 0.75) <= 1e-13
    x = np.linspace(-30, 30, 121) * KT
    ok &= np.max(np.abs(fd(mu + x, mu, KT) + fd(mu - x, mu, KT) - 1.0)) <= 1e-15
    tail = fd(np.array([mu + 800 * KT, mu - 800 * KT]), mu, KT)
    return bool(ok and tail[0] == 0.0 and tail[1] == 1.0)


def test_fermi_dirac_closed_forms():
    assert fermi_closed_forms_hold(oracle.fermi_dirac)


def test_planted_fermi_mistakes_fail():
    """The same checks reject a flipped exponent sign and T used for kT."""
    def flipped(theta, mu, kT):
        return oracle.fermi_dirac(2 * mu - np.asarray(theta), mu, kT)

    def kelvin(theta, mu, kT):
        return oracle.fermi_dirac(theta, mu, 300.0)
    assert not fermi_closed_forms_hold(flipped)
    assert not fermi_closed_forms_hold(kelvin)


def test_fermi_level_matches_library_root_finder():
    """mu from the oracle's bisection equals scipy's Brent root of
    sum_i expit((mu - theta_i)/kT) = n_occ (library logistic function)."""
    for ns, seed in ((48, 1), (512, 2), (4096, 3)):
        th = spectrum(ns, seed)
        n_occ = synth.occupied_count(ns)
        mu, f = oracle.occupations(th, n_occ, KT)
        g = lambda m: float(np.sum(special.expit((m - th) / KT))) - n_occ  # noqa: E731
        mu_ref = optimize.brentq(g, th.min() - 60 * KT, th.max() + 60 * KT, xtol=1e-16, rtol=1e-15, maxiter=500)
        assert abs(mu - mu_ref) <= 1e-14 * max(1.0, abs(mu_ref))
        assert abs(np.sum(f) - n_occ) <= 1e-10
        assert np.all((f >= 0) & (f <= 1)) and np.all(np.diff(f) <= 0)


def test_fermi_level_particle_hole_symmetry():
    """A spectrum symmetric about c, half filled, has mu = c."""
    c = -0.41
    half = spectrum(300, 5, 0.0, 0.3)
    th = np.sort(np.concatenate([c - half, c + half]))
    mu, f = oracle.occupations(th, 300.0, KT)
    assert abs(mu - c) <= 1e-14
    assert np.max(np.abs(f + f[::-1] - 1.0)) <= 1e-12


def test_fermi_level_degenerate_closed_form():
    """ns equal levels theta0 and n_occ electrons pairs: ns f(theta0) = n_occ,
    so mu = theta0 + kT ln(n_occ / (ns - n_occ))."""
    th0 = 0.123
    for ns, n in ((4, 1.0), (10, 7.5), (64, 32.0)):
        mu = oracle.fermi_level(np.full(ns, th0), n, KT)
        assert abs(mu - (th0 + KT * math.log(n / (ns - n)))) <= 1e-14


def test_fermi_level_gapped_low_temperature_limit():
    """With a gap of 1000 kT after the n-th level, the lowest n levels are
    fully occupied, the rest empty, and mu lies in the gap."""
    n, ns = 20, 32
    th = np.concatenate([spectrum(n, 7, -1.0, -0.9), spectrum(ns - n, 8, -0.9 + 1000 * KT, 0.5)])
    mu, f = oracle.occupations(th, float(n), KT)
    assert th[n - 1] < mu < th[n]
    assert np.max(np.abs(f[:n] - 1.0)) <= 1e-12 and np.max(f[n:]) <= 1e-12


def test_fermi_level_monotone_and_argument_checks():
    th = spectrum(100, 9)
    mus = [oracle.fermi_level(th, n, KT) for n in (10.0, 40.0, 40.5, 90.0)]
    assert all(a < b for a, b in zip(mus, mus[1:]))
    for bad in (0.0, 100.0, -1.0):
        with pytest.raises(ValueError):
            oracle.fermi_level(th, bad, KT)
    with pytest.raises(ValueError):
        oracle.fermi_level(th, 10.0, 0.0)


# ------------------------------------------------------ density-matrix blocks
def orthonormal_block(N, ns, seed):
    g = np.random.default_rng(seed)
    q, _ = np.linalg.qr(g.standard_normal((N, ns)))
    return q


def test_density_blocks_brute_force_sum_over_states():
    """P_{K;K}[j, j'] = sum_i f_i x_i[K, j] x_i[K, j'] accumulated state by
    state (outer products), on uneven element sizes."""
    J = np.array([3, 7, 5, 1, 4])
    N, ns = int(J.sum()), 9
    g = np.random.default_rng(11)
    X = g.standard_normal((N, ns))
    f = g.uniform(0, 1, ns)
    blocks = oracle.density_diag_blocks(J, X, f)
    off = np.concatenate([[0], np.cumsum(J)])
    for K in range(len(J)):
        ref = np.zeros((J[K], J[K]))
        for i in range(ns):
            xi = X[off[K]:off[K + 1], i]
            ref += f[i] * np.outer(xi, xi)
        assert np.max(np.abs(blocks[K] - ref)) <= 1e-14
    P = oracle.density_dense(X, f)
    for K in range(len(J)):
        assert np.max(np.abs(blocks[K] - P[off[K]:off[K + 1], off[K]:off[K + 1]])) <= 1e-14


def test_density_blocks_trace_identity_and_bounds():
    """For orthonormal Ritz vectors, sum_K tr P_{K;K} = sum_i f_i = n_occ,
    and each block is symmetric with eigenvalues in [0, 1]."""
    J = np.full(8, 16)
    N, ns = 128, 48
    X = orthonormal_block(N, ns, 12)
    th = spectrum(ns, 13)
    n_occ = synth.occupied_count(ns)
    mu, f = oracle.occupations(th, n_occ, KT)
    blocks = oracle.density_diag_blocks(J, X, f)
    assert abs(sum(np.trace(b) for b in blocks) - n_occ) <= 1e-10
    for b in blocks:
        assert np.array_equal(b, b.T) or np.max(np.abs(b - b.T)) <= 1e-16
        w = np.linalg.eigvalsh(b)
        assert w.min() >= -1e-14 and w.max() <= 1 + 1e-14
    # planted: squared occupations break the trace identity
    sq = oracle.density_diag_blocks(J, X, f * f)
    assert abs(sum(np.trace(b) for b in sq) - n_occ) > 1e-3


def test_density_blocks_completeness():
    """All states fully occupied in a complete orthonormal basis (ns = N):
    X X^T = I, so every diagonal block is the identity."""
    J = np.array([5, 3, 8])
    N = int(J.sum())
    X = orthonormal_block(N, N, 14)
    for b, n in zip(oracle.density_diag_blocks(J, X, np.ones(N)), J):
        assert np.max(np.abs(b - np.eye(n))) <= 1e-14


# ------------------------------------------------------------- re-alignment
def test_alb_samples_orthonormal_and_reproducible():
    J = np.array([16, 24, 8, 32])
    nr = 40
    V = synth.make_alb_samples(J, nr)
    assert np.array_equal(V, synth.make_alb_samples(J, nr))
    Vn = synth.make_next_alb_samples(J, V, nr)
    for K in range(len(J)):
        for W in (V, Vn):
            VK = oracle.element_samples(J, nr, W, K)
            assert VK.shape == (nr, J[K])
            assert np.max(np.abs(VK.T @ VK - np.eye(J[K]))) <= 1e-14
        # close to, but not inside, the old span
        A = oracle.element_samples(J, nr, V, K)
        B = oracle.element_samples(J, nr, Vn, K)
        s = np.linalg.svd(A.T @ B, compute_uv=False)
        assert 0.9 < s.min() < 1 - 1e-6


def test_realign_element_form_equals_whole_matrix_form():
    """eq. basis_rotation_3 (element by element) equals eq. basis_rotation_1
    with the whole N_r x N_b sample matrices (disjoint supports)."""
    J = np.array([6, 9, 4, 7, 5, 8])
    nr, ns = 12, 10
    V = synth.make_alb_samples(J, nr)
    Vn = synth.make_next_alb_samples(J, V, nr)
    X = np.random.default_rng(15).standard_normal((int(J.sum()), ns))
    a = oracle.realign(J, nr, Vn, V, X)
    b = oracle.realign_dense(J, nr, Vn, V, X)
    assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(b))


def test_realign_is_the_l2_projection():
    """X_new_K is the least-squares solution of V_new_K Z = V_old_K X_K
    (numpy lstsq), i.e. the residual is orthogonal to the new span."""
    J = np.array([8, 16, 12])
    nr, ns = 30, 7
    V = synth.make_alb_samples(J, nr)
    Vn = synth.make_next_alb_samples(J, V, nr, delta=0.3)
    X = np.random.default_rng(16).standard_normal((int(J.sum()), ns))
    Xn = oracle.realign(J, nr, Vn, V, X)
    off = np.concatenate([[0], np.cumsum(J)])
    for K in range(len(J)):
        A = oracle.element_samples(J, nr, Vn, K)
        B = oracle.element_samples(J, nr, V, K) @ X[off[K]:off[K + 1]]
        Z = np.linalg.lstsq(A, B, rcond=None)[0]
        assert np.max(np.abs(Xn[off[K]:off[K + 1]] - Z)) <= 1e-13


def test_realign_same_and_rotated_basis():
    """Unchanged basis: X is unchanged.  A basis rotated inside its span,
    V_new_K = V_old_K G_K with G_K orthogonal: X_new_K = G_K^T X_K (a
    transposed overlap would give G_K X_K and fail)."""
    J = np.array([10, 6, 14])
    nr, ns = 20, 5
    V = synth.make_alb_samples(J, nr)
    X = np.random.default_rng(17).standard_normal((int(J.sum()), ns))
    assert np.max(np.abs(oracle.realign(J, nr, V, V, X) - X)) <= 1e-14
    off = np.concatenate([[0], np.cumsum(J)])
    g = np.random.default_rng(18)
    parts, Gs = [], []
    for K in range(len(J)):
        G = synth.haar_orthogonal(int(J[K]), g)
        Gs.append(G)
        parts.append((oracle.element_samples(J, nr, V, K) @ G).T.ravel())
    Vr = np.concatenate(parts)
    Xn = oracle.realign(J, nr, Vr, V, X)
    for K in range(len(J)):
        assert np.max(np.abs(Xn[off[K]:off[K + 1]] - Gs[K].T @ X[off[K]:off[K + 1]])) <= 1e-14
        assert np.max(np.abs(Gs[K] @ X[off[K]:off[K + 1]] - Xn[off[K]:off[K + 1]])) > 1e-3
