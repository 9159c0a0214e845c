"""Pins of the oracle's Fourier-space quadrature (Section 3.1, eqs. 3.5 and 3.7)
against exact integrals.  CPU only."""
import numpy as np
import pytest
from scipy.special import erf, j1

import oracle
from oracle.quadrature import THETA_GL, COSTHETA_GL


@pytest.mark.parametrize("n", [1, 2, 5, 16, 33, 128])
def test_gauss_legendre_moments(n):
    s, w = oracle.gauss_legendre(n)
    for p in range(2 * n):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs(np.sum(w * s ** p) - exact) < 1e-13 * max(1.0, n / 8)


def test_radial_rule_exact_on_polynomials():
    K = 3.7
    r, w = oracle.radial_rule(K, 12)
    assert np.all((r > 0) & (r < K))
    for p in range(24):
        assert abs(np.sum(w * r ** p) - K ** (p + 1) / (p + 1)) < 1e-12 * K ** (p + 1)


@pytest.mark.parametrize("rule", [THETA_GL, COSTHETA_GL])
def test_theta_rules_integrate_sin_measure(rule):
    ct, st, w = oracle.theta_rule(24, rule)
    assert np.allclose(ct ** 2 + st ** 2, 1.0, atol=1e-15)
    assert np.all(st > 0)
    tol = 1e-14 if rule == COSTHETA_GL else 1e-12
    for p in range(12):
        exact = (1.0 + (-1.0) ** p) / (p + 1)        # int_0^pi cos^p sin dtheta
        assert abs(np.sum(w * ct ** p) - exact) < tol


def test_theta_rule_symmetric_under_reflection():
    # theta -> pi - theta maps the rule onto itself: this is what pairs k with -k
    for rule in (THETA_GL, COSTHETA_GL):
        ct, st, w = oracle.theta_rule(17, rule)
        assert np.allclose(ct, -ct[::-1], atol=1e-15)
        assert np.allclose(w, w[::-1], rtol=1e-14)


def test_phi_rule_exact_for_fourier_modes():
    ph, w = oracle.phi_rule(16)
    for m in range(-15, 16):
        exact = 2 * np.pi if m == 0 else 0.0
        assert abs(np.sum(w * np.exp(1j * m * ph)) - exact) < 1e-13


@pytest.mark.parametrize("rule", [THETA_GL, COSTHETA_GL])
def test_spherical_nodes_ball_integrals(rule):
    K = 2.5
    k, W = oracle.spherical_nodes(K, 24, 24, 32, rule)
    r2 = np.sum(k * k, axis=1)
    tol = 1e-13 if rule == COSTHETA_GL else 1e-9
    # volume of the ball: the weights carry dr dtheta dphi (sin theta included), r^2 is the Jacobian
    assert abs(np.sum(W * r2) - 4 * np.pi * K ** 3 / 3) < tol * K ** 3
    # Gaussian over the ball
    exact = np.pi ** 1.5 * erf(K) - 2 * np.pi * K * np.exp(-K * K)
    assert abs(np.sum(W * r2 * np.exp(-r2)) - exact) < tol
    # second moments: every axis gets 4 pi K^5 / 15, mixed ones vanish
    for i in range(3):
        assert abs(np.sum(W * r2 * k[:, i] ** 2) - 4 * np.pi * K ** 5 / 15) < tol * K ** 5
    assert abs(np.sum(W * r2 * k[:, 0] * k[:, 2])) < tol * K ** 5
    # Fourier transform of the ball's indicator at a general vector pins each component's direction
    a = np.array([0.31, -0.52, 0.77])
    A = np.linalg.norm(a)
    exact = 4 * np.pi * (np.sin(K * A) - K * A * np.cos(K * A)) / A ** 3
    got = np.sum(W * r2 * np.exp(1j * (k @ a)))
    assert abs(got - exact) < tol * 10
    # an odd function of a single component integrates to zero only if the signs are right
    got3 = np.sum(W * r2 * k[:, 2] * np.exp(1j * k[:, 2] * 0.9))
    exact3 = 1j * 4 * np.pi * _ball_moment_z(K, 0.9)
    assert abs(got3 - exact3) < tol * 10


def _ball_moment_z(K, b):
    # int_ball k_z sin(b k_z) dk / (4 pi), via the radial form and GL on r
    from numpy.polynomial.legendre import leggauss
    s, w = leggauss(200)
    r = 0.5 * K * (1 + s)
    wr = 0.5 * K * w
    # int_S2 cos(t) sin(b r cos t) dOmega = 4 pi * j1(b r) (spherical Bessel j1)
    x = b * r
    sj1 = np.sin(x) / x ** 2 - np.cos(x) / x
    return float(np.sum(wr * r ** 3 * sj1))


def test_polar_nodes_disk_integrals():
    K = 3.1
    k, W = oracle.polar_nodes(K, 20, 40)
    r = np.sqrt(np.sum(k * k, axis=1))
    assert abs(np.sum(W * r) - np.pi * K * K) < 1e-13
    a = np.array([0.4, -0.9])
    A = np.linalg.norm(a)
    exact = 2 * np.pi * K * j1(K * A) / A
    assert abs(np.sum(W * r * np.exp(1j * (k @ a))) - exact) < 1e-12
    assert abs(np.sum(W * r * k[:, 1] * np.sin(k[:, 1] * 0.7))) > 1e-3   # sin component present
    assert abs(np.sum(W * r * k[:, 0] * np.cos(k[:, 0]))) < 1e-12         # odd integrand


def test_node_set_closed_under_negation():
    # with an even N_phi, (r, pi - theta, phi + pi) is a node: k -> -k, needed for real u
    k, W = oracle.spherical_nodes(1.7, 5, 6, 8, THETA_GL)
    kk = k.reshape(5, 6, 8, 3)
    neg = -kk[:, ::-1, :, :]
    neg = np.roll(neg, -4, axis=2)
    assert np.allclose(kk, neg, atol=1e-14)


def test_dipole_symbol_trace_free_on_sphere():
    # the angular mean of 3 (n.k^)^2 - 1 vanishes: isotropic densities have zero dipole energy
    n = np.array([0.2, -0.5, 0.8])
    n /= np.linalg.norm(n)
    k, W = oracle.spherical_nodes(1.0, 1, 8, 16, COSTHETA_GL)
    S = oracle.symbol(2, k, n)
    assert abs(np.sum(W * S)) < 1e-14
    assert np.allclose(oracle.symbol(0, k), 1.0)
