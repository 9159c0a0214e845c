"""Pins of the 2D Poisson kernel (U = -(1/2pi) log|x|, U^ = 1/|k|^2) in the
oracle: the finite-part radial rule with its node at k = 0, against the
closed-form potential of Gaussians (the shell theorem), in Algorithm 1 and
Algorithm 2.  CPU only."""
import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import closed_forms as cf
from oracle import split
from oracle.quadrature import radial_rule
from oracle.symbols import EULER_GAMMA, origin_coefficient


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("K,n_r", [(3.0, 6), (12.5, 20), (0.7, 4)])
def test_finite_part_rule_is_exact_for_polynomials(K, n_r):
    """sum (w/r) g(r) + g(0) (log K - sum w/r) = int_0^K (g - g(0))/r dr + g(0) log K
    for polynomial g of degree 2 n_r."""
    rng = np.random.default_rng(n_r)
    coef = rng.standard_normal(2 * n_r + 1)               # g(r) = sum_j coef_j r^j
    r, w = radial_rule(K, n_r)
    g = np.polynomial.polynomial.polyval(r, coef)
    rule = float(np.sum(w / r * g)) + coef[0] * (np.log(K) - float(np.sum(w / r)))
    exact = sum(coef[j] * K ** j / j for j in range(1, len(coef))) + coef[0] * np.log(K)
    assert rule == pytest.approx(exact, rel=1e-12, abs=1e-12)
    # the origin coefficient is that weight plus the log kernel's constant, over 2 pi
    c0 = origin_coefficient(wl.POISSON_2D, K, n_r)
    assert c0 == pytest.approx((np.log(K) - np.sum(w / r) + EULER_GAMMA - np.log(2.0)) / (2 * np.pi), rel=1e-15)
    assert origin_coefficient(wl.COULOMB_2D, K, n_r) == 0.0


def test_closed_form_value_at_origin():
    # u(0) = -(1/2pi) int log|y| exp(-|y|^2) dy = gamma / 4
    assert cf.poisson2d_gaussian(np.array([0.0]), 1.0)[0] == pytest.approx(EULER_GAMMA / 4, rel=1e-15)
    r = np.array([1e-4])
    assert cf.poisson2d_gaussian(r, 1.3)[0] == pytest.approx(cf.poisson2d_gaussian(np.array([0.0]), 1.3)[0], abs=1e-7)


def test_gaussian_algorithm1():
    n, box, a = (64, 64), (16.0, 16.0), 1.2
    X = wl.mesh(n, box)
    r = np.sqrt(X[0] ** 2 + X[1] ** 2)
    rho = np.exp(-r ** 2 / a)
    res = oracle.evaluate(wl.Problem("p", 2, n, box, wl.POISSON_2D, 64, 1, 96), rho)
    assert rel(res.u, cf.poisson2d_gaussian(r, a)) < 1e-12
    assert abs(res.energy_physical / res.energy_fourier - 1) < 1e-13
    # without the node at k = 0 the potential is off by a constant of order one
    c0 = origin_coefficient(wl.POISSON_2D, np.pi / 0.25, 64)
    assert rel(res.u - c0 * (16 / 64) ** 2 * rho.sum(), cf.poisson2d_gaussian(r, a)) > 1e-2


def test_shifted_mixture_algorithm1():
    rng = np.random.default_rng(4)
    n, box = (64, 64), (16.0, 16.0)
    mix = wl.random_mixture(rng, 3, 2, -2.0, 2.0, 0.8, 1.3)
    rho = mix.evaluate(n, box)
    res = oracle.evaluate(wl.Problem("p", 2, n, box, wl.POISSON_2D, 96, 1, 128), rho)
    assert rel(res.u, cf.mixture_potential(mix, wl.mesh(n, box), 2, poisson=True)) < 1e-10


def test_gaussian_algorithm2():
    n, box, a = (64, 64), (16.0, 16.0), 1.2
    X = wl.mesh(n, box)
    r = np.sqrt(X[0] ** 2 + X[1] ** 2)
    rho = np.exp(-r ** 2 / a)
    q = wl.Problem("p", 2, n, box, wl.POISSON_2D, 48, 1, 64)
    u, i1, i2, E = split.potential_split(q, rho)
    assert rel(u, cf.poisson2d_gaussian(r, a)) < 1e-9
    assert abs(E / split.energy_split_fourier(q, rho) - 1) < 1e-13
