"""Pins of the oracle's generalized Gaussian radial rule (oracle/ggq.py;
Section 3.3's last remark, the Conclusions), each against something other
than the construction itself:

  * the prolate functions it builds are eigenfunctions of the band-limited
    Fourier operator, int e^{icxt} psi(t) dt = lambda psi(x) (a dropped or
    mistyped term of the tridiagonal matrix breaks this);
  * the radial rule takes the finite-part integrals of the 2D Poisson kernel,
    int_0^1 (cos(s t) - 1)/t dt = Ci(s) - gamma - log s and
    int_0^1 sin(s t)/t dt = Si(s), to eps over the bandwidth it is built for;
  * at vanishing bandwidth it is Gauss-Legendre; its nodes are symmetric and
    its weights positive;
  * on the 2D Poisson kernel of a Gaussian mixture it reaches the closed-form
    potential with fewer radial nodes than the Gauss-Legendre rule with its
    subtracted node at the origin."""
import numpy as np
import pytest
from numpy.polynomial import legendre as leg
from scipy.special import sici

import workloads as wl
from oracle import closed_forms as cf
from oracle.ggq import bandwidth, prolate_coefficients, prolate_eval, prolate_rule
from oracle.symbols import EULER_GAMMA


@pytest.mark.parametrize("c", [5.0, 20.0, 60.0])
def test_prolate_functions_are_eigenfunctions(c):
    cs = prolate_coefficients(c, 12)
    t, wt = leg.leggauss(400)
    x = np.linspace(-0.9, 0.9, 13)
    for n in (0, 1, 4, 7, 11):
        psi_t = prolate_eval(cs[n], t)
        F = np.exp(1j * c * np.outer(x, t)) @ (wt * psi_t)
        psi_x = prolate_eval(cs[n], x)
        j = int(np.argmax(np.abs(psi_x)))
        lam = F[j] / psi_x[j]
        # one eigenvalue for every x (psi has unit norm, so the residual is
        # absolute), real or imaginary by the parity of n
        assert np.max(np.abs(F - lam * psi_x)) < 1e-12
        assert abs((lam * (1j) ** (-n)).imag) < 1e-12


@pytest.mark.parametrize("eps", [1e-5, 1e-10])
@pytest.mark.parametrize("n", [24, 48, 96])
def test_rule_takes_the_finite_part_integrals(n, eps):
    c = bandwidth(n, eps)
    assert c > 1.0
    x, w = prolate_rule(c, n)
    t, v = 0.5 * (1.0 + x), 0.5 * w        # the rule on [0, 1]
    s = np.linspace(0.05, 4.0 * c, 300)    # e^{i s t} on [0, 1] is bandwidth s / 2 on [-1, 1]
    si, ci = sici(s)
    fp_cos = ((np.cos(np.outer(s, t)) - 1.0) / t) @ v
    fp_sin = (np.sin(np.outer(s, t)) / t) @ v
    err = max(np.max(np.abs(fp_cos - (ci - EULER_GAMMA - np.log(s)))), np.max(np.abs(fp_sin - si)))
    assert err < eps


@pytest.mark.parametrize("eps", [1e-5, 1e-10])
@pytest.mark.parametrize("n", [24, 48, 96, 192])
def test_bandwidth_choice_meets_eps(n, eps):
    c = bandwidth(n, eps)
    x, w = prolate_rule(c, n)
    s = np.linspace(0.0, 2.0 * c, 800)
    exact = np.where(s == 0, 2.0, 2.0 * np.sin(s) / np.where(s == 0, 1.0, s))
    assert np.max(np.abs(np.exp(1j * np.outer(s, x)) @ w - exact)) < eps / 100


def test_small_bandwidth_is_gauss_legendre_and_the_rule_is_symmetric():
    for n in (8, 17, 32):
        x, w = prolate_rule(1e-4, n)
        g, gw = leg.leggauss(n)
        assert np.max(np.abs(x - g)) < 1e-8 and np.max(np.abs(w - gw)) < 1e-8
    x, w = prolate_rule(40.0, 44)
    assert np.max(np.abs(x + x[::-1])) < 1e-14 and np.max(np.abs(w - w[::-1])) < 1e-13
    assert np.all(w > 0) and abs(np.sum(w) - 2.0) < 1e-13
    assert bandwidth(16, 1e-10) == 0.0   # too few nodes for a bandwidth: Gauss-Legendre


def _poisson_error(n_r, radial, eps):
    """Max relative error of the radial rule's u against the closed-form 2D
    Poisson potential of a Gaussian mixture, rho^ taken analytically (only the
    radial rule is tested: 256 trapezoid angles are exact to rounding)."""
    from oracle.quadrature import radial_rule
    p = wl.Problem("p1", 2, (64, 48), (16.0, 12.0), wl.POISSON_2D, n_r, 1, 48)
    mix = wl.random_mixture(np.random.default_rng(12), 3, 2, -1.5, 1.5, 0.8, 1.2)
    K = np.pi / max(b / m for b, m in zip(p.box, p.n))
    X = np.array([(a, b) for a in np.linspace(-8, 8, 9) for b in np.linspace(-6, 6, 7)])
    ref = cf.mixture_potential(mix, (X[:, 0], X[:, 1]), 2, poisson=True)

    def rhohat(k):
        out = np.zeros(len(k), complex)
        for A, c, s in zip(mix.amps, mix.centers, mix.widths):
            a = s * s
            out += A * np.pi * a * np.exp(-a * np.sum(k * k, axis=1) / 4) * np.exp(-1j * (k @ np.asarray(c)))
        return out

    r, w = radial_rule(K, n_r, radial, eps)
    ph = 2 * np.pi * np.arange(256) / 256
    k = np.stack([np.outer(r, np.cos(ph)).ravel(), np.outer(r, np.sin(ph)).ravel()], axis=1)
    W = np.outer(w / r, np.full(256, 2 * np.pi / 256)).ravel()
    r0 = rhohat(np.zeros((1, 2)))[0].real
    u = (np.exp(1j * X @ k.T) @ (W * rhohat(k))).real / (2 * np.pi) ** 2
    u += 2 * np.pi * r0 * (np.log(K) - np.sum(w / r)) / (2 * np.pi) ** 2 + (EULER_GAMMA - np.log(2)) / (2 * np.pi) * r0
    return np.max(np.abs(u - ref)) / np.max(np.abs(ref))


def test_fewer_radial_nodes_for_the_poisson_kernel():
    # float64 accuracy: 44 generalized Gaussian nodes beat 48 Gauss-Legendre nodes
    e_ggq = _poisson_error(44, wl.RADIAL_GGQ, 1e-10)
    e_gl = _poisson_error(48, wl.RADIAL_GL, 1e-10)
    assert e_ggq < 1e-9 < e_gl
    # mixed-precision accuracy: 36 beat 40
    e_ggq = _poisson_error(36, wl.RADIAL_GGQ, 1e-5)
    e_gl = _poisson_error(40, wl.RADIAL_GL, 1e-5)
    assert e_ggq < 5e-6 < e_gl
