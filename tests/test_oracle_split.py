"""Pins of the Algorithm 2 oracle (Section 3.3, eqs. 3.9, 3.10, 3.12).  CPU only.

  * the FFT form of I1 against the same trapezoid sum evaluated directly
    (padding, frequency order and normalisation);
  * the windows: p + (1 - p) = 1 without cancellation, their values at the ends
    of the transition, and the k = 0 limit of the split symbol;
  * closed forms: the Coulomb potential and energy of a 3D Gaussian, a 2D
    Gaussian mixture (eq. 4.2), Example 4 (Coulomb) and Example 5 (dipole);
  * invariance: u does not depend on where the window splits the integral,
    while I1 and I2 individually do;
  * agreement with Algorithm 1 at a node set that resolves the full integral;
  * the Fourier-side energy equals the physical-side one.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import closed_forms as cf
from oracle import split

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _examples():
    return json.load(open(os.path.join(GOLDEN, "examples.json")))


# ------------------------------------------------------------- FFT form of I1

@pytest.mark.parametrize("kernel,shape,box", [
    (wl.COULOMB_3D, (6, 5, 4), (5.0, 4.0, 3.5)),
    (wl.DIPOLE_3D, (5, 6, 4), (4.0, 5.0, 3.0)),
    (wl.COULOMB_2D, (7, 6), (4.0, 3.0)),
    (wl.COULOMB_2D, (5, 8), (3.0, 5.0)),
])
def test_i1_fft_equals_direct_trapezoid_sum(kernel, shape, box):
    rng = np.random.default_rng(21)
    rho = rng.standard_normal(shape)
    axis = tuple(wl.unit_vector(rng)) if kernel == wl.DIPOLE_3D else None
    # scales chosen so that 1 - p is far from zero on these coarse frequency grids
    par = {"a": 1.5} if len(shape) == 3 else {"R0": 0.3, "R1": 2.0}
    a = split.i1_fft(rho, box, kernel, par, axis)
    b = split.i1_direct(rho, box, kernel, par, axis)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))


def test_grid_frequencies_order_and_spacing():
    (k,) = split.grid_frequencies((5,), (3.0,))
    dk = 2 * np.pi / (2 * 3.0)
    q = np.array([0, 1, 2, 3, 4, -5, -4, -3, -2, -1])
    assert np.allclose(k, q * dk, rtol=0, atol=1e-15)


# ------------------------------------------------------------- windows

def test_windows_partition_and_transition():
    k = np.linspace(0, 12, 1001)
    for d, par in [(3, {"a": 0.7}), (2, {"R0": 0.5, "R1": 6.0})]:
        p = split.window(k, d, par)
        q = split.one_minus_window(k, d, par)
        assert np.max(np.abs(p + q - 1)) < 2e-16
        assert np.all(np.diff(p) <= 0)
    # eq. 3.10: p3(0) = 1 and p3 = 1/e at |k|^2 = a
    assert split.window(np.array([0.0, np.sqrt(0.7)]), 3, {"a": 0.7})[1] == pytest.approx(np.exp(-1), abs=1e-15)
    assert split.window(np.array([0.0]), 3, {"a": 0.7})[0] == 1.0
    # eq. 3.12: 1/2 at the midpoint, erfc(6)/2 at R0 and R1 (one minus it at R0)
    par = {"R0": 0.5, "R1": 6.0}
    p = split.window(np.array([0.5, 3.25, 6.0]), 2, par)
    assert p[1] == pytest.approx(0.5, abs=1e-16)
    assert p[2] == pytest.approx(1.0759868356249e-17, rel=1e-12)    # erfc(6) / 2
    assert 1 - p[0] == pytest.approx(p[2], rel=1e-2)


def test_split_symbol_limits():
    # 3D Coulomb: (1 - exp(-k^2/a)) / k^2 -> 1/a; the k = 0 value is that limit
    a = 0.9
    k = np.array([[0.0, 0.0, 0.0], [1e-4, 0.0, 0.0], [0.0, 3e-5, 4e-5]])
    M = split.split_symbol(wl.COULOMB_3D, k, {"a": a})
    assert M[0] == 1.0 / a
    assert np.allclose(M[1:], 1.0 / a, rtol=1e-7, atol=0)
    # large |k|: the window is gone, M is the plain symbol 1/|k|^2
    kk = np.array([[30.0, 0.0, 0.0]])
    assert split.split_symbol(wl.COULOMB_3D, kk, {"a": a})[0] == pytest.approx(1 / 900.0, rel=1e-15)
    # dipole: 1 - p vanishes at 0 and the symbol stays bounded
    M = split.split_symbol(wl.DIPOLE_3D, k, {"a": a}, (0.0, 0.0, 1.0))
    assert M[0] == 0.0 and np.all(np.abs(M[1:]) < 1e-7)
    # 2D: at the default scales 1 - p2 is below 1e-20 at k = 0 and (1 - p2)/|k|
    # below 1e-18 at the first grid frequency of any grid, so setting the k = 0
    # value to 0 drops nothing an FP64 sum would keep
    n, box = (64, 48), (20.0, 16.0)
    par = split.default_window(n, box)
    k1 = 2 * np.pi / (2 * max(box))
    assert split.one_minus_window(np.array([0.0]), 2, par)[0] < 1e-20
    assert split.one_minus_window(np.array([k1]), 2, par)[0] / k1 < 1e-18


def test_default_scales_follow_box_not_grid():
    a1 = split.default_window((32, 32, 32), (16.0, 16.0, 16.0))["a"]
    a2 = split.default_window((128, 128, 128), (16.0, 16.0, 16.0))["a"]
    assert a1 == a2 == pytest.approx(2 * (2 * np.pi / 16) ** 2, rel=1e-15)
    par = split.default_window((256, 256), (32.0, 24.0))
    assert par["R0"] == pytest.approx(0.8 * 2 * np.pi / 32) and par["R1"] == pytest.approx(10 * 2 * np.pi / 32)
    # the cut-off: sqrt(40 a) unless the grid's Nyquist radius is smaller
    assert split.default_cutoff((32,) * 3, (16.0,) * 3, {"a": a1}) == pytest.approx(np.sqrt(40 * a1))
    assert split.default_cutoff((8,) * 3, (16.0,) * 3, {"a": a1}) == pytest.approx(np.pi / 2)


# ------------------------------------------------------------- closed forms

def test_coulomb3d_gaussian_closed_form():
    p, rho = wl.coulomb3d_32()
    q = wl.Problem("s3", 3, p.n, p.box, wl.COULOMB_3D, 24, 24, 24)
    u, i1, i2, E = split.potential_split(q, rho)
    X = wl.mesh(p.n, p.box)
    r = np.sqrt(sum(Xi ** 2 for Xi in X))
    assert rel(u, cf.coulomb3d_gaussian(r, 1.0)) < 1e-7
    assert abs(E / cf.coulomb3d_gaussian_energy(1.0) - 1) < 2e-9
    # both parts carry weight: neither alone is the potential
    assert rel(i1, u) > 1e-2 and rel(i2, u) > 1e-2


def test_coulomb2d_mixture_closed_form():
    p, rho, mix = wl.coulomb2d_256()
    q = wl.Problem("s2", 2, p.n, p.box, wl.COULOMB_2D, 60, 1, 60)
    u, i1, i2, E = split.potential_split(q, rho)
    X = wl.mesh(p.n, p.box)
    assert rel(u, cf.mixture_potential(mix, X, 2)) < 2e-8
    assert abs(E / cf.mixture_energy(mix, 2) - 1) < 1e-11


def test_example4_coulomb_closed_form():
    a = _examples()["example4"]["a"]
    n, box = (32, 32, 32), (12.0, 12.0, 12.0)
    q = wl.Problem("s4", 3, n, box, wl.COULOMB_3D, 32, 32, 32)
    u, _, _, _ = split.potential_split(q, wl.log_density(n, box, a))
    assert rel(u, cf.example4_potential(wl.mesh(n, box), a)) < 1e-7


def test_example5_dipole_closed_form():
    ex = _examples()["example5"]
    a, nv = ex["a"], np.array(ex["n"])
    nv = nv / np.linalg.norm(nv)
    n, box = (32, 32, 32), (12.0, 12.0, 12.0)
    q = wl.Problem("s5", 3, n, box, wl.DIPOLE_3D, 32, 32, 32, axis=tuple(nv))
    rho = wl.log_density(n, box, a)
    u, _, _, _ = split.potential_split(q, rho)
    ut = cf.example5_potential(wl.mesh(n, box), a, nv)
    assert rel(u, ut) < 2e-8
    # the opposite axis gives the same potential (the symbol is even in n); a
    # different axis does not
    u2, _, _, _ = split.potential_split(wl.Problem("s5", 3, n, box, wl.DIPOLE_3D, 32, 32, 32,
                                                   axis=tuple(-nv)), rho)
    assert rel(u2, u) < 1e-13
    u3, _, _, _ = split.potential_split(wl.Problem("s5", 3, n, box, wl.DIPOLE_3D, 32, 32, 32,
                                                   axis=(0.0, 0.0, 1.0)), rho)
    assert rel(u3, u) > 1e-2


@pytest.mark.parametrize("kernel,shape,box", [
    (wl.COULOMB_3D, (12, 10, 8), (6.0, 5.0, 4.0)),
    (wl.DIPOLE_3D, (10, 12, 8), (5.0, 6.0, 4.0)),
    (wl.COULOMB_2D, (24, 20), (8.0, 6.0)),
])
def test_fourier_side_energy_equals_physical_side(kernel, shape, box):
    """Substituting eq. 3.2 into H sum rho u gives the Fourier form exactly."""
    rng = np.random.default_rng(29)
    mix = wl.random_mixture(rng, 3, len(shape), -1.0, 1.0, 0.6, 0.9)
    rho = mix.evaluate(shape, box)
    axis = tuple(wl.unit_vector(rng)) if kernel == wl.DIPOLE_3D else (0.0, 0.0, 1.0)
    q = wl.Problem("ef", len(shape), shape, box, kernel, 10, 8, 12, axis=axis, lam=1.7)
    _, _, _, E = split.potential_split(q, rho)
    Ef = split.energy_split_fourier(q, rho)
    assert abs(Ef - E) < 1e-13 * abs(E)


# ------------------------------------------------------------- invariance

@pytest.mark.parametrize("dim", [2, 3])
def test_potential_independent_of_window_scale(dim):
    """Moving the window moves weight between I1 and I2 but leaves u unchanged."""
    if dim == 3:
        n, box = (24, 24, 24), (12.0, 12.0, 12.0)
        rho = wl.gaussian(n, box, a=1.0)
        kern = wl.COULOMB_3D
        base = split.default_window(n, box)
        alt = {"a": 2.0 * base["a"]}
    else:
        n, box = (64, 64), (16.0, 16.0)
        rho = wl.gaussian(n, box, a=1.0)
        kern = wl.COULOMB_2D
        base = split.default_window(n, box)
        alt = {"R0": 1.5 * base["R0"], "R1": 1.5 * base["R1"]}
    out = []
    for par in (base, alt):
        q = wl.Problem("inv", dim, n, box, kern, 48 if dim == 3 else 64, 48 if dim == 3 else 1, 48 if dim == 3 else 96,
                       kmax=split.default_cutoff(n, box, par))
        out.append(split.potential_split(q, rho, par))
    (u1, a1, b1, _), (u2, a2, b2, _) = out
    assert rel(u2, u1) < 1e-8
    assert rel(a2, a1) > 1e-3 and rel(b2, b1) > 1e-3


def test_agrees_with_algorithm1_at_resolving_nodes():
    """A density resolved by the grid (rho^ below 1e-10 at pi / h) and small at the
    box edges, so that Algorithm 1's ball and I1's cube of frequencies see the
    same integrand."""
    rng = np.random.default_rng(23)
    n, box = (28, 28, 28), (11.2, 11.2, 11.2)
    mix = wl.random_mixture(rng, 3, 3, -0.6, 0.6, 1.2, 1.3)
    rho = mix.evaluate(n, box)
    axis = tuple(wl.unit_vector(rng))
    ref = oracle.evaluate(wl.Problem("a1", 3, n, box, wl.DIPOLE_3D, 80, 40, 80, axis=axis), rho)
    u, _, _, E = split.potential_split(wl.Problem("a2", 3, n, box, wl.DIPOLE_3D, 32, 32, 32, axis=axis), rho)
    assert rel(u, ref.u) < 1e-6
    assert abs(E - ref.energy_physical) < 1e-12 * abs(ref.energy_physical)
