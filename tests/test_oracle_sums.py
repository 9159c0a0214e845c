"""Pins of the oracle's direct sums (eq. 3.2, eq. 3.7 / Algorithm 1, the energy
remark after Algorithm 2) against brute force, closed forms from the paper's
examples, the printed Example 7 energies and exact invariants.  CPU only."""
import cmath
import json
import os

import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import closed_forms as cf
from oracle.quadrature import THETA_GL, COSTHETA_GL

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


# ------------------------------------------------------------- brute force

def _brute_rho_hat(rho, box, k):
    n = rho.shape
    h = [R / N for N, R in zip(n, box)]
    H = float(np.prod(h))
    out = []
    for kj in k:
        acc = 0j
        for idx in np.ndindex(*n):
            x = [-box[i] / 2 + idx[i] * h[i] for i in range(len(n))]
            acc += rho[idx] * cmath.exp(-1j * sum(kj[i] * x[i] for i in range(len(n))))
        out.append(H * acc)
    return np.array(out)


def _brute_sum(v, k, n, box):
    h = [R / N for N, R in zip(n, box)]
    out = np.zeros(n, dtype=complex)
    for idx in np.ndindex(*n):
        x = [-box[i] / 2 + idx[i] * h[i] for i in range(len(n))]
        out[idx] = sum(vj * cmath.exp(1j * sum(kj[i] * x[i] for i in range(len(n)))) for vj, kj in zip(v, k))
    return out


@pytest.mark.parametrize("shape,box", [((3, 4, 5), (2.0, 3.0, 1.5)), ((6, 5), (4.0, 2.5))])
def test_rho_hat_brute_force(shape, box):
    rng = np.random.default_rng(11)
    rho = rng.standard_normal(shape)
    k = rng.uniform(-2, 2, size=(7, len(shape)))
    assert np.allclose(oracle.rho_hat(rho, box, k), _brute_rho_hat(rho, box, k), rtol=0, atol=1e-13)


@pytest.mark.parametrize("shape,box", [((3, 4, 5), (2.0, 3.0, 1.5)), ((6, 5), (4.0, 2.5))])
def test_sum_to_grid_and_points_brute_force(shape, box):
    rng = np.random.default_rng(12)
    k = rng.uniform(-2, 2, size=(9, len(shape)))
    v = rng.standard_normal(9) + 1j * rng.standard_normal(9)
    ref = _brute_sum(v, k, shape, box)
    assert np.allclose(oracle.sum_to_grid(v, k, shape, box), ref, rtol=0, atol=1e-12)
    idx = np.array([[rng.integers(0, s) for s in shape] for _ in range(10)])
    pts = oracle.sum_to_points(v, k, shape, box, idx)
    assert np.allclose(pts, ref[tuple(idx.T)], rtol=0, atol=1e-12)


def test_separable_rho_hat_equals_general_sum():
    # a separable density's trapezoid sum, by the per-axis regrouping, equals the general sum
    rng = np.random.default_rng(15)
    n, box = (12, 10, 14), (6.0, 5.0, 7.0)
    f = [rng.standard_normal(m) for m in n]
    rho = f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :]
    k = rng.uniform(-3, 3, size=(40, 3))
    a = oracle.rho_hat_separable(f, box, k)
    b = oracle.rho_hat(rho, box, k)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))
    f2 = [rng.standard_normal(m) for m in n[:2]]
    rho2 = f2[0][:, None] * f2[1][None, :]
    k2 = rng.uniform(-3, 3, size=(30, 2))
    assert np.allclose(oracle.rho_hat_separable(f2, box[:2], k2), oracle.rho_hat(rho2, box[:2], k2), rtol=0,
                       atol=1e-12 * np.max(np.abs(rho2)) * np.prod(box[:2]))


def test_lattice_sum_brute_force():
    # the type-1 sum at a product set of grid indices (and at a line) equals brute force there
    rng = np.random.default_rng(13)
    shape, box = (5, 4, 6), (3.0, 2.5, 4.0)
    k = rng.uniform(-2, 2, size=(11, 3))
    v = rng.standard_normal(11) + 1j * rng.standard_normal(11)
    ref = _brute_sum(v, k, shape, box)
    lists = [np.array([4, 0, 2]), np.array([1, 3]), np.array([5, 0, 3, 2])]
    got = oracle.sum_to_lattice(v, k, shape, box, lists)
    assert got.shape == (3, 2, 4)
    assert np.allclose(got, ref[np.ix_(*lists)], rtol=0, atol=1e-12)
    line = oracle.sum_to_lattice(v, k, shape, box, [np.arange(5), [2], [3]])
    assert np.allclose(line[:, 0, 0], ref[:, 2, 3], rtol=0, atol=1e-12)
    got2 = oracle.sum_to_lattice(v[:7], k[:7, :2], (6, 5), (4.0, 2.5), [np.array([5, 1]), np.array([0, 4, 2])])
    ref2 = _brute_sum(v[:7], k[:7, :2], (6, 5), (4.0, 2.5))
    assert np.allclose(got2, ref2[np.ix_([5, 1], [0, 4, 2])], rtol=0, atol=1e-12)


def test_separable_terms_rho_hat_equals_general_sum():
    # |psi|^2 of complex wave packets as a sum of complex separable terms: its
    # transform by the per-term regrouping equals the general sum on the assembled
    # density, and equals brute force on a tiny grid
    rng = np.random.default_rng(16)
    pk = wl.random_wave_packets(rng, p=3, lo=-1.0, hi=1.0)
    n, box = (11, 9, 13), (6.0, 5.0, 7.0)
    psi = pk.evaluate(n, box)
    rho = np.abs(psi) ** 2
    coefs, factors = pk.density_terms(n, box)
    assert len(coefs) == 9
    k = rng.uniform(-2.5, 2.5, size=(40, 3))
    a = oracle.rho_hat_separable_sum(coefs, factors, box, k)
    b = oracle.rho_hat(rho, box, k)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))
    # the transform of a real density is Hermitian: rho^(-k) = conj rho^(k)
    am = oracle.rho_hat_separable_sum(coefs, factors, box, -k)
    assert np.max(np.abs(am - np.conj(a))) < 1e-12 * np.max(np.abs(a))
    n3, box3 = (3, 4, 3), (2.0, 3.0, 2.5)
    c3, f3 = pk.density_terms(n3, box3)
    k3 = k[:5]
    assert np.allclose(oracle.rho_hat_separable_sum(c3, f3, box3, k3),
                       _brute_rho_hat(np.abs(pk.evaluate(n3, box3)) ** 2, box3, k3), rtol=0, atol=1e-13)
    # a real Gaussian mixture through the same route
    mix = wl.random_mixture(rng, 3, 3, -1.0, 1.0, 0.8, 1.5)
    cm, fm = mix.density_terms(n, box)
    assert np.max(np.abs(oracle.rho_hat_separable_sum(cm, fm, box, k)
                         - oracle.rho_hat(mix.evaluate(n, box), box, k))) < 1e-12 * np.max(np.abs(b))


def test_rho_hat_of_shifted_gaussian():
    # rho = exp(-|x-c|^2): the trapezoid sum converges to pi^{3/2} exp(-|k|^2/4) exp(-i k.c);
    # the phase pins the sign of the exponent and the grid offset x_n = -R/2 + n h
    n, box = (28, 30, 26), (14.0, 15.0, 13.0)
    c = np.array([0.7, -1.1, 0.4])
    rho = wl.gaussian(n, box, 1.0, center=c)
    rng = np.random.default_rng(3)
    # |k_i| <= 1.5 keeps the trapezoid rule's aliased images (distance 2 pi/h - 1.5) below 1e-13
    k = rng.uniform(-1.5, 1.5, size=(20, 3))
    exact = np.pi ** 1.5 * np.exp(-np.sum(k * k, axis=1) / 4) * np.exp(-1j * (k @ c))
    assert np.max(np.abs(oracle.rho_hat(rho, box, k) - exact)) < 1e-12


# ------------------------------------------------------------- closed forms

@pytest.mark.parametrize("rule,nodes,tol", [(COSTHETA_GL, (64, 32, 64), 5e-9), (THETA_GL, (96, 48, 96), 2e-10)])
def test_coulomb3d_gaussian_closed_form(rule, nodes, tol):
    n, box = (32, 32, 32), (10.0, 10.0, 10.0)
    p = wl.Problem("pin", 3, n, box, wl.COULOMB_3D, *nodes, theta_rule=rule)
    res = oracle.evaluate(p, wl.gaussian(n, box, 1.0))
    X = wl.mesh(n, box)
    r = np.sqrt(sum(x * x for x in X))
    assert rel(res.u, cf.coulomb3d_gaussian(r, 1.0)) < tol
    E = cf.coulomb3d_gaussian_energy(1.0, 1.0)
    assert abs(E - 0.9843506216076512) < 1e-15
    assert abs(res.energy_fourier - E) < 1e-11 * E
    assert abs(res.energy_physical - res.energy_fourier) < 1e-14 * E
    assert res.imag_max < 1e-14 * np.max(np.abs(res.u))


def test_example1_coulomb2d_closed_form():
    ex = json.load(open(os.path.join(GOLDEN, "examples.json")))["example1"]
    a = ex["a"]
    n, box = (48, 48), (16.0, 16.0)
    p = wl.Problem("ex1", 2, n, box, wl.COULOMB_2D, 64, 1, 128)
    res = oracle.evaluate(p, wl.gaussian(n, box, a))
    X = wl.mesh(n, box)
    r = np.sqrt(X[0] ** 2 + X[1] ** 2)
    assert rel(res.u, cf.coulomb2d_gaussian(r, a)) < 1e-13
    assert abs(res.energy_fourier / cf.coulomb2d_gaussian_energy(a) - 1) < 1e-13


def test_example4_coulomb_log_density():
    a = json.load(open(os.path.join(GOLDEN, "examples.json")))["example4"]["a"]
    n, box = (32, 32, 32), (12.0, 12.0, 12.0)
    p = wl.Problem("ex4", 3, n, box, wl.COULOMB_3D, 64, 32, 64, theta_rule=COSTHETA_GL)
    res = oracle.evaluate(p, wl.log_density(n, box, a))
    assert rel(res.u, cf.example4_potential(wl.mesh(n, box), a)) < 1e-6


def test_example5_dipole_log_density():
    ex = json.load(open(os.path.join(GOLDEN, "examples.json")))["example5"]
    a, nvec = ex["a"], np.array(ex["n"])
    nvec = nvec / np.linalg.norm(nvec)
    n, box = (32, 32, 32), (12.0, 12.0, 12.0)
    p = wl.Problem("ex5", 3, n, box, wl.DIPOLE_3D, 96, 48, 96, theta_rule=COSTHETA_GL, axis=tuple(nvec))
    res = oracle.evaluate(p, wl.log_density(n, box, a))
    assert rel(res.u, cf.example5_potential(wl.mesh(n, box), a, nvec)) < 5e-8
    # a sign flip of the anisotropic part (the variant -rho + 3 d_nn u_Cou) misses by O(1)
    wrong = -2 * wl.log_density(n, box, a) - cf.example5_potential(wl.mesh(n, box), a, nvec)
    assert rel(res.u, wrong) > 0.1


@pytest.mark.parametrize("case", ["I", "II", "III"])
def test_example7_printed_dipole_energies(case):
    g = json.load(open(os.path.join(GOLDEN, "example7.json")))
    c = g["cases"][case]
    lam = 8 * np.pi / 3
    gx, gz = c["gx"], c["gz"]
    assert abs(cf.example7_energy(gx, gz, lam) - c["E_exact"]) < 1e-16
    # box and cutoff wide enough that rho and rho^ are below 1e-16 at the edges
    Lx, Lz = 6.2 / np.sqrt(gx), 6.2 / np.sqrt(gz)
    K = 12.5 * np.sqrt(max(gx, gz))
    h = np.pi / K
    Nx, Nz = int(np.ceil(Lx / h)) * 2, int(np.ceil(Lz / h)) * 2
    n, box = (Nx, Nx, Nz), (Nx * h, Nx * h, Nz * h)
    rho = wl.example7_density(n, box, gx, gz)
    k, W = oracle.spherical_nodes(K, 40, 40, 40, COSTHETA_GL)
    cc = oracle.coefficients(wl.DIPOLE_3D, k, W, (0.0, 0.0, 1.0))
    E = oracle.energy_fourier(cc, oracle.rho_hat(rho, box, k), lam)
    assert abs(E - c["E_exact"]) < 2e-14
    # the paper's own computed value at 27000 nodes sits within its printed error
    assert abs(c["E_table7"] - c["E_exact"]) <= 1.05 * c["abs_err_table7"]


def test_mixture_energies_2d_and_3d():
    rng = np.random.default_rng(7)
    mix2 = wl.random_mixture(rng, 3, 2, -2.0, 2.0, 0.8, 1.2)
    n2, box2 = (64, 64), (24.0, 24.0)
    p2 = wl.Problem("m2", 2, n2, box2, wl.COULOMB_2D, 64, 1, 160)
    r2 = oracle.evaluate(p2, mix2.evaluate(n2, box2))
    assert abs(r2.energy_fourier / cf.mixture_energy(mix2, 2) - 1) < 1e-9
    mix3 = wl.random_mixture(rng, 2, 3, -1.0, 1.0, 0.9, 1.1)
    n3, box3 = (32, 32, 32), (12.0, 12.0, 12.0)
    p3 = wl.Problem("m3", 3, n3, box3, wl.COULOMB_3D, 48, 24, 48, theta_rule=COSTHETA_GL)
    r3 = oracle.evaluate(p3, mix3.evaluate(n3, box3))
    assert abs(r3.energy_fourier / cf.mixture_energy(mix3, 3) - 1) < 1e-8
    X = wl.mesh(n3, box3)
    assert rel(r3.u, cf.mixture_potential(mix3, X, 3)) < 1e-4


# ------------------------------------------------------------- invariants

def _small_dipole(seed=5):
    rng = np.random.default_rng(seed)
    n, box = (10, 12, 8), (5.0, 6.0, 4.0)
    axis = wl.unit_vector(rng)
    p = wl.Problem("inv", 3, n, box, wl.DIPOLE_3D, 8, 6, 12, axis=tuple(axis))
    return p, rng


def test_energy_identity_and_real_potential():
    p, rng = _small_dipole()
    rho = rng.standard_normal(p.n)
    res = oracle.evaluate(p, rho)
    assert abs(res.energy_physical - res.energy_fourier) < 1e-13 * np.sum(np.abs(res.c) * np.abs(res.rhohat) ** 2)
    assert res.imag_max < 1e-13 * np.max(np.abs(res.u))


def test_operator_self_adjoint_and_linear():
    p, rng = _small_dipole(6)
    k, W = oracle.fourier_nodes(p)
    r1, r2 = rng.standard_normal(p.n), rng.standard_normal(p.n)
    A1 = oracle.apply_operator(r1, p.box, p.kernel, k, W, p.axis)
    A2 = oracle.apply_operator(r2, p.box, p.kernel, k, W, p.axis)
    assert abs(np.sum(A1 * r2) - np.sum(r1 * A2)) < 1e-12 * np.linalg.norm(A1) * np.linalg.norm(r2)
    A12 = oracle.apply_operator(2.0 * r1 - 3.0 * r2, p.box, p.kernel, k, W, p.axis)
    assert np.allclose(A12, 2.0 * A1 - 3.0 * A2, atol=1e-12 * np.max(np.abs(A12)))


def test_translation_covariance():
    # u_n = sum_l A(x_n - x_l) rho_l: shifting a compactly supported rho by whole cells shifts u
    n, box = (16, 16, 16), (8.0, 8.0, 8.0)
    p = wl.Problem("tr", 3, n, box, wl.COULOMB_3D, 12, 8, 16)
    rng = np.random.default_rng(8)
    rho = np.zeros(n)
    rho[5:9, 4:8, 6:10] = rng.standard_normal((4, 4, 4))
    u = oracle.evaluate(p, rho).u
    us = oracle.evaluate(p, np.roll(rho, (2, 3, -1), axis=(0, 1, 2))).u
    assert np.allclose(us[2:, 3:, :-1], u[:-2, :-3, 1:], atol=1e-12 * np.max(np.abs(u)))


@pytest.mark.parametrize("kernel,d,pu,pe", [(wl.COULOMB_3D, 3, 2, 5), (wl.DIPOLE_3D, 3, 0, 3), (wl.COULOMB_2D, 2, 1, 3)])
def test_exact_scaling_laws(kernel, d, pu, pe):
    rng = np.random.default_rng(9)
    n = (8, 10, 6)[:d]
    box = (4.0, 5.0, 3.0)[:d]
    rho = rng.standard_normal(n)
    s = 1.7
    axis = tuple(wl.unit_vector(rng))
    args = dict(axis=axis) if kernel == wl.DIPOLE_3D else {}
    p1 = wl.Problem("s1", d, n, box, kernel, 6, 4, 8, **args)
    p2 = wl.Problem("s2", d, n, tuple(s * b for b in box), kernel, 6, 4, 8, **args)
    r1, r2 = oracle.evaluate(p1, rho), oracle.evaluate(p2, rho)
    assert np.allclose(r2.u, s ** pu * r1.u, rtol=0, atol=1e-12 * np.max(np.abs(r2.u)))
    assert abs(r2.energy_fourier - s ** pe * r1.energy_fourier) < 1e-12 * abs(r2.energy_fourier)


def test_xy_swap_symmetry():
    n, box = (12, 12, 10), (6.0, 6.0, 5.0)
    rng = np.random.default_rng(10)
    axis = wl.unit_vector(rng)
    rho = rng.standard_normal(n)
    p = wl.Problem("sw", 3, n, box, wl.DIPOLE_3D, 8, 6, 16, axis=tuple(axis))
    ps = wl.Problem("sw", 3, n, box, wl.DIPOLE_3D, 8, 6, 16, axis=(axis[1], axis[0], axis[2]))
    u = oracle.evaluate(p, rho).u
    us = oracle.evaluate(ps, np.transpose(rho, (1, 0, 2))).u
    assert np.allclose(us, np.transpose(u, (1, 0, 2)), atol=1e-12 * np.max(np.abs(u)))


def test_energy_gradients_against_finite_differences():
    p, rng = _small_dipole(14)
    k, W = oracle.fourier_nodes(p)
    psi = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)

    def E_of(psi_):
        rho = np.abs(psi_) ** 2
        u, rh, c, _ = oracle.potential(rho, p.box, p.kernel, k, W, p.axis)
        return oracle.energy_physical(rho, u, p.box, p.lam), u

    E0, u = E_of(psi)
    g_rho = oracle.energy_gradient_rho(u, p.box, p.lam)
    g_psi = oracle.energy_gradient_psi(u, psi, p.box, p.lam)
    d = 1e-4
    for idx in [(0, 0, 0), (3, 7, 2), (9, 11, 7)]:
        # dE/dRe psi + i dE/dIm psi = 2 dE/dpsi*
        e = np.zeros(p.n)
        e[idx] = d
        dre = (E_of(psi + e)[0] - E_of(psi - e)[0]) / (2 * d)
        dim = (E_of(psi + 1j * e)[0] - E_of(psi - 1j * e)[0]) / (2 * d)
        assert abs((dre + 1j * dim) - 2 * g_psi[idx]) < 1e-7 * max(1.0, abs(g_psi[idx]))
        # and with respect to rho directly
        rho = np.abs(psi) ** 2
        up = oracle.potential(rho + e, p.box, p.kernel, k, W, p.axis)[0]
        um = oracle.potential(rho - e, p.box, p.kernel, k, W, p.axis)[0]
        dr = (oracle.energy_physical(rho + e, up, p.box, p.lam) - oracle.energy_physical(rho - e, um, p.box, p.lam)) / (2 * d)
        assert abs(dr - g_rho[idx]) < 1e-7 * max(1.0, abs(g_rho[idx]))
