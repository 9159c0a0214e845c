"""Pins of the time-splitting driver in the oracle (`oracle.gpe`).  CPU only.

  * the free Schroedinger flow of a moving Gaussian packet (exact solution);
  * the energies of a Gaussian against closed forms;
  * exact time reversibility of the Strang step with every term on (trap,
    local and nonlocal interactions), and norm conservation in real time;
  * the imaginary-time flow reaching the harmonic ground state (energy
    sum gamma_j / 2) and, with interactions, lowering the energy.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import gpe

_zero = lambda rho: np.zeros_like(rho)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _free_packet(X, t, s, k0):
    """psi(x, t) of i psi_t = -1/2 Lap psi from exp(-|x|^2/(2 s^2) + i k0.x)."""
    d = len(X)
    a = s * s + 1j * t
    r2 = sum((Xi - ki * t) ** 2 for Xi, ki in zip(X, k0))
    phase = sum(ki * Xi for ki, Xi in zip(k0, X)) - 0.5 * t * sum(ki * ki for ki in k0)
    return (s * s / a) ** (d / 2.0) * np.exp(-r2 / (2.0 * a) + 1j * phase)


@pytest.mark.parametrize("n,box,k0", [((80, 80), (24.0, 24.0), (1.0, -0.5)),
                                      ((40, 40, 40), (16.0, 16.0, 16.0), (0.5, 0.0, -0.7))])
def test_free_packet_is_exact(n, box, k0):
    X = wl.mesh(n, box)
    psi0 = _free_packet(X, 0.0, 1.0, k0)
    dt, steps = 0.05, 10
    V = np.zeros(n)
    psi = gpe.strang(psi0, box, V, 0.0, 0.0, dt, steps, _zero)
    assert rel(psi, _free_packet(X, dt * steps, 1.0, k0)) < 1e-10
    # the sign of i: the packet moves along +k0
    assert rel(psi, _free_packet(X, -dt * steps, 1.0, k0)) > 1e-2


def test_gaussian_energies_closed_form():
    n, box, s, gam, beta = (48, 40, 44), (16.0, 14.0, 15.0), 1.1, (0.8, 1.3, 1.0), 2.5
    X = wl.mesh(n, box)
    psi = np.exp(-sum(Xi ** 2 for Xi in X) / (2 * s * s)).astype(complex)
    V = gpe.harmonic(n, box, gam)
    e = gpe.energies(psi, box, V, beta, 0.0, _zero)
    nrm = (np.pi * s * s) ** 1.5
    assert e["norm"] == pytest.approx(nrm, rel=1e-12)
    assert e["kinetic"] == pytest.approx(3 / (4 * s * s) * nrm, rel=1e-12)
    assert e["trap"] == pytest.approx(sum(0.5 * g * g * s * s / 2 for g in gam) * nrm, rel=1e-12)
    assert e["local"] == pytest.approx(0.5 * beta * (np.pi * s * s / 2) ** 1.5, rel=1e-12)
    assert e["mu"] == pytest.approx((e["kinetic"] + e["trap"] + 2 * e["local"]) / nrm, rel=1e-14)


def _dipole_setup():
    p = wl.Problem("g", 3, (16, 16, 16), (10.0, 10.0, 10.0), wl.DIPOLE_3D, 10, 8, 12,
                   axis=tuple(wl.unit_vector(np.random.default_rng(3))))
    X = wl.mesh(p.n, p.box)
    psi = np.exp(-(X[0] ** 2 / 2.0 + X[1] ** 2 / 3.0 + X[2] ** 2 / 1.6)) * np.exp(0.3j * X[0])
    V = gpe.harmonic(p.n, p.box, (1.0, 0.8, 1.4))
    pot = lambda rho: oracle.evaluate(p, rho).u
    return p, psi, V, pot


def test_strang_is_time_reversible_and_unitary():
    p, psi0, V, pot = _dipole_setup()
    psi1 = gpe.strang(psi0, p.box, V, 3.0, 20.0, 0.01, 4, pot)
    assert gpe.norm(psi1, p.box) == pytest.approx(gpe.norm(psi0, p.box), rel=1e-13)
    assert rel(psi1, psi0) > 1e-3
    back = gpe.strang(psi1, p.box, V, 3.0, 20.0, -0.01, 4, pot)
    assert rel(back, psi0) < 1e-12


def test_real_time_energy_drift_is_second_order():
    p, psi0, V, pot = _dipole_setup()
    e0 = gpe.energies(psi0, p.box, V, 3.0, 20.0, pot)["total"]
    drift = []
    for dt, steps in ((0.01, 4), (0.005, 8)):
        psi = gpe.strang(psi0, p.box, V, 3.0, 20.0, dt, steps, pot)
        drift.append(abs(gpe.energies(psi, p.box, V, 3.0, 20.0, pot)["total"] - e0))
    assert drift[1] < drift[0] / 3      # halving dt cuts the drift about fourfold


def test_imaginary_time_reaches_harmonic_ground_state():
    n, box, gam = (48, 48), (14.0, 14.0), (1.0, 1.5)
    X = wl.mesh(n, box)
    V = gpe.harmonic(n, box, gam)
    psi0 = np.exp(-(X[0] - 0.5) ** 2 - 0.3 * X[1] ** 2).astype(complex)
    psi = gpe.strang(psi0, box, V, 0.0, 0.0, 0.01, 2500, _zero, imaginary=True)
    e = gpe.energies(psi, box, V, 0.0, 0.0, _zero)
    assert e["norm"] == pytest.approx(1.0, rel=1e-13)
    assert e["total"] == pytest.approx(0.5 * sum(gam), abs=2e-5)
    ground = np.prod([(g / np.pi) ** 0.25 * np.exp(-g * Xi ** 2 / 2) for g, Xi in zip(gam, X)], axis=0)
    assert rel(np.abs(psi), ground) < 1e-3


def test_imaginary_time_with_interactions_lowers_energy():
    p, psi0, V, pot = _dipole_setup()
    psi0 = psi0 / np.sqrt(gpe.norm(psi0, p.box))
    es = [gpe.energies(psi0, p.box, V, 3.0, 20.0, pot)["total"]]
    psi = psi0
    for _ in range(3):
        psi = gpe.strang(psi, p.box, V, 3.0, 20.0, 0.02, 5, pot, imaginary=True)
        es.append(gpe.energies(psi, p.box, V, 3.0, 20.0, pot)["total"])
    assert all(b < a for a, b in zip(es, es[1:]))
