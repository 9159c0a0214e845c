"""GPU parity of the time-splitting driver (jgb_gpe_*) against `oracle.gpe`,
through the C ABI:

  * the free flow of a moving Gaussian packet against its exact solution;
  * real-time steps with a trap, local and nonlocal (3D dipole) interactions,
    the potential by Algorithm 1 and by Algorithm 2, float64 and mixed;
  * imaginary-time steps (2D Coulomb) with renormalisation;
  * the seven energies of jgb_gpe_energy;
  * graph replays against eager steps, with eager work between the replays;
  * time reversibility on the device (steps of dt, then of -dt).
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import gpe, split
from gpu_util import rel_l2, say

pytestmark = pytest.mark.gpu
import torch  # noqa: E402
import paper_1311_4120_amd as jgb  # noqa: E402  (a missing library fails, never skips)

_KERN = {wl.COULOMB_3D: "coulomb3d", wl.COULOMB_2D: "coulomb2d", wl.DIPOLE_3D: "dipole3d", wl.DIPOLE_2D: "dipole2d"}


def _driver(p, dt, beta, trap, prec, imaginary=False, split_=False):
    nodes = (p.n_r, p.n_theta, p.n_phi) if p.dim == 3 else (p.n_r, p.n_phi)
    return jgb.GPE(p.n, p.box, _KERN[p.kernel], nodes, dt=dt, beta=beta, trap=trap, imaginary=imaginary,
                   eps=1e-10 if prec == "fp64" else 1e-5, precision=prec, lam=p.lam, axis=p.axis,
                   split=split_)


def _cdt(prec):
    return torch.complex128 if prec == "fp64" else torch.complex64


def _packet(X, t, s, k0):
    d = len(X)
    a = s * s + 1j * t
    r2 = sum((Xi - ki * t) ** 2 for Xi, ki in zip(X, k0))
    phase = sum(ki * Xi for ki, Xi in zip(k0, X)) - 0.5 * t * sum(ki * ki for ki in k0)
    return (s * s / a) ** (d / 2.0) * np.exp(-r2 / (2.0 * a) + 1j * phase)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_free_packet(prec):
    p = wl.Problem("f", 2, (80, 80), (24.0, 24.0), wl.COULOMB_2D, 8, 1, 8, lam=0.0)
    X = wl.mesh(p.n, p.box)
    psi = torch.tensor(_packet(X, 0.0, 1.0, (1.0, -0.5)), dtype=_cdt(prec), device="cuda")
    drv = _driver(p, 0.05, 0.0, (0.0, 0.0), prec)
    drv.step(psi, 10)
    e = rel_l2(psi.cpu().numpy(), _packet(X, 0.5, 1.0, (1.0, -0.5)))
    say("gpe free packet", prec, "%.2e" % e)
    assert e < (1e-10 if prec == "fp64" else 2e-5)
    drv.close()


def _dipole_case():
    p = wl.Problem("g", 3, (16, 16, 16), (10.0, 10.0, 10.0), wl.DIPOLE_3D, 10, 8, 12, lam=20.0,
                   axis=tuple(wl.unit_vector(np.random.default_rng(3))))
    X = wl.mesh(p.n, p.box)
    psi = np.exp(-(X[0] ** 2 / 2.0 + X[1] ** 2 / 3.0 + X[2] ** 2 / 1.6)) * np.exp(0.3j * X[0])
    return p, psi, (1.0, 0.8, 1.4), 3.0


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("alg", [1, 2])
def test_real_time_matches_oracle(alg, prec):
    p, psi0, trap, beta = _dipole_case()
    V = gpe.harmonic(p.n, p.box, trap)
    pot = (lambda r: oracle.evaluate(p, r).u) if alg == 1 else (lambda r: split.potential_split(p, r)[0])
    ref = gpe.strang(psi0, p.box, V, beta, p.lam, 0.01, 4, pot)
    drv = _driver(p, 0.01, beta, trap, prec, split_=(alg == 2))
    psi = torch.tensor(psi0, dtype=_cdt(prec), device="cuda")
    drv.step(psi, 4)
    e = rel_l2(psi.cpu().numpy(), ref)
    _, en = drv.energy(psi)
    eref = gpe.energies(ref, p.box, V, beta, p.lam, pot)
    ee = max(abs(en[k] - eref[k]) / max(abs(eref[k]), 1e-300) for k in eref)
    say("gpe real time, algorithm", alg, prec, "psi %.2e  energies %.2e" % (e, ee))
    tol = 1e-9 if prec == "fp64" else 2e-5
    assert e < tol and ee < tol
    drv.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_imaginary_time_matches_oracle(prec):
    p = wl.Problem("i", 2, (48, 40), (12.0, 10.0), wl.COULOMB_2D, 20, 1, 28, lam=2.0)
    X = wl.mesh(p.n, p.box)
    psi0 = np.exp(-(X[0] - 0.4) ** 2 - 0.5 * X[1] ** 2) * (1 + 0.2j * X[1])
    trap, beta = (1.0, 1.3), 1.5
    V = gpe.harmonic(p.n, p.box, trap)
    pot = lambda r: oracle.evaluate(p, r).u
    ref = gpe.strang(psi0, p.box, V, beta, p.lam, 0.02, 5, pot, imaginary=True)
    drv = _driver(p, 0.02, beta, trap, prec, imaginary=True)
    psi = torch.tensor(psi0, dtype=_cdt(prec), device="cuda")
    drv.step(psi, 5)
    e = rel_l2(psi.cpu().numpy(), ref)
    _, en = drv.energy(psi)
    eref = gpe.energies(ref, p.box, V, beta, p.lam, pot)
    ee = max(abs(en[k] - eref[k]) / abs(eref[k]) for k in eref)
    say("gpe imaginary time", prec, "psi %.2e  energies %.2e  norm %.15f" % (e, ee, en["norm"]))
    tol = 1e-9 if prec == "fp64" else 2e-5
    assert e < tol and ee < tol
    drv.close()


def test_graph_replays_match_eager_steps():
    p, psi0, trap, beta = _dipole_case()
    drv = _driver(p, 0.01, beta, trap, "fp64")
    a = torch.tensor(psi0, dtype=torch.complex128, device="cuda")
    b = a.clone()
    for rep in range(3):
        drv.step(a, 2, graph=True)
        torch.cuda.synchronize()
        _ = (a.abs() ** 2).sum().item()        # eager work between the replays
        drv.step(b, 2, graph=False)
        torch.cuda.synchronize()
        d = (a - b).abs().max().item()
        say("gpe graph vs eager, replay", rep, "max |diff| %.1e" % d)
        assert d == 0.0
    drv.close()


def test_time_reversibility_on_device():
    p, psi0, trap, beta = _dipole_case()
    fwd = _driver(p, 0.01, beta, trap, "fp64")
    bwd = _driver(p, -0.01, beta, trap, "fp64")
    psi = torch.tensor(psi0, dtype=torch.complex128, device="cuda")
    fwd.step(psi, 4)
    moved = rel_l2(psi.cpu().numpy(), psi0)
    bwd.step(psi, 4)
    e = rel_l2(psi.cpu().numpy(), psi0)
    say("gpe reversibility: moved %.2e, back %.2e" % (moved, e))
    assert moved > 1e-3 and e < 1e-12
    fwd.close()
    bwd.close()
