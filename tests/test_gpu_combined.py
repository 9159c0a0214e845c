"""GPU parity of feature combinations, through the C ABI:

  * a batch whose members use Algorithm 2 and the newer kernels (two-
    orientation 3D dipole, 2.5D dipole, 2D Poisson): every replay equals each
    member's eager evaluation bitwise and matches the oracle;
  * the GPE driver with the 2.5D dipole and the 2D Poisson potential;
  * Algorithm 2 at the largest line length (n = 512 on one axis: the paired
    first inverse pass with two line pairs per block).
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import gpe, split
from gpu_util import make_plan, rel_l2, say

pytestmark = pytest.mark.gpu
import torch  # noqa: E402
import paper_1311_4120_amd as jgb  # noqa: E402  (a missing library fails, never skips)

_NAMES = {wl.COULOMB_3D: "coulomb3d", wl.COULOMB_2D: "coulomb2d", wl.DIPOLE_3D: "dipole3d",
          wl.DIPOLE_2D: "dipole2d", wl.POISSON_2D: "poisson2d"}


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return tuple(v / np.linalg.norm(v))


def _members():
    rng = np.random.default_rng(51)
    specs = [
        (wl.Problem("b1", 3, (16, 20, 16), (8.0, 10.0, 8.0), wl.DIPOLE_3D, 12, 8, 16, axis=_unit([0.2, 0.5, 0.8]),
                    axis2=_unit([0.9, -0.1, 0.3])), True),
        (wl.Problem("b2", 2, (32, 40), (10.0, 12.0), wl.DIPOLE_2D, 20, 1, 24, axis=_unit([0.3, -0.5, 0.8]),
                    alpha=0.6), True),
        (wl.Problem("b3", 2, (40, 32), (12.0, 10.0), wl.POISSON_2D, 24, 1, 32), False),
        (wl.Problem("b4", 3, (16, 16, 20), (8.0, 8.0, 10.0), wl.COULOMB_3D, 12, 8, 16, eps=1e-5,
                    precision=wl.MIXED), True),
        (wl.Problem("b5", 2, (40, 40), (12.0, 12.0), wl.POISSON_2D, 20, 1, 28, eps=1e-5, precision=wl.MIXED), True),
    ]
    out = []
    for p, sp in specs:
        mix = wl.random_mixture(rng, 3, p.dim, -1.0, 1.0, 0.8, 1.2)
        nodes = (p.n_r, p.n_theta, p.n_phi) if p.dim == 3 else (p.n_r, p.n_phi)
        kw = dict(n=p.n, box=p.box, kernel=_NAMES[p.kernel], nodes=nodes, eps=p.eps,
                  precision="fp64" if p.precision == wl.FP64 else "mixed", axis=p.axis, axis2=p.axis2,
                  alpha=p.alpha, split=sp)
        out.append((p, sp, kw, mix.evaluate(p.n, p.box)))
    return out


def test_batch_of_split_and_new_kernels():
    mem = _members()
    b = jgb.Batch([kw for _, _, kw, _ in mem], nstreams=2)
    dts = [torch.float64 if kw["precision"] == "fp64" else torch.float32 for _, _, kw, _ in mem]
    rhos = [torch.tensor(r, dtype=dt, device="cuda") for (_, _, _, r), dt in zip(mem, dts)]
    u, E = b.bind(rhos)
    for rep in range(2):
        b.run()
        torch.cuda.synchronize()
        for i, (p, sp, kw, r) in enumerate(mem):
            ue, Ee = b.plans[i].potential(rhos[i])
            torch.cuda.synchronize()
            assert torch.equal(u[i], ue), (rep, i)
            assert E[i].item() == Ee.item(), (rep, i)
    for i, (p, sp, kw, r) in enumerate(mem):
        rin = r if kw["precision"] == "fp64" else r.astype(np.float32).astype(np.float64)
        ref = split.potential_split(p, rin)[0] if sp else oracle.evaluate(p, rin).u
        e = rel_l2(u[i].cpu().numpy(), ref)
        say("batch member %d %s split=%s %s relL2 %.2e" % (i, kw["kernel"], sp, kw["precision"], e))
        assert e < p.eps
    b.close()


@pytest.mark.parametrize("kern", [wl.DIPOLE_2D, wl.POISSON_2D])
def test_gpe_with_2d_kernels(kern):
    p = wl.Problem("g2", 2, (48, 40), (12.0, 10.0), kern, 20, 1, 28, lam=3.0,
                   axis=_unit([0.4, -0.3, 0.6]) if kern == wl.DIPOLE_2D else (0.0, 0.0, 1.0), alpha=0.2)
    X = wl.mesh(p.n, p.box)
    psi0 = np.exp(-(X[0] - 0.3) ** 2 / 1.5 - X[1] ** 2 / 1.2) * np.exp(0.4j * X[1])
    trap, beta = (1.0, 1.2), 2.0
    V = gpe.harmonic(p.n, p.box, trap)
    pot = lambda r: oracle.evaluate(p, r).u
    ref = gpe.strang(psi0, p.box, V, beta, p.lam, 0.01, 4, pot)
    drv = jgb.GPE(p.n, p.box, _NAMES[kern], (p.n_r, p.n_phi), dt=0.01, beta=beta, trap=trap, eps=1e-10,
                  precision="fp64", lam=p.lam, axis=p.axis, alpha=p.alpha)
    psi = torch.tensor(psi0, dtype=torch.complex128, device="cuda")
    drv.step(psi, 4)
    e = rel_l2(psi.cpu().numpy(), ref)
    _, en = drv.energy(psi)
    eref = gpe.energies(ref, p.box, V, beta, p.lam, pot)
    ee = max(abs(en[k] - eref[k]) / abs(eref[k]) for k in eref)
    say("gpe with", _NAMES[kern], "psi %.2e energies %.2e" % (e, ee))
    assert e < 1e-9 and ee < 1e-9
    drv.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_split_largest_line(prec):
    p = wl.Problem("l", 3, (512, 8, 10), (64.0, 4.0, 5.0), wl.DIPOLE_3D, 10, 8, 12, axis=_unit([0.7, 0.2, -0.3]))
    rng = np.random.default_rng(61)
    mix = wl.random_mixture(rng, 3, 3, -0.5, 0.5, 0.9, 1.2)
    rho = mix.evaluate(p.n, p.box)
    u_ref, _, _, E_ref = split.potential_split(p, rho)
    eps = 1e-10 if prec == "fp64" else 1e-5
    plan = make_plan(p, eps=eps, precision=prec, split=True)
    u, E = plan.potential(torch.tensor(rho, dtype=torch.float64 if prec == "fp64" else torch.float32, device="cuda"))
    e = rel_l2(u.cpu().numpy(), u_ref)
    eE = abs(E.item() - E_ref) / abs(E_ref)
    say("split, n = (512, 8, 10)", prec, "relL2 %.2e  E %.2e" % (e, eE))
    assert e < eps and eE < eps
    plan.close()
