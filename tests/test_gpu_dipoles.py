"""GPU parity of the remaining dipole symbols (3D with two orientations, eq.
dipkerneldF; 2.5D with one or two orientations, alpha and n_3, eqs.
dipkernelF2d and dipkernelF2dd) against the oracle, through the C ABI, by
Algorithm 1 and by Algorithm 2 (JGB_FLAG_SPLIT), in float64 (eps = 1e-10) and
mixed precision (eps = 1e-5): u, both energies and the node coefficients."""
import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import split
from gpu_util import make_plan, rel_l2, say

pytestmark = pytest.mark.gpu
import torch  # noqa: E402


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return tuple(v / np.linalg.norm(v))


CASES = {
    "dipole3d_nm": wl.Problem("d1", 3, (20, 16, 24), (10.0, 8.0, 12.0), wl.DIPOLE_3D, 16, 12, 16,
                              axis=_unit([0.3, -0.7, 0.5]), axis2=_unit([0.8, 0.1, -0.4])),
    "dipole3d_nm_costheta": wl.Problem("d2", 3, (16, 18, 16), (8.0, 9.0, 8.0), wl.DIPOLE_3D, 14, 10, 14,
                                       theta_rule=wl.COSTHETA_GL, axis=_unit([0.1, 0.2, 0.97]),
                                       axis2=_unit([-0.5, 0.8, 0.3])),
    "dipole2d_inplane": wl.Problem("d3", 2, (48, 64), (12.0, 16.0), wl.DIPOLE_2D, 24, 1, 32,
                                   axis=_unit([0.5246, -0.85135, 0.0])),
    "dipole2d_one_alpha": wl.Problem("d4", 2, (40, 40), (10.0, 10.0), wl.DIPOLE_2D, 20, 1, 28,
                                     axis=_unit([0.3, -0.5, 0.8]), alpha=-0.4),
    "dipole2d_two_alpha": wl.Problem("d5", 2, (40, 50), (10.0, 12.5), wl.DIPOLE_2D, 20, 1, 28,
                                     axis=_unit([0.3, -0.5, 0.8]), axis2=_unit([-0.6, 0.2, 0.5]), alpha=0.7),
}


def _rho(p, seed=8):
    rng = np.random.default_rng(seed)
    lo = -0.15 * min(p.box)
    mix = wl.random_mixture(rng, 3, p.dim, lo, -lo, 0.07 * min(p.box) + 0.2, 0.1 * min(p.box) + 0.4)
    return mix.evaluate(p.n, p.box)


_REF = {}


def _ref(name, alg):
    key = (name, alg)
    if key not in _REF:
        p = CASES[name]
        rho = _rho(p)
        if alg == 1:
            r = oracle.evaluate(p, rho)
            _REF[key] = (rho, r.u, r.energy_physical, r.c)
        else:
            u, _, _, E = split.potential_split(p, rho)
            _REF[key] = (rho, u, E, None)
    return _REF[key]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("alg", [1, 2])
@pytest.mark.parametrize("name", list(CASES))
def test_dipole_symbols_match_oracle(name, alg, prec):
    p = CASES[name]
    rho, u_ref, E_ref, c_ref = _ref(name, alg)
    eps = 1e-10 if prec == "fp64" else 1e-5
    say("dipole symbols", name, "algorithm", alg, prec)
    plan = make_plan(p, eps=eps, precision=prec, split=(alg == 2))
    dt = torch.float64 if prec == "fp64" else torch.float32
    rt = torch.tensor(rho, dtype=dt, device="cuda")
    u, E = plan.potential(rt)
    Ef = plan.energy(rt)
    e = rel_l2(u.cpu().numpy(), u_ref)
    scale = 0.5 * p.lam * np.prod([b / m for b, m in zip(p.box, p.n)]) * float(np.sum(np.abs(rho * u_ref)))
    eE = abs(E.item() - E_ref) / scale
    eEf = abs(Ef.item() - E_ref) / scale
    msg = "   relL2(u) %.2e  E %.2e  E_F %.2e" % (e, eE, eEf)
    if c_ref is not None:
        _, _, cg = plan.nodes()
        ec = np.max(np.abs(cg.cpu().numpy() - c_ref)) / np.max(np.abs(c_ref))
        msg += "  c %.2e" % ec
        assert ec < 1e-13
    say(msg)
    assert e < eps and eE < eps and eEf < eps
    plan.close()
