"""GPU parity of every stage of the path against the oracle on small grids
that span several tiles and ragged tails.  Calls go through the C ABI."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import MODES, half_index, make_plan, rel_l2, say

pytestmark = pytest.mark.gpu

import torch  # noqa: E402


def _cases():
    rng = np.random.default_rng(21)
    ax = tuple(wl.unit_vector(rng))
    return {
        "coulomb3d_theta": wl.Problem("c3t", 3, (16, 12, 20), (8.0, 7.0, 9.0), wl.COULOMB_3D, 10, 8, 12),
        "coulomb3d_costheta": wl.Problem("c3c", 3, (24, 16, 18), (10.0, 8.0, 9.0), wl.COULOMB_3D, 12, 9, 14,
                                         theta_rule=wl.COSTHETA_GL),
        "dipole3d": wl.Problem("d3", 3, (20, 24, 16), (9.0, 10.0, 8.0), wl.DIPOLE_3D, 12, 10, 16, axis=ax),
        "coulomb2d": wl.Problem("c2", 2, (40, 36), (12.0, 11.0), wl.COULOMB_2D, 24, 1, 30),
    }


CASES = _cases()


def _rho(p, seed=3):
    rng = np.random.default_rng(seed)
    mix = wl.random_mixture(rng, 3, p.dim, -1.5, 1.5, 0.8, 1.4)
    return mix.evaluate(p.n, p.box)


@pytest.mark.parametrize("name", list(CASES))
def test_nodes_match_oracle(name):
    p = CASES[name]
    say("nodes", name)
    plan = make_plan(p)
    k, W, c = (t.cpu().numpy() for t in plan.nodes())
    torch.cuda.synchronize()
    ko, Wo = oracle.fourier_nodes(p)
    co = oracle.coefficients(p.kernel, ko, Wo, p.axis)
    assert np.max(np.abs(k - ko)) <= 4e-16 * np.max(np.abs(ko)) * 8
    assert np.max(np.abs(W - Wo) / np.abs(Wo)) < 1e-13
    assert np.max(np.abs(c - co)) <= 1e-13 * np.max(np.abs(co))
    plan.close()


# (name, tap-kernel forms): every case with the staged interpolation and the
# three-axis gather, the 3D cases also with the interpolation by tiles and
# with the spreading by rings
VARIANTS = [(n, "staged") for n in CASES] + [(n, m) for n in CASES if CASES[n].dim == 3 for m in ("tiles", "rings")]


@pytest.mark.parametrize("name,mode", VARIANTS)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_transform_matches_oracle(name, mode, prec):
    p = CASES[name]
    eps = 1e-10 if prec == "fp64" else 1e-5
    say("transform", name, prec, mode)
    rho = _rho(p)
    dt = torch.float64 if prec == "fp64" else torch.float32
    plan = make_plan(p, eps=eps, precision=prec, **MODES[mode])
    got = plan.transform(torch.tensor(rho, dtype=dt, device="cuda")).cpu().numpy()
    ko, Wo = oracle.fourier_nodes(p)
    rho_in = rho if prec == "fp64" else rho.astype(np.float32).astype(np.float64)
    ref = oracle.rho_hat(rho_in, p.box, ko[half_index(p)])
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    say("   max rel err", err)
    assert err < eps
    plan.close()


@pytest.mark.parametrize("name,mode", VARIANTS)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_potential_and_energy_match_oracle(name, mode, prec):
    p = CASES[name]
    eps = 1e-10 if prec == "fp64" else 1e-5
    say("potential", name, prec, mode)
    rho = _rho(p)
    dt = torch.float64 if prec == "fp64" else torch.float32
    plan = make_plan(p, eps=eps, precision=prec, **MODES[mode])
    rt = torch.tensor(rho, dtype=dt, device="cuda")
    u, E = plan.potential(rt)
    Ef = plan.energy(rt)
    u = u.cpu().numpy()
    rho_in = rho if prec == "fp64" else rho.astype(np.float32).astype(np.float64)
    res = oracle.evaluate(p, rho_in)
    e_u = rel_l2(u, res.u)
    e_E = abs(E.item() - res.energy_physical) / abs(res.energy_physical)
    e_Ef = abs(Ef.item() - res.energy_fourier) / abs(res.energy_fourier)
    say("   relL2 u %.3e  E %.3e  E_F %.3e" % (e_u, e_E, e_Ef))
    assert e_u < eps
    assert e_E < eps
    assert e_Ef < eps
    plan.close()
