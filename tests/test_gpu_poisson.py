"""GPU parity of the 2D Poisson kernel (U = -(1/2pi) log|x|, the finite-part
radial rule with its node at k = 0) against the oracle, through the C ABI, by
Algorithm 1 and Algorithm 2, in float64 (eps = 1e-10) and mixed precision
(eps = 1e-5): u, both energies, the origin coefficient and the backward
product."""
import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import split
from oracle.symbols import origin_coefficient
from gpu_util import make_plan, rel_l2, say

pytestmark = pytest.mark.gpu
import torch  # noqa: E402

CASES = {
    "poisson2d": wl.Problem("p1", 2, (64, 48), (16.0, 12.0), wl.POISSON_2D, 32, 1, 48),
    "poisson2d_kmax": wl.Problem("p2", 2, (40, 50), (10.0, 12.5), wl.POISSON_2D, 20, 1, 32, kmax=6.0),
}


def _rho(p, seed=12):
    rng = np.random.default_rng(seed)
    mix = wl.random_mixture(rng, 3, 2, -1.5, 1.5, 0.8, 1.2)
    return mix.evaluate(p.n, p.box)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("alg", [1, 2])
@pytest.mark.parametrize("name", list(CASES))
def test_poisson_matches_oracle(name, alg, prec):
    p = CASES[name]
    rho = _rho(p)
    if alg == 1:
        r = oracle.evaluate(p, rho)
        u_ref, E_ref = r.u, r.energy_physical
    else:
        u_ref, _, _, E_ref = split.potential_split(p, rho)
    eps = 1e-10 if prec == "fp64" else 1e-5
    say("poisson", name, "algorithm", alg, prec)
    plan = make_plan(p, eps=eps, precision=prec, split=(alg == 2))
    K = plan.info["kmax"]
    assert plan.info["origin_coef"] == pytest.approx(origin_coefficient(wl.POISSON_2D, K, p.n_r), rel=1e-13)
    dt = torch.float64 if prec == "fp64" else torch.float32
    rt = torch.tensor(rho, dtype=dt, device="cuda")
    u, E = plan.potential(rt)
    Ef = plan.energy(rt)
    e = rel_l2(u.cpu().numpy(), u_ref)
    eE = abs(E.item() - E_ref) / abs(E_ref)
    eEf = abs(Ef.item() - E_ref) / abs(E_ref)
    g = _rho(p, seed=13)
    gb = plan.backward(torch.tensor(g, dtype=dt, device="cuda")).cpu().numpy()
    gref = oracle.evaluate(p, g).u if alg == 1 else split.potential_split(p, g)[0]
    eb = rel_l2(gb, gref)
    say("   relL2(u) %.2e  E %.2e  E_F %.2e  backward %.2e" % (e, eE, eEf, eb))
    assert e < eps and eE < eps and eEf < eps and eb < eps
    plan.close()
