"""GPU parity of the paper's own spreading kernel (JGB_FLAG_GAUSSIAN_KERNEL;
Section 2: the heat kernel g_tau with tau = 6/N^2 on the grid of 2N points per
axis, a Gaussian over the nearest 12 points, and the deconvolution
sqrt(pi/tau) e^{k^2 tau}; the paper quotes about six digits) through the C ABI:

  * the plan reports width 12 and no semicircle shape parameter;
  * u and E against the oracle's direct sums (no NUFFT: independent of the
    spreading kernel) for the 3D Coulomb and dipole kernels and the 2D Coulomb
    kernel, Algorithms 1 and 2, FP64 and mixed, each tap-kernel form in 3D,
    within 5e-6 (the paper's about six digits: 1.5e-6 at most on these smooth
    densities)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import split
from gpu_util import MODES, make_plan, rel_l2, say

pytestmark = pytest.mark.gpu
import torch  # noqa: E402

CASES = {
    "coulomb3d": wl.Problem("g1", 3, (24, 20, 16), (8.0, 8.0, 8.0), wl.COULOMB_3D, 16, 8, 16),
    "dipole3d": wl.Problem("g2", 3, (20, 24, 16), (9.0, 10.0, 8.0), wl.DIPOLE_3D, 20, 12, 16,
                           axis=(0.36, 0.48, 0.8)),
    "coulomb2d": wl.Problem("g3", 2, (48, 40), (12.0, 10.0), wl.COULOMB_2D, 32, 1, 48),
}
TOL = 5e-6


def _rho(p):
    return wl.random_mixture(np.random.default_rng(5), 3, p.dim, -1.5, 1.5, 0.8, 1.4).evaluate(p.n, p.box)


def test_plan_reports_the_gaussian():
    p = CASES["coulomb3d"]
    plan = make_plan(p, eps=1e-6, gaussian_kernel=True)
    info = plan.info
    say("gaussian plan: width", info["width"], "beta", info["beta"])
    assert info["width"] == 12 and info["beta"] == 0.0
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("alg", [1, 2])
@pytest.mark.parametrize("name", list(CASES))
def test_gaussian_kernel_matches_the_oracle(name, alg, prec):
    p = CASES[name]
    eps = 1e-6 if prec == "fp64" else 1e-5
    q = wl.Problem(**{**p.__dict__, "eps": eps})
    rho = _rho(q)
    rho_in = rho if prec == "fp64" else rho.astype(np.float32).astype(np.float64)
    if alg == 1:
        res = oracle.evaluate(q, rho_in)
        u_ref, E_ref = res.u, res.energy_physical
    else:
        u_ref, _, _, E_ref = split.potential_split(q, rho_in)
    modes = ["staged", "tiles+rings"] if q.dim == 3 and alg == 1 else ["staged"]
    dt = torch.float64 if prec == "fp64" else torch.float32
    for mode in modes:
        plan = make_plan(q, eps=eps, precision=prec, split=(alg == 2), gaussian_kernel=True, **MODES[mode])
        u, E = plan.potential(torch.tensor(rho, dtype=dt, device="cuda"))
        e = rel_l2(u.cpu().numpy(), u_ref)
        eE = abs(E.item() - E_ref) / max(abs(E_ref), 1e-300)
        say("gaussian kernel", name, "alg", alg, prec, mode, "relL2(u) %.2e  E %.2e" % (e, eE))
        assert e < TOL and eE < TOL
        plan.close()
