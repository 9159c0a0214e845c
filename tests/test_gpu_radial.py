"""GPU parity of the generalized Gaussian radial rule (JGB_FLAG_RADIAL_GGQ;
Section 3.3's last remark, the Conclusions) through the C ABI:

  * the plan's radial nodes, weights and bandwidth against the oracle's rule;
  * u and E of the 2D Poisson kernel (Algorithms 1 and 2) and of the 3D dipole
    against the oracle evaluated with the same rule, FP64 and mixed;
  * against the closed-form 2D Poisson potential of a Gaussian mixture: 44
    generalized Gaussian radial nodes reach the accuracy of 52 Gauss-Legendre
    nodes (and beat 48)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import closed_forms as cf
from oracle import split
from oracle.ggq import bandwidth
from oracle.quadrature import radial_rule
from gpu_util import make_plan, rel_l2, say

pytestmark = pytest.mark.gpu
import torch  # noqa: E402

MIX = wl.random_mixture(np.random.default_rng(12), 3, 2, -1.5, 1.5, 0.8, 1.2)


def _poisson(n_r, radial, n_phi=48):
    return wl.Problem("p1", 2, (64, 48), (16.0, 12.0), wl.POISSON_2D, n_r, 1, n_phi, radial=radial)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_radial_rule_matches_the_oracle(prec):
    p = _poisson(44, wl.RADIAL_GGQ)
    eps = 1e-10 if prec == "fp64" else 1e-5
    plan = make_plan(p, eps=eps, precision=prec, radial_ggq=True)
    c = plan.info["radial_c"]
    say("radial rule", prec, "c %.4f" % c)
    assert c == pytest.approx(bandwidth(44, eps), rel=1e-14) and c > 1.0
    k, W, _ = (t.cpu().numpy() for t in plan.nodes())
    K = np.pi / 0.25
    r_ref, w_ref = radial_rule(K, 44, wl.RADIAL_GGQ, eps)
    r = np.hypot(k[:, 0], k[:, 1]).reshape(44, -1)[:, 0]
    assert np.max(np.abs(r - r_ref)) < 1e-12 * K
    wr = W.reshape(44, -1)[:, 0] / (2 * np.pi / p.n_phi)
    assert np.max(np.abs(wr - w_ref)) < 1e-12 * K
    plan.close()


CASES = [("poisson2d", 1, _poisson(44, wl.RADIAL_GGQ)), ("poisson2d", 2, _poisson(44, wl.RADIAL_GGQ)),
         ("dipole3d", 1, wl.Problem("d3", 3, (20, 24, 16), (9.0, 10.0, 8.0), wl.DIPOLE_3D, 28, 12, 16,
                                    axis=(0.36, 0.48, 0.8), radial=wl.RADIAL_GGQ))]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name,alg,p", CASES, ids=["%s-alg%d" % (c[0], c[1]) for c in CASES])
def test_potential_with_the_radial_rule_matches_the_oracle(name, alg, p, prec):
    eps = 1e-10 if prec == "fp64" else 1e-5
    q = wl.Problem(**{**p.__dict__, "eps": eps})
    rho = MIX.evaluate(q.n, q.box) if q.dim == 2 else wl.random_mixture(
        np.random.default_rng(3), 3, 3, -1.5, 1.5, 0.8, 1.4).evaluate(q.n, q.box)
    rho_in = rho if prec == "fp64" else rho.astype(np.float32).astype(np.float64)
    if alg == 1:
        res = oracle.evaluate(q, rho_in)
        u_ref, E_ref = res.u, res.energy_physical
    else:
        u_ref, _, _, E_ref = split.potential_split(q, rho_in)
    plan = make_plan(q, eps=eps, precision=prec, radial_ggq=True, split=(alg == 2))
    dt = torch.float64 if prec == "fp64" else torch.float32
    u, E = plan.potential(torch.tensor(rho, dtype=dt, device="cuda"))
    e = rel_l2(u.cpu().numpy(), u_ref)
    eE = abs(E.item() - E_ref) / max(abs(E_ref), 1e-300)
    say("radial GGQ", name, "alg", alg, prec, "relL2(u) %.2e  E %.2e" % (e, eE))
    assert e < eps and eE < eps
    plan.close()


def test_fewer_radial_nodes_at_equal_accuracy():
    """u on the grid against the closed-form potential (128 angles, so the
    radial rule sets the error): the generalized Gaussian rule's 44 nodes
    against Gauss-Legendre's 48 and 52."""
    errs = {}
    for n_r, radial in ((44, wl.RADIAL_GGQ), (48, wl.RADIAL_GL), (52, wl.RADIAL_GL)):
        p = _poisson(n_r, radial, n_phi=128)
        plan = make_plan(p, eps=1e-10, precision="fp64", radial_ggq=(radial == wl.RADIAL_GGQ))
        rho = MIX.evaluate(p.n, p.box)
        u = plan.potential(torch.tensor(rho, dtype=torch.float64, device="cuda"))[0].cpu().numpy()
        X = wl.grid_axes(p.n, p.box)
        ref = cf.mixture_potential(MIX, np.meshgrid(*X, indexing="ij"), 2, poisson=True)
        errs[(n_r, radial)] = np.max(np.abs(u - ref)) / np.max(np.abs(ref))
        plan.close()
    say("closed form: GGQ 44 %.2e  GL 48 %.2e  GL 52 %.2e" % (errs[(44, 1)], errs[(48, 0)], errs[(52, 0)]))
    assert errs[(44, 1)] < 1e-9 < errs[(48, 0)]
    assert errs[(44, 1)] < 1.5 * errs[(52, 0)]
