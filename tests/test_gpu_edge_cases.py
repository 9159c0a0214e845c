"""GPU parity at the edges of what a plan accepts, against the full oracle:

  * the largest grid per axis (n = 512, oversampled to 1024 points, the most the
    gather's 10-bit tap offsets address), in 3D along one axis and in 2D on both;
  * the smallest node sets (one radial and one polar node, two azimuthal ones:
    a single node in the half set) and the smallest grids (n = 8 per axis);
  * a cut-off below the default pi / max h;
  * the accuracy extremes (eps = 1e-13, the widest kernel, and eps = 1e-2);
  * a zero density (u, E and the transform exactly zero).
Calls go through the C ABI; every case is checked in float64 and, where its
eps allows, in mixed precision."""
import numpy as np
import pytest

import oracle
import workloads as wl
from gpu_util import half_index, make_plan, rel_l2, say

pytestmark = pytest.mark.gpu
import torch  # noqa: E402


def _axis(seed):
    return tuple(wl.unit_vector(np.random.default_rng(seed)))


CASES = {
    # one axis at the largest size, the others small and unequal
    "dipole3d_n512_axis0": wl.Problem("e1", 3, (512, 8, 10), (64.0, 4.0, 5.0), wl.DIPOLE_3D, 12, 8, 12,
                                      axis=_axis(31)),
    # a 2D grid at the largest size on both axes
    "coulomb2d_512": wl.Problem("e2", 2, (512, 512), (32.0, 32.0), wl.COULOMB_2D, 16, 1, 24),
    # the smallest grid and node set: n = 8, nodes (1, 1, 2) -> one half-set node
    "coulomb3d_min": wl.Problem("e3", 3, (8, 8, 8), (6.0, 6.0, 6.0), wl.COULOMB_3D, 1, 1, 2),
    "coulomb2d_min": wl.Problem("e4", 2, (8, 10), (5.0, 6.0), wl.COULOMB_2D, 1, 1, 2),
    # a cut-off below the default
    "dipole3d_kmax": wl.Problem("e5", 3, (16, 20, 12), (8.0, 9.0, 7.0), wl.DIPOLE_3D, 10, 8, 12, axis=_axis(32),
                                kmax=1.7),
}


def _rho(p, seed=5):
    rng = np.random.default_rng(seed)
    lo = -0.2 * min(p.box)
    mix = wl.random_mixture(rng, 3, p.dim, lo, -lo, 0.06 * min(p.box) + 0.3, 0.1 * min(p.box) + 0.5)
    return mix.evaluate(p.n, p.box)


_REF = {}


def _oracle(name):
    if name not in _REF:
        p = CASES[name]
        rho = _rho(p)
        _REF[name] = (rho, oracle.evaluate(p, rho))
    return _REF[name]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_edge_case_matches_oracle(name, prec):
    p = CASES[name]
    rho, res = _oracle(name)
    eps = 1e-10 if prec == "fp64" else 1e-5
    say("edge case", name, prec, "grid", p.n, "nodes", (p.n_r, p.n_theta, p.n_phi))
    plan = make_plan(p, eps=eps, precision=prec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    rt = torch.tensor(rho, dtype=dt, device="cuda")
    u, E = plan.potential(rt)
    Ef = plan.energy(rt)
    th = plan.transform(rt).cpu().numpy()
    ref = res.rhohat[half_index(p)]
    et = np.max(np.abs(th - ref)) / np.max(np.abs(ref))
    e = rel_l2(u.cpu().numpy(), res.u)
    scale = 0.5 * p.lam * float(np.sum(np.abs(res.c) * np.abs(res.rhohat) ** 2))
    eE = abs(E.item() - res.energy_physical) / scale
    eEf = abs(Ef.item() - res.energy_fourier) / scale
    say("   transform %.2e  relL2(u) %.2e  E %.2e  E_F %.2e" % (et, e, eE, eEf))
    assert et < eps and e < eps and eE < eps and eEf < eps
    plan.close()


@pytest.mark.parametrize("eps", [1e-13, 1e-2])
def test_accuracy_extremes(eps):
    """The widest kernel (eps = 1e-13) and the narrowest (eps = 1e-2), fp64."""
    p = wl.Problem("e6", 3, (16, 12, 10), (8.0, 7.0, 6.5), wl.DIPOLE_3D, 10, 8, 12, axis=_axis(33))
    rho = _rho(p, seed=9)
    res = oracle.evaluate(p, rho)
    plan = make_plan(p, eps=eps, precision="fp64")
    say("accuracy extreme eps", eps, "width", plan.info["width"])
    u, E = plan.potential(torch.tensor(rho, dtype=torch.float64, device="cuda"))
    e = rel_l2(u.cpu().numpy(), res.u)
    say("   relL2(u) %.2e" % e)
    assert e < eps
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_zero_density(prec):
    p = wl.Problem("e7", 3, (16, 18, 10), (8.0, 8.0, 8.0), wl.DIPOLE_3D, 8, 6, 10, axis=_axis(34))
    eps = 1e-10 if prec == "fp64" else 1e-5
    plan = make_plan(p, eps=eps, precision=prec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    z = torch.zeros(p.n, dtype=dt, device="cuda")
    u, E = plan.potential(z)
    assert torch.count_nonzero(u).item() == 0 and E.item() == 0.0
    assert plan.energy(z).item() == 0.0
    assert torch.count_nonzero(plan.transform(z)).item() == 0
    plan.close()


@pytest.mark.parametrize("n", [(24, 20, 30), (96, 12, 10)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_spectrum_reach_after_a_larger_density(prec, n):
    """Under the interpolation by tiles the forward transform's last pass stores,
    per line of the spectrum, only the range that the listed tiles read (their
    points, or the mirror images past nf2 / 2); the rest keeps what an earlier
    call left there.  A call after one on a density a million times larger must
    equal, bit for bit, the same call on a fresh plan: no point outside the
    stored ranges is read.  The grids span several tiles per axis, with ragged
    edges; the second one's 192-point lines along the masked pass take fewer
    lines per block than the unmasked pass would (a divisor of its threads)."""
    box = tuple(0.375 * v for v in n)
    p = wl.Problem("r1", 3, n, box, wl.DIPOLE_3D, 12, 10, 16, axis=_axis(33))
    eps = 1e-10 if prec == "fp64" else 1e-5
    dt = torch.float64 if prec == "fp64" else torch.float32
    rng = np.random.default_rng(34)
    rho_a = torch.tensor(1e6 * rng.standard_normal(p.n), dtype=dt, device="cuda")
    rho_b = torch.tensor(rng.standard_normal(p.n), dtype=dt, device="cuda")
    used = make_plan(p, eps=eps, precision=prec, interp_tiles=True)
    fresh = make_plan(p, eps=eps, precision=prec, interp_tiles=True)
    try:
        assert used.info["interp_chunk"] == 0  # the interpolation by tiles
        used.potential(rho_a)
        u1, e1 = used.potential(rho_b)
        u2, e2 = fresh.potential(rho_b)
        torch.cuda.synchronize()
        say("reach", prec, "max |u1 - u2| %.3e" % float((u1 - u2).abs().max()))
        assert torch.equal(u1, u2) and float(e1) == float(e2)
    finally:
        used.close()
        fresh.close()
