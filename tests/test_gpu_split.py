"""GPU parity of Algorithm 2 (JGB_FLAG_SPLIT, Section 3.3) against the oracle's
`split.potential_split`, through the C ABI:

  * u, the physical-side E and the Fourier-side E (jgb_energy) for the three
    kernels, in float64 (eps = 1e-10) and mixed precision (eps = 1e-5), on
    grids of several tiles with unequal, non-power-of-two sides;
  * the plan's window and I2 cut-off equal the oracle's defaults; the node
    coefficients carry the window;
  * rho^ at I2's nodes (jgb_transform), the backward product (A symmetric);
  * explicit windows and cut-offs, a window so wide that I2's ball reaches
    pi / max h, the smallest grid, a zero density;
  * a 128^3 dipole at the default window, checked on sampled points.
"""
import numpy as np
import pytest

import oracle
import workloads as wl
from oracle import split
from gpu_util import MODES, half_index, make_plan, rel_l2, say

pytestmark = pytest.mark.gpu
import torch  # noqa: E402


def _axis(seed):
    return tuple(wl.unit_vector(np.random.default_rng(seed)))


def _rho(p, seed=5, count=3):
    rng = np.random.default_rng(seed)
    lo = -0.15 * min(p.box)
    mix = wl.random_mixture(rng, count, p.dim, lo, -lo, 0.07 * min(p.box) + 0.2, 0.1 * min(p.box) + 0.4)
    return mix.evaluate(p.n, p.box)


def _par(p, window):
    if window is None or all(w == 0 for w in window):
        return split.default_window(p.n, p.box)
    return {"a": window[0]} if p.dim == 3 else {"R0": window[0], "R1": window[1]}


CASES = {
    "coulomb3d": (wl.Problem("s1", 3, (24, 20, 16), (12.0, 10.0, 8.0), wl.COULOMB_3D, 16, 12, 16), None),
    "dipole3d": (wl.Problem("s2", 3, (20, 24, 18), (10.0, 12.0, 9.0), wl.DIPOLE_3D, 16, 12, 16,
                            axis=_axis(41)), None),
    "coulomb2d": (wl.Problem("s3", 2, (64, 48), (16.0, 12.0), wl.COULOMB_2D, 24, 1, 32), None),
    "dipole3d_costheta": (wl.Problem("s4", 3, (16, 16, 20), (8.0, 8.0, 10.0), wl.DIPOLE_3D, 14, 10, 14,
                                     theta_rule=wl.COSTHETA_GL, axis=_axis(42)), None),
    # explicit window and a cut-off below the default
    "coulomb3d_window": (wl.Problem("s5", 3, (16, 24, 20), (8.0, 12.0, 10.0), wl.COULOMB_3D, 14, 10, 14,
                                    kmax=2.5), (0.9, 0.0)),
    "coulomb2d_window": (wl.Problem("s6", 2, (40, 50), (10.0, 12.5), wl.COULOMB_2D, 20, 1, 28), (0.4, 3.5)),
    # a window so wide that I2's ball is the whole alias-free ball pi / max h
    "dipole3d_wide": (wl.Problem("s7", 3, (16, 16, 16), (8.0, 8.0, 8.0), wl.DIPOLE_3D, 16, 12, 16,
                                 axis=_axis(43)), (60.0, 0.0)),
    # the smallest grid
    "coulomb3d_min": (wl.Problem("s8", 3, (8, 8, 8), (6.0, 6.0, 6.0), wl.COULOMB_3D, 6, 4, 6), None),
}

_REF = {}


def _oracle(name):
    if name not in _REF:
        p, window = CASES[name]
        rho = _rho(p)
        par = _par(p, window)
        u, i1, i2, E = split.potential_split(p, rho, par)
        _REF[name] = (rho, par, u, E)
    return _REF[name]


def _plan(p, window, eps, prec, mode="staged"):
    return make_plan(p, eps=eps, precision=prec, split=True, window=window or (0.0, 0.0), **MODES[mode])


def _rings_fit(p):
    # the spreading by rings needs every oversampled side >= its tile (16, 8,
    # 16) + w - 1, w = 12 at eps = 1e-10
    return p.dim == 3 and 2 * p.n[0] >= 27 and 2 * p.n[1] >= 19 and 2 * p.n[2] >= 27


# every case with the staged interpolation and the three-axis gather; the 3D
# ones also with the interpolation by tiles, and with the spreading by rings
# where their grids allow it
VARIANTS = ([(n, "staged") for n in CASES] + [(n, "tiles") for n in CASES if CASES[n][0].dim == 3]
            + [(n, "rings") for n in CASES if _rings_fit(CASES[n][0])])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("name,mode", VARIANTS)
def test_split_matches_oracle(name, mode, prec):
    p, window = CASES[name]
    rho, par, u_ref, E_ref = _oracle(name)
    eps = 1e-10 if prec == "fp64" else 1e-5
    say("split", name, prec, "grid", p.n, "nodes", (p.n_r, p.n_theta, p.n_phi), "window", par, mode)
    plan = _plan(p, window, eps, prec, mode)
    K2 = p.kmax if p.kmax > 0 else split.default_cutoff(p.n, p.box, par)
    assert plan.info["kmax"] == pytest.approx(K2, rel=1e-14)
    want = (par["a"], 0.0) if p.dim == 3 else (par["R0"], par["R1"])
    assert plan.info["window"] == pytest.approx(list(want), rel=1e-14)
    dt = torch.float64 if prec == "fp64" else torch.float32
    rt = torch.tensor(rho, dtype=dt, device="cuda")
    u, E = plan.potential(rt)
    Ef = plan.energy(rt)
    e = rel_l2(u.cpu().numpy(), u_ref)
    scale = 0.5 * p.lam * np.prod([b / m for b, m in zip(p.box, p.n)]) * float(np.sum(np.abs(rho * u_ref)))
    eE = abs(E.item() - E_ref) / scale
    eEf = abs(Ef.item() - E_ref) / scale
    say("   relL2(u) %.2e  E %.2e  E_F %.2e" % (e, eE, eEf))
    assert e < eps and eE < eps and eEf < eps
    plan.close()


@pytest.mark.parametrize("name", ["coulomb3d", "dipole3d", "coulomb2d"])
def test_split_nodes_transform_and_backward(name):
    p, window = CASES[name]
    rho, par, u_ref, _ = _oracle(name)
    plan = _plan(p, window, 1e-10, "fp64")
    q = p if p.kmax > 0 else wl.Problem(**{**p.__dict__, "kmax": split.default_cutoff(p.n, p.box, par)})
    k, W = oracle.fourier_nodes(q)
    c_ref = split.i2_coefficients(p.kernel, k, W, par, p.axis)
    kg, wg, cg = plan.nodes()
    assert np.max(np.abs(kg.cpu().numpy() - k)) < 1e-12 * np.max(np.abs(k))
    assert np.max(np.abs(cg.cpu().numpy() - c_ref)) < 1e-13 * np.max(np.abs(c_ref))
    rt = torch.tensor(rho, dtype=torch.float64, device="cuda")
    th = plan.transform(rt).cpu().numpy()
    ref = oracle.rho_hat(rho, p.box, k)[half_index(q)]
    et = np.max(np.abs(th - ref)) / np.max(np.abs(ref))
    # the backward product applies the same symmetric operator
    g = _rho(p, seed=17)
    gb = plan.backward(torch.tensor(g, dtype=torch.float64, device="cuda")).cpu().numpy()
    gref = split.potential_split(p, g, par)[0]
    eb = rel_l2(gb, gref)
    say("split", name, "transform %.2e backward %.2e" % (et, eb))
    assert et < 1e-10 and eb < 1e-10
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_split_zero_density(prec):
    p, window = CASES["dipole3d"]
    plan = _plan(p, window, 1e-10 if prec == "fp64" else 1e-5, prec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    z = torch.zeros(p.n, dtype=dt, device="cuda")
    u, E = plan.potential(z)
    assert torch.count_nonzero(u).item() == 0 and E.item() == 0.0
    assert plan.energy(z).item() == 0.0
    plan.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_split_dipole128_sampled(prec):
    """The 128^3 dipole density at the default window and I2 cut-off, with a
    node set that resolves I2 (40 x 32 x 64 nodes): u at 400 sampled points
    against the oracle's full-grid I1 (an FFT) plus I2 summed at those points,
    and E against the Fourier-side sum."""
    p0, rho = wl.dipole3d_128()
    p = wl.Problem("s128", 3, p0.n, p0.box, wl.DIPOLE_3D, 40, 32, 64, axis=p0.axis)
    eps = 1e-10 if prec == "fp64" else 1e-5
    par = split.default_window(p.n, p.box)
    q = wl.Problem(**{**p.__dict__, "kmax": split.default_cutoff(p.n, p.box, par)})
    say("split dipole 128^3", prec, "K2 %.4f" % q.kmax)
    plan = _plan(p, None, eps, prec)
    dt = torch.float64 if prec == "fp64" else torch.float32
    u, E = plan.potential(torch.tensor(rho, dtype=dt, device="cuda"))
    u = u.cpu().numpy()
    i1 = split.i1_fft(rho, p.box, p.kernel, par, p.axis)
    k, W = oracle.fourier_nodes(q)
    c = split.i2_coefficients(p.kernel, k, W, par, p.axis)
    x = wl.grid_axes(p.n, p.box)
    f = [np.exp(-x[0] ** 2 / 1.0), np.exp(-x[1] ** 2 / 1.5 ** 2), np.exp(-x[2] ** 2 / 0.7 ** 2)]
    assert np.allclose(f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :], rho, rtol=0, atol=1e-15)
    rh = oracle.rho_hat_separable(f, p.box, k)
    rng = np.random.default_rng(7)
    idx = np.stack([rng.integers(0, m, 400) for m in p.n], axis=1)
    ref = i1[tuple(idx.T)] + np.real(oracle.sum_to_points(c * rh, k, p.n, p.box, idx))
    e = rel_l2(u[tuple(idx.T)], ref)
    E_ref = split.energy_split_fourier(q, rho, par, rh=rh)
    eE = abs(E.item() - E_ref) / abs(E_ref)
    say("   sampled relL2(u) %.2e  E %.2e" % (e, eE))
    assert e < eps and eE < eps
    plan.close()


@pytest.mark.parametrize("name", ["dipole3d", "coulomb2d"])
def test_split_calls_interleave(name):
    """The potential path (forward passes but the last, paired unmix, fused
    first inverse pass) and the energy and transform paths (full forward
    spectrum, separate unmix) share the plan's grids: a potential after an
    energy and a transform call equals the first potential bit for bit."""
    p, window = CASES[name]
    rho = _rho(p)
    plan = _plan(p, window, 1e-10, "fp64")
    rt = torch.tensor(rho, dtype=torch.float64, device="cuda")
    u1, E1 = plan.potential(rt)
    u1 = u1.clone()
    plan.energy(rt)
    plan.transform(rt)
    u2, E2 = plan.potential(rt)
    torch.cuda.synchronize()
    say("split interleaved calls", name, "max |u2 - u1| %.1e" % (u2 - u1).abs().max().item())
    assert torch.equal(u1, u2) and E1.item() == E2.item()
    plan.close()
