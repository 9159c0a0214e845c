"""The stored oracle values at sampled outputs of the large workloads
(tests/golden/sampled_*.npz, written by tests/golden/make_sampled.py from the
oracle alone) agree with the oracle recomputed here at a few of them, so the
files cannot drift from the oracle or the seeded inputs.  CPU only."""
import os
import sys

import numpy as np

import oracle
import workloads as wl

sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
import make_sampled  # noqa: E402
from gpu_util import load_sampled  # noqa: E402


def _check_points(name, p, coefs, factors, npts=4):
    ref = load_sampled(name)
    assert tuple(ref["n"]) == tuple(p.n)
    k, W = oracle.fourier_nodes(p)
    c = oracle.coefficients(p.kernel, k, W, p.axis, p.axis2, p.alpha)
    rh = oracle.rho_hat_separable_sum(coefs, factors, p.box, k)
    assert abs(oracle.energy_fourier(c, rh, p.lam) / float(ref["energy"]) - 1) < 1e-13
    up = oracle.sum_to_points(c * rh, k, p.n, p.box, ref["points"][:npts]).real
    scale = np.max(np.abs(ref["u_line0"]))
    assert np.max(np.abs(up - ref["u_points"][:npts])) < 1e-13 * scale
    # a sub-lattice point and a centre-line point through the general point sum
    lat = [ref["lattice%d" % a] for a in range(3)]
    c0 = ref["center"]
    idx = np.array([[lat[0][3], lat[1][5], lat[2][7]], [7, c0[1], c0[2]]])
    up = oracle.sum_to_points(c * rh, k, p.n, p.box, idx).real
    assert abs(up[0] - ref["u_lattice"][3, 5, 7]) < 1e-13 * scale
    assert abs(up[1] - ref["u_line0"][7]) < 1e-13 * scale


def test_headline_sampled_values():
    p, rho = wl.dipole3d_128()
    x = wl.grid_axes(p.n, p.box)
    f = [np.exp(-x[0] ** 2), np.exp(-x[1] ** 2 / 1.5 ** 2), np.exp(-x[2] ** 2 / 0.7 ** 2)]
    _check_points("dipole3d_128", p, np.array([1.0 + 0j]), [f])


def test_batched_member_sampled_values():
    members = wl.batched_coulomb()
    assert make_sampled.batched_members() == [7, 3, 0, 1]
    p, mix = members[7]
    coefs, factors = mix.density_terms(p.n, p.box)
    _check_points("batched_coulomb_7", p, coefs, factors)
    for i in (3, 0, 1):
        assert tuple(load_sampled("batched_coulomb_%d" % i)["n"]) == members[i][0].n


def test_wave_packet_transform_samples():
    p, packets = wl.dipole_grad_256()
    ref = load_sampled("dipole_grad_256")
    k, W = oracle.fourier_nodes(p)
    hi = make_sampled.half_index(p)
    sel = ref["half_sel"][:: 256]
    coefs, factors = packets.density_terms(p.n, p.box)
    rh = oracle.rho_hat_separable_sum(coefs, factors, p.box, k[hi[sel]])
    want = ref["rhohat_half"][:: 256]
    assert np.max(np.abs(rh - want)) < 1e-13 * np.max(np.abs(ref["rhohat_half"]))
