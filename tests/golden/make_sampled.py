"""Write the oracle's values at sampled outputs of the large workloads to
tests/golden/sampled_<name>.npz, for the GPU parity tests at full size.

Calls only oracle/ and workloads/: the transform of eq. 3.2 at every node
(exactly, by the separable-term regrouping of the density), the weights and
symbol of eq. 3.7, the Fourier-side energy, and the type-1 sum of eq. 3.7 at

  * a random sub-lattice: 16 distinct random indices per axis (4096 points),
  * the three axis lines through the grid centre,
  * 512 independent random grid points,

plus (dipole_grad_256) the transform at 4096 random nodes of the half node set
(phi index < n_phi / 2) that the library keeps.

Usage: python tests/golden/make_sampled.py [name ...]   (default: all)
The node range of each sum is split over a process pool; the parts are
partial sums of the same finite sums, added in a fixed order.
"""
import os
import sys
import time
from multiprocessing import get_context

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as wl  # noqa: E402

_G = {}   # inherited by the forked workers


def _rho_hat_part(rng):
    s, e = rng
    return oracle.rho_hat_separable_sum(_G["coefs"], _G["factors"], _G["box"], _G["k"][s:e])


def _lattice_part(args):
    (s, e), lists = args
    return oracle.sum_to_lattice(_G["v"][s:e], _G["k"][s:e], _G["n"], _G["box"], lists)


def _points_part(args):
    (s, e), idx = args
    return oracle.sum_to_points(_G["v"][s:e], _G["k"][s:e], _G["n"], _G["box"], idx)


def _ranges(M, parts):
    b = np.linspace(0, M, parts + 1).astype(np.int64)
    return [(int(b[i]), int(b[i + 1])) for i in range(parts)]


def half_index(p):
    """Natural indices (into the oracle's node order) of the half node set, phi index < n_phi / 2."""
    a, b, l = np.meshgrid(np.arange(p.n_r), np.arange(p.n_theta), np.arange(p.n_phi // 2), indexing="ij")
    return ((a * p.n_theta + b) * p.n_phi + l).ravel()


def sample(name, p, coefs, factors, seed, half_nodes=0, procs=8):
    t0 = time.time()
    k, W = oracle.fourier_nodes(p)
    c = oracle.coefficients(p.kernel, k, W, p.axis, p.axis2, p.alpha)
    M = k.shape[0]
    _G.update(k=k, coefs=coefs, factors=factors, box=p.box, n=p.n)
    parts = _ranges(M, 4 * procs)
    ctx = get_context("fork")
    with ctx.Pool(procs) as pool:
        rh = np.concatenate(pool.map(_rho_hat_part, parts))
    print("  %s: transform at %d nodes, %.1f s" % (name, M, time.time() - t0), flush=True)
    v = c * rh
    _G["v"] = v
    E = oracle.energy_fourier(c, rh, p.lam)
    rng = np.random.default_rng(seed)
    lat = [np.sort(rng.choice(N, 16, replace=False)) for N in p.n]
    ctr = [N // 2 for N in p.n]
    lines = []
    for a in range(3):
        li = [np.array([ctr[b]]) for b in range(3)]
        li[a] = np.arange(p.n[a])
        lines.append(li)
    pts = np.stack([rng.integers(0, N, 512) for N in p.n], axis=1)
    with ctx.Pool(procs) as pool:
        u_lat = sum(pool.map(_lattice_part, [(r, lat) for r in parts])).real
        u_lines = [sum(pool.map(_lattice_part, [(r, li) for r in parts])).real.ravel() for li in lines]
        u_pts = sum(pool.map(_points_part, [(r, pts) for r in parts])).real
    out = dict(name=name, n=np.array(p.n), n_nodes=np.array([p.n_r, p.n_theta, p.n_phi]), energy=E,
               lattice0=lat[0], lattice1=lat[1], lattice2=lat[2], u_lattice=u_lat,
               u_line0=u_lines[0], u_line1=u_lines[1], u_line2=u_lines[2], center=np.array(ctr),
               points=pts, u_points=u_pts)
    if half_nodes:
        hi = half_index(p)
        sel = np.sort(rng.choice(hi.size, half_nodes, replace=False))
        out.update(half_sel=sel, rhohat_half=rh[hi[sel]])
    path = os.path.join(HERE, "sampled_%s.npz" % name)
    np.savez_compressed(path, **out)
    print("  wrote %s (%.1f s, E = %.15e)" % (path, time.time() - t0, E), flush=True)


def dipole3d_128():
    p, rho = wl.dipole3d_128()
    x = wl.grid_axes(p.n, p.box)
    f = [np.exp(-x[0] ** 2 / 1.0 ** 2), np.exp(-x[1] ** 2 / 1.5 ** 2), np.exp(-x[2] ** 2 / 0.7 ** 2)]
    assert np.max(np.abs(f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :] - rho)) < 1e-15
    sample("dipole3d_128", p, np.array([1.0 + 0j]), [f], seed=301)


def dipole_grad_256():
    p, packets = wl.dipole_grad_256()
    coefs, factors = packets.density_terms(p.n, p.box)
    sample("dipole_grad_256", p, coefs, factors, seed=501, half_nodes=4096)


def batched_members():
    """The first member of each grid size of the 64-density batch."""
    members = wl.batched_coulomb()
    seen = {}
    for i, (p, mix) in enumerate(members):
        seen.setdefault(p.n[0], i)
    return [seen[N] for N in sorted(seen)]


def batched_coulomb():
    members = wl.batched_coulomb()
    for i in batched_members():
        p, mix = members[i]
        coefs, factors = mix.density_terms(p.n, p.box)
        sample("batched_coulomb_%d" % i, p, coefs, factors, seed=400 + i)


JOBS = {"dipole3d_128": dipole3d_128, "dipole_grad_256": dipole_grad_256, "batched_coulomb": batched_coulomb}

if __name__ == "__main__":
    names = sys.argv[1:] or list(JOBS)
    for nm in names:
        JOBS[nm]()
