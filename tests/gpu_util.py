"""Helpers shared by the GPU tests: build a plan for a workloads.Problem and
compare with the oracle."""
import sys

import numpy as np

import workloads as wl


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# the plan's tap-kernel forms: the staged interpolation and the gather over
# all three axes (the defaults), the interpolation by tiles, the spreading by
# rings, and both
MODES = {"staged": {}, "tiles": {"interp_tiles": True}, "rings": {"spread_rings": True},
         "tiles+rings": {"interp_tiles": True, "spread_rings": True}}


def make_plan(problem, **kw):
    import paper_1311_4120_amd as jgb
    nodes = (problem.n_r, problem.n_theta, problem.n_phi) if problem.dim == 3 else (problem.n_r, problem.n_phi)
    kernel = {wl.COULOMB_3D: "coulomb3d", wl.COULOMB_2D: "coulomb2d", wl.DIPOLE_3D: "dipole3d",
              wl.DIPOLE_2D: "dipole2d", wl.POISSON_2D: "poisson2d"}[problem.kernel]
    args = dict(eps=problem.eps, precision="fp64" if problem.precision == wl.FP64 else "mixed",
                lam=problem.lam, axis=problem.axis, theta_rule="theta" if problem.theta_rule == wl.THETA_GL else "costheta",
                kmax=problem.kmax, axis2=problem.axis2, alpha=problem.alpha)
    args.update(kw)
    return jgb.Plan(problem.n, problem.box, kernel, nodes, **args)


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def half_index(problem):
    """Natural indices (into the oracle's full node order) of the device's half node set."""
    nph = problem.n_phi
    if problem.dim == 3:
        a, b, l = np.meshgrid(np.arange(problem.n_r), np.arange(problem.n_theta), np.arange(nph // 2), indexing="ij")
        return ((a * problem.n_theta + b) * nph + l).ravel()
    a, l = np.meshgrid(np.arange(problem.n_r), np.arange(nph // 2), indexing="ij")
    return (a * nph + l).ravel()


def load_sampled(name):
    """The oracle's values at sampled outputs of a large workload (written by
    tests/golden/make_sampled.py, which calls only the oracle)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sampled_%s.npz" % name)
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def sampled_errors(u, ref):
    """u (the whole grid, numpy) against the sampled oracle values: the random
    sub-lattice, the three axis lines through the centre and the random points.
    Returns (rel-L2 over all samples, max error / max |u| of the grid, sample count)."""
    got, want = [], []
    lat = (ref["lattice0"], ref["lattice1"], ref["lattice2"])
    got.append(u[np.ix_(*lat)].ravel())
    want.append(ref["u_lattice"].ravel())
    c = ref["center"]
    got += [u[:, c[1], c[2]], u[c[0], :, c[2]], u[c[0], c[1], :]]
    want += [ref["u_line0"], ref["u_line1"], ref["u_line2"]]
    got.append(u[tuple(ref["points"].T)])
    want.append(ref["u_points"])
    g = np.concatenate(got)
    w = np.concatenate(want)
    return rel_l2(g, w), float(np.max(np.abs(g - w)) / np.max(np.abs(u))), g.size
