"""Helpers shared by the GPU tests: build a plan for a workloads.Problem and
compare with the oracle."""
import sys

import numpy as np

import workloads as wl


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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
