"""Fourier-space quadrature nodes and weights (Section 3.1, eqs. 3.5 and 3.7;
Algorithm 1, step 3).  Oracle: test infrastructure only.

The integral (3.3) over the ball |k| <= P is rewritten in spherical (3D) or
polar (2D) coordinates (3.5); the |k|^{d-1} Jacobian is left out of the
weights here and carried by the symbol S(k) = |k|^{d-1} U^(k) (symbols.py),
so that W_j is the weight of the measure dr dtheta dphi (3D, with the sin
theta factor) or dr dphi (2D).

  radial    r: Gauss-Legendre on [0, K]
  polar     theta (3D): Gauss-Legendre on [0, pi] with the sin(theta) factor
            (the literal reading of eq. 3.7), or Gauss-Legendre in cos(theta)
            on [-1, 1] (the same integral after t = cos theta)
  azimuth   phi: trapezoidal rule, phi_l = 2 pi l / N_phi, l = 0..N_phi-1

Node order (the order of every per-node array): radial index slowest, then
theta, then phi fastest.
"""
from __future__ import annotations

import numpy as np

THETA_GL = 0
COSTHETA_GL = 1


def gauss_legendre(n: int):
    """Gauss-Legendre nodes and weights on [-1, 1] (library routine)."""
    s, w = np.polynomial.legendre.leggauss(int(n))
    return s.astype(np.float64), w.astype(np.float64)


def radial_rule(K: float, n_r: int, radial: int = 0, eps: float = 1e-10):
    """r_a = K (1 + s_a)/2, w_a = K omega_a / 2 on [0, K]: Gauss-Legendre
    (radial = 0), or the generalized Gaussian rule of ggq.py for band-limited
    integrands (radial = 1) at accuracy eps."""
    if radial == 1:
        from .ggq import radial_rule_ggq
        return radial_rule_ggq(K, n_r, eps)
    s, w = gauss_legendre(n_r)
    return 0.5 * K * (1.0 + s), 0.5 * K * w


def theta_rule(n_theta: int, rule: int = THETA_GL):
    """Returns (cos theta_b, sin theta_b, w_b) with w_b the weight of sin(theta) dtheta."""
    s, w = gauss_legendre(n_theta)
    if rule == THETA_GL:
        th = 0.5 * np.pi * (1.0 + s)
        return np.cos(th), np.sin(th), 0.5 * np.pi * w * np.sin(th)
    if rule == COSTHETA_GL:
        return s.copy(), np.sqrt((1.0 - s) * (1.0 + s)), w.copy()
    raise ValueError("unknown theta rule")


def phi_rule(n_phi: int):
    """Trapezoidal rule on the periodic interval [0, 2 pi)."""
    l = np.arange(int(n_phi), dtype=np.float64)
    return 2.0 * np.pi * l / n_phi, np.full(int(n_phi), 2.0 * np.pi / n_phi)


def spherical_nodes(K, n_r, n_theta, n_phi, rule=THETA_GL, radial=0, eps=1e-10):
    """k_j = r (sin th cos ph, sin th sin ph, cos th), W_j = w_r w_th w_ph.  Shapes (M,3), (M,)."""
    r, wr = radial_rule(K, n_r, radial, eps)
    ct, st, wt = theta_rule(n_theta, rule)
    ph, wp = phi_rule(n_phi)
    R = r[:, None, None]
    k1 = R * st[None, :, None] * np.cos(ph)[None, None, :]
    k2 = R * st[None, :, None] * np.sin(ph)[None, None, :]
    k3 = R * ct[None, :, None] * np.ones(n_phi)[None, None, :]
    W = wr[:, None, None] * wt[None, :, None] * wp[None, None, :]
    k = np.stack([k1.ravel(), k2.ravel(), k3.ravel()], axis=1)
    return k, W.ravel()


def polar_nodes(K, n_r, n_phi, radial=0, eps=1e-10):
    """k_j = r (cos ph, sin ph), W_j = w_r w_ph.  Shapes (M,2), (M,)."""
    r, wr = radial_rule(K, n_r, radial, eps)
    ph, wp = phi_rule(n_phi)
    k1 = r[:, None] * np.cos(ph)[None, :]
    k2 = r[:, None] * np.sin(ph)[None, :]
    W = wr[:, None] * wp[None, :]
    return np.stack([k1.ravel(), k2.ravel()], axis=1), W.ravel()


def default_kmax(n, box):
    """K = pi / max_j h_j: the largest radius whose ball stays inside the
    trapezoid rule's alias-free band |k_j| <= pi / h_j (the cutoff P of eq. 3.3)."""
    return np.pi / max(float(R) / int(N) for N, R in zip(n, box))


def fourier_nodes(problem):
    """Nodes and weights of a workloads.Problem."""
    K = problem.kmax if problem.kmax > 0 else default_kmax(problem.n, problem.box)
    radial = getattr(problem, "radial", 0)
    if problem.dim == 3:
        return spherical_nodes(K, problem.n_r, problem.n_theta, problem.n_phi, problem.theta_rule, radial, problem.eps)
    return polar_nodes(K, problem.n_r, problem.n_phi, radial, problem.eps)
