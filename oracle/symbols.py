"""Jacobian-cancelled symbols S(k) = |k|^{d-1} U^(k).  Oracle: test infrastructure only.

  3D Coulomb   U^ = 1/|k|^2                          (eq. Cou3D)       -> S = 1
  2.5D Coulomb U^ = 1/|k|                            (eq. Cou2D)       -> S = 1
  3D dipole    U^ = -(m.n) + 3 (n.k)(m.k)/|k|^2      (eqs. dipkernelF, dipkerneldF)
                                                     -> S = 3 (n.k)(m.k) - (m.n) |k|^2
  2.5D dipole  U^ = -alpha + 3 [(n_p.k)(m_p.k) - n_3 m_3 |k|^2] / (2 |k|)
                                                     (eqs. dipkernelF2d, dipkernelF2dd)
                                                     -> S = -alpha |k| + (3/2) [(n_p.k)(m_p.k) - n_3 m_3 |k|^2]

  2D Poisson   U = -(1/2pi) log|x|, U^ = 1/|k|^2 (the example after Section 4's
               conclusion of a symbol the Jacobian does not cancel)   -> S = 1/|k|

n and m are unit 3-vectors (the two dipole orientations; m = n for one
orientation), n_p = (n_1, n_2) and m_p = (m_1, m_2) their in-plane parts, alpha
a real constant.  Each S is smooth (Section 3.1, after eq. 3.5; the 2.5D dipole's
-alpha |k| is linear along every ray, which the radial rule integrates exactly)
and is evaluated as written; U^ itself is never formed.  Coefficients of the
weighted sum (3.7): c_j = (2 pi)^{-d} W_j S(k_j).
"""
from __future__ import annotations

import numpy as np

COULOMB_3D = 0
COULOMB_2D = 1
DIPOLE_3D = 2
DIPOLE_2D = 3
POISSON_2D = 4

EULER_GAMMA = 0.57721566490153286061


def symbol(kernel, k, axis=None, axis2=None, alpha=0.0):
    """S(k) at the rows of k.  axis = n, axis2 = m (None: m = n), alpha for the 2.5D dipole."""
    k = np.asarray(k, dtype=np.float64)
    if kernel in (COULOMB_3D, COULOMB_2D):
        return np.ones(k.shape[0])
    if kernel == POISSON_2D:
        kk = np.einsum("ij,ij->i", k, k)
        with np.errstate(divide="ignore"):
            return np.where(kk > 0, 1.0 / np.sqrt(kk), np.inf)
    n = np.asarray(axis, dtype=np.float64)
    m = n if axis2 is None else np.asarray(axis2, dtype=np.float64)
    kk = np.einsum("ij,ij->i", k, k)
    if kernel == DIPOLE_3D:
        return 3.0 * (k @ n) * (k @ m) - float(m @ n) * kk
    if kernel == DIPOLE_2D:
        return -alpha * np.sqrt(kk) + 1.5 * ((k @ n[:2]) * (k @ m[:2]) - n[2] * m[2] * kk)
    raise ValueError("unknown kernel")


def coefficients(kernel, k, W, axis=None, axis2=None, alpha=0.0):
    d = k.shape[1]
    return W * symbol(kernel, k, axis, axis2, alpha) / (2.0 * np.pi) ** d


def origin_coefficient(kernel, K, n_r, radial=0, eps=1e-10):
    """The coefficient c_0 of the node k = 0 (zero for every kernel but the 2D Poisson one).

    For U = -(1/2pi) log|x| the radial integrand g(r)/r, g(r) = int rho^ e^{ik.x} dphi,
    is not integrable at 0; the log kernel fixes its finite part: with
    g(0) = 2 pi rho^(0) and rho^ negligible beyond K,
        u(x) = (2pi)^{-2} [ int_0^K (g(r) - g(0))/r dr + g(0) log K ] + (gamma - log 2)/(2pi) rho^(0),
    the constant from u(0) = gamma/4 for rho = exp(-|x|^2).  The radial integral
    is taken by the Gauss-Legendre rule of the other kernels, the subtracted
    g(0) giving the node at 0:
        sum_a (w_a / r_a) g(r_a) + g(0) (log K - sum_a w_a / r_a),
    exact when g is a polynomial of degree <= 2 n_r (then (g - g(0))/r has
    degree <= 2 n_r - 1).  So c_0 = (log K - sum_a w_a/r_a + gamma - log 2) / (2pi),
    with (r_a, w_a) the radial rule in use (radial, eps: see quadrature.radial_rule),
    and the node adds c_0 rho^(0) = c_0 H sum rho to u everywhere."""
    if kernel != POISSON_2D:
        return 0.0
    from .quadrature import radial_rule
    r, w = radial_rule(K, n_r, radial, eps)
    return (np.log(K) - float(np.sum(w / r)) + EULER_GAMMA - np.log(2.0)) / (2.0 * np.pi)
