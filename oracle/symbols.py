"""Jacobian-cancelled symbols S(k) = |k|^{d-1} U^(k).  Oracle: test infrastructure only.

  3D Coulomb   U^ = 1/|k|^2                          (eq. Cou3D)       -> S = 1
  2.5D Coulomb U^ = 1/|k|                            (eq. Cou2D)       -> S = 1
  3D dipole    U^ = -(m.n) + 3 (n.k)(m.k)/|k|^2      (eqs. dipkernelF, dipkerneldF)
                                                     -> S = 3 (n.k)(m.k) - (m.n) |k|^2
  2.5D dipole  U^ = -alpha + 3 [(n_p.k)(m_p.k) - n_3 m_3 |k|^2] / (2 |k|)
                                                     (eqs. dipkernelF2d, dipkernelF2dd)
                                                     -> S = -alpha |k| + (3/2) [(n_p.k)(m_p.k) - n_3 m_3 |k|^2]

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


def symbol(kernel, k, axis=None, axis2=None, alpha=0.0):
    """S(k) at the rows of k.  axis = n, axis2 = m (None: m = n), alpha for the 2.5D dipole."""
    k = np.asarray(k, dtype=np.float64)
    if kernel in (COULOMB_3D, COULOMB_2D):
        return np.ones(k.shape[0])
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
