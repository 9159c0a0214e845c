"""Jacobian-cancelled symbols S(k) = |k|^{d-1} U^(k).  Oracle: test infrastructure only.

  3D Coulomb   U^ = 1/|k|^2                (eq. Cou3D)     -> S = 1
  2.5D Coulomb U^ = 1/|k|                  (eq. Cou2D)     -> S = 1
  3D dipole    U^ = -1 + 3 (n.k)^2/|k|^2   (eq. dipkernelF) -> S = 3 (n.k)^2 - |k|^2

The product is smooth (Section 3.1, after eq. 3.5), so S is evaluated as the
polynomial it is; U^ itself is never formed.  Coefficients of the weighted sum
(3.7): c_j = (2 pi)^{-d} W_j S(k_j).
"""
from __future__ import annotations

import numpy as np

COULOMB_3D = 0
COULOMB_2D = 1
DIPOLE_3D = 2


def symbol(kernel, k, axis=None):
    k = np.asarray(k, dtype=np.float64)
    if kernel in (COULOMB_3D, COULOMB_2D):
        return np.ones(k.shape[0])
    if kernel == DIPOLE_3D:
        n = np.asarray(axis, dtype=np.float64)
        nk = k @ n
        return 3.0 * nk * nk - np.einsum("ij,ij->i", k, k)
    raise ValueError("unknown kernel")


def coefficients(kernel, k, W, axis=None):
    d = k.shape[1]
    return W * symbol(kernel, k, axis) / (2.0 * np.pi) ** d
