"""Direct (no NUFFT) evaluation of the discrete potential and energy.
Oracle: test infrastructure only.

Definitions, all in FP64, on the grid x_n = -R_j/2 + n_j h_j, h_j = R_j/N_j,
n_j = 0..N_j-1, H = prod_j h_j:

  rho^_j = H sum_n rho_n exp(-i k_j . x_n)               trapezoid rule, eq. 3.2
  u_n    = Re sum_j c_j rho^_j exp(+i k_j . x_n)          quadrature (3.7) of (3.5)
  E      = (lambda/2) H sum_n rho_n u_n                   energy remark after Alg. 2
         = (lambda/2) sum_j c_j |rho^_j|^2                (substitute rho^, rho real)

with c_j = (2 pi)^{-d} W_j S(k_j) (symbols.py) and the nodes of quadrature.py.
These are Algorithm 1's steps 4 and 5 evaluated as plain sums: O(N M) work.

The exponential factorises over axes, exp(-i k.x) = prod_j exp(-i k_j x_j), so
each sum is taken as a matrix product over the first axis followed by
elementwise products with the other axes' phase tables.  That is a
regrouping of the same finite sum, not an approximation.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .quadrature import fourier_nodes, default_kmax
from .symbols import coefficients, origin_coefficient

_CHUNK_ELEMS = 1 << 23   # complex elements per intermediate block (128 MB)


def _axes(n, box):
    return [-0.5 * float(R) + np.arange(int(N), dtype=np.float64) * (float(R) / int(N))
            for N, R in zip(n, box)]


def _cell_volume(n, box):
    return float(np.prod([float(R) / int(N) for N, R in zip(n, box)]))


def rho_hat(rho, box, k):
    """Type-2 sum rho^_j = H sum_n rho_n exp(-i k_j . x_n) at every node (eq. 3.2)."""
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.shape
    d = rho.ndim
    x = _axes(n, box)
    H = _cell_volume(n, box)
    k = np.asarray(k, dtype=np.float64)
    M = k.shape[0]
    out = np.empty(M, dtype=np.complex128)
    rest = int(np.prod(n[1:]))
    B = max(1, _CHUNK_ELEMS // max(rest, 1))
    flat = rho.reshape(n[0], rest)
    for s in range(0, M, B):
        kb = k[s:s + B]
        P = [np.exp(-1j * np.outer(kb[:, j], x[j])) for j in range(d)]
        T = P[0] @ flat                                   # (B, N2[*N3])
        if d == 2:
            out[s:s + B] = np.einsum("bj,bj->b", T, P[1])
        else:
            T = T.reshape(kb.shape[0], n[1], n[2])
            T2 = np.einsum("bjk,bj->bk", T, P[1])
            out[s:s + B] = np.einsum("bk,bk->b", T2, P[2])
    return H * out


def rho_hat_separable(factors, box, k):
    """rho^_j for a separable density rho_n = prod_i f_i[n_i] (f_i the per-axis samples).

    The trapezoid sum of eq. 3.2 factorises exactly into one 1D sum per axis,
    rho^_j = H prod_i sum_{n_i} f_i[n_i] exp(-i k_{j,i} x_{n_i}): O(M sum_i N_i)
    instead of O(M N).  Used at grid sizes where the general sum is too slow."""
    k = np.asarray(k, dtype=np.float64)
    n = [len(f) for f in factors]
    x = _axes(n, box)
    H = _cell_volume(n, box)
    M = k.shape[0]
    out = np.empty(M, dtype=np.complex128)
    B = max(1, _CHUNK_ELEMS // max(n))
    for s in range(0, M, B):
        kb = k[s:s + B]
        acc = np.ones(kb.shape[0], dtype=np.complex128)
        for i, f in enumerate(factors):
            acc *= np.exp(-1j * np.outer(kb[:, i], x[i])) @ np.asarray(f, dtype=np.float64)
        out[s:s + B] = acc
    return H * out


def rho_hat_separable_sum(coefs, factors, box, k):
    """rho^_j for a density given as a finite sum of separable terms,
    rho_n = sum_t coef_t prod_i f_{t,i}[n_i], the factors complex in general
    (rho = |psi|^2 of a sum of Gaussian wave packets is such a sum; the total is
    real).  By linearity of eq. 3.2 and the per-axis factorisation of the
    exponential, rho^_j = H sum_t coef_t prod_i sum_{n_i} f_{t,i}[n_i]
    exp(-i k_{j,i} x_{n_i}), which is what is evaluated: one phase table per
    axis, contracted with every term's factor on that axis."""
    k = np.asarray(k, dtype=np.float64)
    coefs = np.asarray(coefs, dtype=np.complex128)
    d = len(factors[0])
    n = [len(f) for f in factors[0]]
    x = _axes(n, box)
    H = _cell_volume(n, box)
    F = [np.stack([np.asarray(ft[i], dtype=np.complex128) for ft in factors], axis=1) for i in range(d)]  # (N_i, T)
    M = k.shape[0]
    out = np.empty(M, dtype=np.complex128)
    B = max(1, _CHUNK_ELEMS // max(max(n), len(coefs)))
    for s in range(0, M, B):
        kb = k[s:s + B]
        acc = np.ones((kb.shape[0], len(coefs)), dtype=np.complex128)
        for i in range(d):
            acc *= np.exp(-1j * np.outer(kb[:, i], x[i])) @ F[i]
        out[s:s + B] = acc @ coefs
    return H * out


def sum_to_grid(v, k, n, box):
    """Type-1 sum f_n = sum_j v_j exp(+i k_j . x_n) on the whole grid (complex)."""
    v = np.asarray(v, dtype=np.complex128)
    k = np.asarray(k, dtype=np.float64)
    d = len(n)
    x = _axes(n, box)
    rest = int(np.prod(n[1:]))
    out = np.zeros((int(n[0]), rest), dtype=np.complex128)
    M = k.shape[0]
    B = max(1, _CHUNK_ELEMS // max(rest, 1))
    for s in range(0, M, B):
        kb = k[s:s + B]
        P = [np.exp(1j * np.outer(kb[:, j], x[j])) for j in range(d)]
        if d == 2:
            Q = v[s:s + B, None] * P[1]
        else:
            Q = (v[s:s + B, None, None] * P[1][:, :, None] * P[2][:, None, :]).reshape(kb.shape[0], rest)
        out += P[0].T @ Q
    return out.reshape(tuple(int(t) for t in n))


def sum_to_points(v, k, n, box, index):
    """f_s = sum_j v_j exp(+i k_j . x_{n_s}) at selected grid points.

    index: integer array (S, d) of grid indices."""
    v = np.asarray(v, dtype=np.complex128)
    k = np.asarray(k, dtype=np.float64)
    index = np.asarray(index, dtype=np.int64)
    d = len(n)
    x = _axes(n, box)
    X = np.stack([x[j][index[:, j]] for j in range(d)], axis=1)   # (S, d) coordinates
    S = index.shape[0]
    out = np.zeros(S, dtype=np.complex128)
    M = k.shape[0]
    B = max(1, _CHUNK_ELEMS // max(S, 1))
    for s in range(0, M, B):
        out += v[s:s + B] @ np.exp(1j * (k[s:s + B] @ X.T))
    return out


def sum_to_lattice(v, k, n, box, index_lists):
    """Type-1 sum f = sum_j v_j exp(+i k_j . x) at the product set of grid
    indices index_lists[0] x index_lists[1] (x index_lists[2]): the sum of
    sum_to_grid restricted to a subset of the grid (a sub-lattice, or a line
    when the other lists have one index), with the same per-axis phase tables.
    Returns an array of shape (len(index_lists[0]), len(index_lists[1]), ...)."""
    v = np.asarray(v, dtype=np.complex128)
    k = np.asarray(k, dtype=np.float64)
    d = len(n)
    ax = _axes(n, box)
    x = [ax[j][np.asarray(index_lists[j], dtype=np.int64)] for j in range(d)]
    L = [len(xj) for xj in x]
    rest = int(np.prod(L[1:]))
    out = np.zeros((L[0], rest), dtype=np.complex128)
    M = k.shape[0]
    B = max(1, _CHUNK_ELEMS // max(rest, max(L), 1))
    for s in range(0, M, B):
        kb = k[s:s + B]
        P = [np.exp(1j * np.outer(kb[:, j], x[j])) for j in range(d)]
        if d == 2:
            Q = v[s:s + B, None] * P[1]
        else:
            Q = (v[s:s + B, None, None] * P[1][:, :, None] * P[2][:, None, :]).reshape(kb.shape[0], rest)
        out += P[0].T @ Q
    return out.reshape(tuple(L))


def energy_fourier(c, rhohat, lam):
    return 0.5 * lam * float(np.sum(c * (rhohat.real ** 2 + rhohat.imag ** 2)))


def energy_physical(rho, u, box, lam):
    return 0.5 * lam * _cell_volume(rho.shape, box) * float(np.sum(rho * u))


def potential(rho, box, kernel, k, W, axis=None, axis2=None, alpha=0.0):
    """u = Re sum_j c_j rho^_j exp(i k_j.x_n); returns (u, rho^, c, max|Im|)."""
    c = coefficients(kernel, k, W, axis, axis2, alpha)
    rh = rho_hat(rho, box, k)
    f = sum_to_grid(c * rh, k, rho.shape, box)
    return f.real.copy(), rh, c, float(np.max(np.abs(f.imag))) if f.size else 0.0


def apply_operator(g, box, kernel, k, W, axis=None, axis2=None, alpha=0.0):
    """A g with A_{nl} = H Re sum_j c_j exp(i k_j.(x_n - x_l)); A is symmetric, so this is
    also the vector-Jacobian product of u with respect to rho."""
    return potential(np.asarray(g, dtype=np.float64), box, kernel, k, W, axis, axis2, alpha)[0]


def energy_gradient_rho(u, box, lam):
    """dE/drho_n = lambda H u_n (E = (lambda/2) H rho^T A rho with A symmetric)."""
    return lam * _cell_volume(u.shape, box) * u


def energy_gradient_psi(u, psi, box, lam):
    """dE/dpsi*_n = lambda H u_n psi_n for rho = |psi|^2."""
    return lam * _cell_volume(u.shape, box) * u * psi


@dataclass
class Result:
    u: np.ndarray
    energy_physical: float
    energy_fourier: float
    rhohat: np.ndarray
    c: np.ndarray
    k: np.ndarray
    W: np.ndarray
    imag_max: float


def evaluate(problem, rho):
    """Full oracle evaluation of a workloads.Problem on density rho (FP64).  A kernel
    with a node at k = 0 (the 2D Poisson one) adds c_0 rho^(0) to u and
    (lambda/2) c_0 rho^(0)^2 to the Fourier-side energy."""
    rho = np.asarray(rho, dtype=np.float64)
    k, W = fourier_nodes(problem)
    u, rh, c, im = potential(rho, problem.box, problem.kernel, k, W, problem.axis, problem.axis2, problem.alpha)
    K = problem.kmax if problem.kmax > 0 else default_kmax(problem.n, problem.box)
    c0 = origin_coefficient(problem.kernel, K, problem.n_r, getattr(problem, "radial", 0), problem.eps)
    r0 = _cell_volume(rho.shape, problem.box) * float(np.sum(rho))
    u = u + c0 * r0
    return Result(u=u,
                  energy_physical=energy_physical(rho, u, problem.box, problem.lam),
                  energy_fourier=energy_fourier(c, rh, problem.lam) + 0.5 * problem.lam * c0 * r0 * r0,
                  rhohat=rh, c=c, k=k, W=W, imag_max=im)
