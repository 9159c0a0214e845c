"""Generalized Gaussian radial rule for band-limited integrands (the remark at
the end of Section 3.3 and the Conclusions: where the change to polar or
spherical coordinates leaves the radial integrand hard to integrate, a
generalized Gaussian rule is built for it).  Oracle: test infrastructure only.

The radial integrand of the NUFFT's Fourier integral along a ray,
r -> rho^(r e) e^{i r e.x}, is band-limited: its frequencies e.(x - x') are
bounded by the box's diameter.  For such functions the generalized Gaussian
rules of Xiao, Rokhlin and Yarvin (Prolate spheroidal wavefunctions,
quadrature and interpolation, Inverse Problems 17, 2001) need fewer nodes than
Gauss-Legendre: the n-node rule of bandwidth c on [-1, 1] takes as nodes the n
roots of the prolate spheroidal wave function psi_n^c, and as weights the
solution of

    sum_j w_j psi_i^c(x_j) = int_{-1}^{1} psi_i^c(x) dx,   i = 0 .. n-1,

and integrates e^{i s x}, |s| <= 2c, to about the size of the prolate
eigenvalue |lambda_n| (at c -> 0 it becomes Gauss-Legendre).  The prolate
functions are computed from their expansion in normalised Legendre
polynomials, psi^c = sum_k beta_k sqrt(k + 1/2) P_k, whose coefficient vectors
are the eigenvectors of a symmetric tridiagonal matrix (one for even k, one
for odd k) with

    A_kk       = k (k + 1) + c^2 (2 k (k + 1) - 1) / ((2k + 3)(2k - 1)),
    A_k,k+2    = c^2 (k + 2)(k + 1) / ((2k + 3) sqrt((2k + 1)(2k + 5))),

psi_n^c being the eigenvector of the n-th smallest eigenvalue overall.

The bandwidth the plan chooses for n nodes and accuracy eps is

    c = (pi / 2) (n - 2 - 1.8 log10(10 / eps) - 0.06 n)

(Gauss-Legendre when c < 1): the rule then integrates e^{i s x}, |s| <= 2c,
well within eps (tests/test_oracle_ggq.py checks this for n up to 256).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as leg
from scipy.linalg import eigh_tridiagonal
from scipy.optimize import brentq

RADIAL_GL = 0
RADIAL_GGQ = 1


def bandwidth(n: int, eps: float) -> float:
    """The bandwidth c of the n-node rule at accuracy eps (0: Gauss-Legendre)."""
    c = 0.5 * np.pi * (n - 2.0 - 1.8 * np.log10(10.0 / eps) - 0.06 * n)
    return float(c) if c >= 1.0 else 0.0


def prolate_coefficients(c: float, count: int):
    """Normalised-Legendre coefficient vectors of psi_0^c .. psi_{count-1}^c."""
    M = 2 * count + int(np.ceil(2.0 * c)) + 64
    out = [None] * count
    for par in (0, 1):
        k = np.arange(par, M, 2).astype(np.float64)
        d = k * (k + 1) + c * c * (2 * k * (k + 1) - 1) / ((2 * k + 3) * (2 * k - 1))
        kk = k[:-1]
        e = c * c * (kk + 2) * (kk + 1) / ((2 * kk + 3) * np.sqrt((2 * kk + 1) * (2 * kk + 5)))
        _, v = eigh_tridiagonal(d, e)   # eigenvalues ascending
        for i in range(len(k)):
            n = 2 * i + par
            if n < count:
                coef = np.zeros(M)
                coef[par::2] = v[:, i]
                out[n] = coef
    return out


def prolate_eval(coef, x):
    """psi(x) = sum_k coef_k sqrt(k + 1/2) P_k(x)."""
    k = np.arange(len(coef))
    return leg.legval(np.asarray(x, dtype=np.float64), coef * np.sqrt(k + 0.5))


def prolate_rule(c: float, n: int):
    """Nodes (ascending) and weights of the n-node rule of bandwidth c on [-1, 1]."""
    cs = prolate_coefficients(c, n + 1)
    psin = cs[n]
    grid = np.cos(np.linspace(np.pi, 0.0, 40 * n + 400))
    f = prolate_eval(psin, grid)
    roots = []
    for i in range(len(grid) - 1):
        if f[i] == 0.0:
            roots.append(grid[i])
        elif f[i] * f[i + 1] < 0.0:
            roots.append(brentq(lambda t: float(prolate_eval(psin, t)), grid[i], grid[i + 1], xtol=1e-16, rtol=1e-15))
    x = np.array(roots)
    if len(x) != n:
        raise ValueError("psi_%d^%g has %d roots in (-1, 1)" % (n, c, len(x)))
    A = np.array([prolate_eval(cs[i], x) for i in range(n)])
    b = np.array([np.sqrt(2.0) * cs[i][0] for i in range(n)])
    w = np.linalg.solve(A, b)
    return x, w


def radial_rule_ggq(K: float, n_r: int, eps: float):
    """The generalized Gaussian radial rule on [0, K]: r = K (1 + x)/2, w = K w_x / 2."""
    c = bandwidth(n_r, eps)
    if c == 0.0:
        s, w = leg.leggauss(n_r)
    else:
        s, w = prolate_rule(c, n_r)
    return 0.5 * K * (1.0 + s), 0.5 * K * w
