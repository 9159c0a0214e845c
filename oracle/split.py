"""Algorithm 2 (Section 3.3): the partition-of-unity split of eq. 3.9.
TEST INFRASTRUCTURE ONLY (see the package header).

    u = I1 + I2,
    I1(x) = (2 pi)^{-d} int e^{ik.x} (1 - p(k)) U^(k) rho^(k) dk,
    I2(x) = (2 pi)^{-d} int e^{ik.x} p(k) U^(k) rho^(k) dk.

Windows: 3D p3(k) = exp(-|k|^2 / a) (eq. 3.10); 2D
p2(k) = erfc(12 (|k| - (R0 + R1)/2) / (R1 - R0)) / 2 (eq. 3.12).  The remarks
after eqs. 3.10 and 3.12 give the scales as multiples of the Fourier spacing
(written there as 1/max h); they are read as multiples of dk = 2 pi / max_j R_j,
which is what makes I2's node count independent of N: a = 2 dk^2,
R0 = 0.8 dk, R1 = 10 dk.  I2 then needs nodes only up to
K2 = min(pi / max h, sqrt(40 a)) in 3D (p3 < 5e-18 beyond) and
K2 = min(pi / max h, R1) in 2D (p2 < 2e-17 beyond).

I1 is smooth in k, so it is discretised by the trapezoid rule on the regular grid
k_q = 2 pi q / (sigma R_j) per axis, q = -sigma N_j/2 .. sigma N_j/2 - 1, with
oversampling sigma = 2 (Algorithm 2, step 3), and rho^ at those frequencies is
the trapezoid transform of eq. 3.2.  Written out, that is the periodic
convolution of the zero-padded density with the symbol M = (1 - p) U^:

    I1 = IDFT_{sigma N}( M(k_q) * DFT_{sigma N}(rho placed at m mod sigma N) ), cropped,

evaluated here with numpy's FFT as the library step.  `i1_direct` evaluates the
same trapezoid sum with the direct sums of `direct.py` instead, which pins the
FFT form (padding, index order, normalisation).  At k = 0, M takes its limit:
1/a for the 3D Coulomb kernel, 0 for the dipole (1 - p vanishes and U^ is
bounded), and 0 for the 2D Coulomb kernel (1 - p2 is below 1e-20 there for
the default scales; the limit of (1 - p2)/|k| itself does not exist).

I2 is Algorithm 1 with the coefficients c_j = (2 pi)^{-d} W_j S(k_j) p(k_j) (and,
for the 2D Poisson kernel, its node at k = 0, where p = 1).
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.special import erfc

from .direct import _axes, _cell_volume, rho_hat, sum_to_grid
from .quadrature import fourier_nodes
from .symbols import COULOMB_2D, COULOMB_3D, DIPOLE_3D, origin_coefficient, symbol

SIGMA = 2


def default_window(n, box):
    """Window scales in units of dk = 2 pi / max R: a = 2 dk^2 (3D), R0 = 0.8 dk, R1 = 10 dk (2D)."""
    dk = 2.0 * np.pi / max(float(R) for R in box)
    if len(n) == 3:
        return {"a": 2.0 * dk * dk}
    return {"R0": 0.8 * dk, "R1": 10.0 * dk}


def default_cutoff(n, box, par):
    """Radius of I2's node set: where the window has decayed below FP64 resolution,
    at most the alias-free pi / max h."""
    hmax = max(float(R) / int(N) for N, R in zip(n, box))
    K = np.pi / hmax
    if len(n) == 3:
        return min(K, float(np.sqrt(40.0 * par["a"])))
    return min(K, float(par["R1"]))


def window(kabs, dim, par):
    """p_d(|k|) (eqs. 3.10 and 3.12)."""
    kabs = np.asarray(kabs, dtype=np.float64)
    if dim == 3:
        return np.exp(-kabs ** 2 / par["a"])
    R0, R1 = par["R0"], par["R1"]
    return 0.5 * erfc(12.0 * (kabs - 0.5 * (R0 + R1)) / (R1 - R0))


def one_minus_window(kabs, dim, par):
    """1 - p_d(|k|), without cancellation."""
    kabs = np.asarray(kabs, dtype=np.float64)
    if dim == 3:
        return -np.expm1(-kabs ** 2 / par["a"])
    R0, R1 = par["R0"], par["R1"]
    return 0.5 * erfc(-12.0 * (kabs - 0.5 * (R0 + R1)) / (R1 - R0))


def grid_frequencies(n, box, sigma=SIGMA):
    """k_q per axis for q in numpy FFT order on the sigma-times oversampled grid."""
    out = []
    for N, R in zip(n, box):
        L = sigma * int(N)
        q = np.fft.fftfreq(L, d=1.0 / L)            # 0, 1, .., L/2 - 1, -L/2, .., -1
        out.append(2.0 * np.pi * q / (sigma * float(R)))
    return out


def split_symbol(kernel, k, par, axis=None, axis2=None, alpha=0.0):
    """M(k) = (1 - p(k)) U^(k) at frequency vectors k (rows), with the k = 0 limits."""
    k = np.asarray(k, dtype=np.float64)
    d = k.shape[1]
    k2 = np.einsum("ij,ij->i", k, k)
    kabs = np.sqrt(k2)
    omp = one_minus_window(kabs, d, par)
    S = symbol(kernel, k, axis, axis2, alpha)       # |k|^{d-1} U^
    zero = k2 == 0.0
    den = np.where(zero, 1.0, kabs ** (d - 1))
    M = omp * S / den
    if kernel == COULOMB_3D:
        M[zero] = 1.0 / par["a"]
    else:                                           # dipoles: (1-p) -> 0, U^ bounded; 2D: reading above
        M[zero] = 0.0
    return M


def _grid_k(n, box, sigma=SIGMA):
    ks = grid_frequencies(n, box, sigma)
    mesh = np.meshgrid(*ks, indexing="ij")
    return np.stack([m.ravel() for m in mesh], axis=1), [len(v) for v in ks]


def i1_fft(rho, box, kernel, par, axis=None, sigma=SIGMA, axis2=None, alpha=0.0):
    """I1 on the grid by the padded FFT convolution."""
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.shape
    k, L = _grid_k(n, box, sigma)
    M = split_symbol(kernel, k, par, axis, axis2, alpha).reshape(L)
    pad = np.zeros(L, dtype=np.float64)
    idx = np.ix_(*[np.arange(-(N // 2), N - N // 2) % Lj for N, Lj in zip(n, L)])
    pad[idx] = rho
    # Re: on a Nyquist plane the grid frequency is its own mirror on that axis,
    # and a symbol that is not a function of |k| alone (the dipole's) takes
    # different values at k and at the mirror of -k there; the real part uses
    # their mean, as the real integral (I1 is real) requires
    conv = np.fft.ifftn(M * np.fft.fftn(pad))
    return conv[idx].real.copy()


def i1_direct(rho, box, kernel, par, axis=None, sigma=SIGMA, axis2=None, alpha=0.0):
    """The same trapezoid sum by the direct sums: weights (1/(sigma R_j))^d M(k_q)
    on the regular frequency grid, rho^(k_q) from eq. 3.2.  Small grids only."""
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.shape
    k, _ = _grid_k(n, box, sigma)
    w = 1.0 / np.prod([sigma * float(R) for R in box])
    M = split_symbol(kernel, k, par, axis, axis2, alpha)
    rh = rho_hat(rho, box, k)
    return sum_to_grid(w * M * rh, k, n, box).real.copy()


def i2_coefficients(kernel, k, W, par, axis=None, axis2=None, alpha=0.0):
    d = k.shape[1]
    kabs = np.sqrt(np.einsum("ij,ij->i", k, k))
    return W * symbol(kernel, k, axis, axis2, alpha) * window(kabs, d, par) / (2.0 * np.pi) ** d


def i1_energy(rho, box, kernel, par, axis=None, sigma=SIGMA, axis2=None, alpha=0.0):
    """H sum_n rho_n I1_n in Fourier form: (prod_j sigma R_j)^{-1} sum_q M(k_q) |rho^(k_q)|^2
    (substitute eq. 3.2 into the trapezoid sum of I1; rho real)."""
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.shape
    k, L = _grid_k(n, box, sigma)
    M = split_symbol(kernel, k, par, axis, axis2, alpha).reshape(L)
    pad = np.zeros(L, dtype=np.float64)
    idx = np.ix_(*[np.arange(-(N // 2), N - N // 2) % Lj for N, Lj in zip(n, L)])
    pad[idx] = rho
    rh = _cell_volume(n, box) * np.fft.fftn(pad)
    return float(np.sum(M * np.abs(rh) ** 2)) / np.prod([sigma * float(R) for R in box])


def energy_split_fourier(problem, rho, par=None, rh=None):
    """E = (lambda/2) [sum_j c_j p(k_j) |rho^_j|^2 + I1's Fourier-form share], equal to
    the physical-side (lambda/2) H sum rho u for real rho.  rh: rho^ at I2's nodes,
    if already known."""
    rho = np.asarray(rho, dtype=np.float64)
    par = default_window(problem.n, problem.box) if par is None else par
    if problem.kmax <= 0:
        problem = dataclasses.replace(problem, kmax=default_cutoff(problem.n, problem.box, par))
    k, W = fourier_nodes(problem)
    c = i2_coefficients(problem.kernel, k, W, par, problem.axis, problem.axis2, problem.alpha)
    if rh is None:
        rh = rho_hat(rho, problem.box, k)
    r0 = _cell_volume(rho.shape, problem.box) * float(np.sum(rho))
    e2 = float(np.sum(c * np.abs(rh) ** 2)) + origin_coefficient(problem.kernel, problem.kmax, problem.n_r, getattr(problem, "radial", 0), problem.eps) * r0 * r0
    e1 = i1_energy(rho, problem.box, problem.kernel, par, problem.axis, axis2=problem.axis2, alpha=problem.alpha)
    return 0.5 * problem.lam * (e1 + e2)


def potential_split(problem, rho, par=None):
    """Algorithm 2 on a workloads.Problem (its node counts are I2's, its kmax I2's
    cut-off, the default one when 0): returns (u, I1, I2, E) with
    E = (lambda/2) H sum rho u (the energy remark)."""
    rho = np.asarray(rho, dtype=np.float64)
    par = default_window(problem.n, problem.box) if par is None else par
    i1 = i1_fft(rho, problem.box, problem.kernel, par, problem.axis, axis2=problem.axis2, alpha=problem.alpha)
    if problem.kmax <= 0:
        problem = dataclasses.replace(problem, kmax=default_cutoff(problem.n, problem.box, par))
    k, W = fourier_nodes(problem)
    c = i2_coefficients(problem.kernel, k, W, par, problem.axis, problem.axis2, problem.alpha)
    i2 = sum_to_grid(c * rho_hat(rho, problem.box, k), k, rho.shape, problem.box).real
    # the node at k = 0 of the 2D Poisson kernel belongs to I2 (p(0) = 1)
    i2 = i2 + origin_coefficient(problem.kernel, problem.kmax, problem.n_r, getattr(problem, "radial", 0), problem.eps) * _cell_volume(rho.shape, problem.box) * float(np.sum(rho))
    u = i1 + i2
    E = 0.5 * problem.lam * _cell_volume(rho.shape, problem.box) * float(np.sum(rho * u))
    return u, i1, i2, E
