"""Seeded synthetic inputs for the free-space convolution u = U*rho.

This module holds only input generation: the uniform grid of the problem
statement (Section 3.1, eq. 3.2 and Algorithm 1: x_n = -R_j/2 + n_j R_j/N_j,
n_j = 0..N_j-1), closed-form densities evaluated on it, and the named
workload configurations.  It contains none of the method's arithmetic (no
quadrature, no transform, no symbol), so both the oracle and the GPU path
may import it.

Densities follow the paper's numerical examples (Section 4): isotropic and
anisotropic Gaussians (Examples 1 and 7), the Laplacian-of-Gaussian density
of eq. 4.10 (Examples 4 and 5), plus seeded Gaussian mixtures and wave
packets that stand in for the application densities rho = |psi|^2 of the
introduction.  Every random draw uses numpy.random.default_rng(seed) in the
order written below.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import numpy as np

COULOMB_3D = 0
COULOMB_2D = 1
DIPOLE_3D = 2
DIPOLE_2D = 3
POISSON_2D = 4

FP64 = 0
MIXED = 1

THETA_GL = 0
COSTHETA_GL = 1


def grid_axes(n: Sequence[int], box: Sequence[float]):
    """Per-axis coordinates x_{n_j} = -R_j/2 + n_j h_j, h_j = R_j/N_j (eq. 3.2)."""
    return [(-0.5 * float(R) + np.arange(int(N), dtype=np.float64) * (float(R) / int(N)))
            for N, R in zip(n, box)]


def mesh(n, box):
    axes = grid_axes(n, box)
    return np.meshgrid(*axes, indexing="ij")


# ---------------------------------------------------------------- densities

def gaussian(n, box, a=1.0, center=None, amp=1.0):
    """amp * exp(-|x-c|^2 / a) on the grid (Example 1 uses a = 1.3)."""
    X = mesh(n, box)
    c = np.zeros(len(n)) if center is None else np.asarray(center, dtype=np.float64)
    r2 = sum((Xi - ci) ** 2 for Xi, ci in zip(X, c))
    return amp * np.exp(-r2 / a)


def anisotropic_gaussian(n, box, s, center=None):
    """exp(-sum_i (x_i-c_i)^2 / s_i^2)."""
    X = mesh(n, box)
    c = np.zeros(len(n)) if center is None else np.asarray(center, dtype=np.float64)
    q = sum((Xi - ci) ** 2 / float(si) ** 2 for Xi, ci, si in zip(X, c, s))
    return np.exp(-q)


def log_density(n, box, a):
    """Eq. 4.10: rho = [-2 beta + 4 sum x_i^2/a_i^2] exp(-g), g = sum x_i^2/a_i."""
    X = mesh(n, box)
    beta = sum(1.0 / ai for ai in a)
    g = sum(Xi ** 2 / ai for Xi, ai in zip(X, a))
    q = sum(Xi ** 2 / ai ** 2 for Xi, ai in zip(X, a))
    return (-2.0 * beta + 4.0 * q) * np.exp(-g)


def example7_density(n, box, gx, gz):
    """Example 7: pi^{-3/2} gx sqrt(gz) exp(-(gx (x^2+y^2) + gz z^2))."""
    X = mesh(n, box)
    return np.pi ** -1.5 * gx * np.sqrt(gz) * np.exp(-(gx * (X[0] ** 2 + X[1] ** 2) + gz * X[2] ** 2))


@dataclass
class Mixture:
    amps: np.ndarray      # (G,)
    centers: np.ndarray   # (G, d)
    widths: np.ndarray    # (G,) sigma_g: term = A exp(-|x-c|^2/sigma^2)

    def evaluate(self, n, box):
        X = mesh(n, box)
        out = np.zeros(tuple(int(v) for v in n))
        for A, c, s in zip(self.amps, self.centers, self.widths):
            r2 = sum((Xi - ci) ** 2 for Xi, ci in zip(X, c))
            out += A * np.exp(-r2 / s ** 2)
        return out


    def density_terms(self, n, box):
        """The same density as a sum of separable terms: A exp(-|x-c|^2/sigma^2) =
        A prod_i exp(-(x_i-c_i)^2/sigma^2).  Returns (coefficients, per-term lists
        of per-axis samples)."""
        axes = grid_axes(n, box)
        coefs, factors = [], []
        for A, c, s in zip(self.amps, self.centers, self.widths):
            coefs.append(complex(A))
            factors.append([np.exp(-(x - ci) ** 2 / s ** 2) for x, ci in zip(axes, c)])
        return np.array(coefs), factors


def random_mixture(rng, g, d, center_lo, center_hi, width_lo, width_hi, amp_lo=0.5, amp_hi=2.0):
    centers = rng.uniform(center_lo, center_hi, size=(g, d))
    widths = rng.uniform(width_lo, width_hi, size=g)
    amps = rng.uniform(amp_lo, amp_hi, size=g)
    return Mixture(amps=amps, centers=centers, widths=widths)


def unit_vector(rng, d=3):
    v = rng.standard_normal(d)
    return v / np.linalg.norm(v)


@dataclass
class WavePackets:
    amps: np.ndarray
    phases: np.ndarray
    centers: np.ndarray
    widths: np.ndarray
    k0: np.ndarray

    def evaluate(self, n, box, dtype=np.complex128):
        X = mesh(n, box)
        psi = np.zeros(tuple(int(v) for v in n), dtype=np.complex128)
        for a, th, c, s, k in zip(self.amps, self.phases, self.centers, self.widths, self.k0):
            r2 = sum((Xi - ci) ** 2 for Xi, ci in zip(X, c))
            kx = sum(Xi * ki for Xi, ki in zip(X, k))
            psi += a * np.exp(1j * th) * np.exp(-r2 / (2 * s * s)) * np.exp(1j * kx)
        return psi.astype(dtype)


    def packet_factors(self, n, box):
        """Per packet: the complex amplitude a e^{i theta} and the per-axis samples
        exp(-(x_i-c_i)^2/(2 s^2)) exp(i k0_i x_i), whose product over axes times
        the amplitude is the packet on the grid."""
        axes = grid_axes(n, box)
        out = []
        for a, th, c, s, k in zip(self.amps, self.phases, self.centers, self.widths, self.k0):
            f = [np.exp(-(x - ci) ** 2 / (2 * s * s)) * np.exp(1j * x * ki) for x, ci, ki in zip(axes, c, k)]
            out.append((a * np.exp(1j * th), f))
        return out

    def density_terms(self, n, box):
        """rho = |psi|^2 as the sum over packet pairs (p, q) of the separable terms
        amp_p conj(amp_q) prod_i f_{p,i} conj(f_{q,i}).  Returns (coefficients,
        per-term lists of per-axis samples)."""
        pf = self.packet_factors(n, box)
        coefs, factors = [], []
        for ap, fp in pf:
            for aq, fq in pf:
                coefs.append(ap * np.conj(aq))
                factors.append([a * np.conj(b) for a, b in zip(fp, fq)])
        return np.array(coefs), factors


def random_wave_packets(rng, p=6, lo=-6.0, hi=6.0):
    centers = rng.uniform(lo, hi, size=(p, 3))
    widths = rng.uniform(1.0, 2.0, size=p)
    amps = rng.uniform(0.5, 1.0, size=p)
    phases = rng.uniform(0.0, 2 * np.pi, size=p)
    # |k0| <= 2, uniform in the ball
    dirs = rng.standard_normal((p, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    radii = 2.0 * rng.uniform(0.0, 1.0, size=p) ** (1.0 / 3.0)
    k0 = dirs * radii[:, None]
    return WavePackets(amps=amps, phases=phases, centers=centers, widths=widths, k0=k0)


# ---------------------------------------------------------------- configs

RADIAL_GL, RADIAL_GGQ = 0, 1   # Gauss-Legendre, generalized Gaussian (band-limited)


@dataclass
class Problem:
    """One evaluation of u = U*rho: grid, box, kernel and Fourier node counts."""
    name: str
    dim: int
    n: Tuple[int, ...]
    box: Tuple[float, ...]
    kernel: int
    n_r: int
    n_theta: int
    n_phi: int
    theta_rule: int = THETA_GL
    axis: Tuple[float, float, float] = (0.0, 0.0, 1.0)
    axis2: Optional[Tuple[float, float, float]] = None   # second dipole orientation m (None: m = n)
    alpha: float = 0.0                                   # the 2.5D dipole's -alpha delta term
    lam: float = 1.0
    eps: float = 1e-10
    precision: int = FP64
    kmax: float = 0.0   # 0 -> pi / max_j h_j
    radial: int = 0     # radial rule: RADIAL_GL or RADIAL_GGQ

    @property
    def npoints(self):
        return int(np.prod(self.n))

    @property
    def nnodes(self):
        return self.n_r * self.n_phi * (self.n_theta if self.dim == 3 else 1)


def coulomb3d_32(theta_rule=THETA_GL):
    """32^3 grid over [-8,8)^3, rho = exp(-|x|^2), nodes (32,16,32)."""
    p = Problem("coulomb3d_32", 3, (32, 32, 32), (16.0, 16.0, 16.0), COULOMB_3D, 32, 16, 32,
                theta_rule=theta_rule)
    rho = gaussian(p.n, p.box, a=1.0)
    return p, rho


def coulomb2d_256(seed=2):
    """256^2 grid over [-16,16)^2, 8 seeded Gaussians, polar nodes (64,128)."""
    rng = np.random.default_rng(seed)
    mix = random_mixture(rng, 8, 2, -4.0, 4.0, 0.5, 1.5)
    p = Problem("coulomb2d_256", 2, (256, 256), (32.0, 32.0), COULOMB_2D, 64, 1, 128)
    return p, mix.evaluate(p.n, p.box), mix


def dipole3d_128(precision=FP64, seed=3, nodes="pattern"):
    """128^3 grid over [-12,12)^3, rho = |psi|^2 for psi with axes (1,1.5,0.7).

    nodes="pattern": (128,64,128) with the theta Gauss-Legendre rule, identical work in
    both precisions; nodes="resolved": the accuracy-matched cos(theta)-rule sets,
    (256,128,256) in float64 (eps 1e-10) and (192,96,192) in mixed precision (eps 1e-5);
    nodes="split": the node sets of I2 in Algorithm 2 at the default window and
    cut-off (kmax = 0), matched to the same accuracies: (28,20,40) cos(theta) in
    float64 (1.5e-11 from the converged potential) and (20,16,32) in mixed
    precision (1.8e-6)."""
    rng = np.random.default_rng(seed)
    axis = tuple(unit_vector(rng, 3))
    eps = 1e-10 if precision == FP64 else 1e-5
    if nodes == "pattern":
        nr, nt, nph, rule = 128, 64, 128, THETA_GL
    elif nodes == "split":
        nr, nt, nph, rule = (28, 20, 40, COSTHETA_GL) if precision == FP64 else (20, 16, 32, COSTHETA_GL)
    elif precision == FP64:
        nr, nt, nph, rule = 256, 128, 256, COSTHETA_GL
    else:
        nr, nt, nph, rule = 192, 96, 192, COSTHETA_GL
    p = Problem("dipole3d_128", 3, (128, 128, 128), (24.0, 24.0, 24.0), DIPOLE_3D, nr, nt, nph,
                theta_rule=rule, axis=axis, eps=eps, precision=precision)
    # psi = exp(-sum x_i^2 / (2 a_i^2)) -> rho = |psi|^2 = exp(-sum x_i^2 / a_i^2)
    rho = anisotropic_gaussian(p.n, p.box, (1.0, 1.5, 0.7))
    return p, rho


def batched_coulomb(seed=4, count=64):
    """64 densities, N_b ~ U{64,96,128,160}^3, half-widths L ~ U[8,16], 4 Gaussians each."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        N = int(rng.choice([64, 96, 128, 160]))
        L = float(rng.uniform(8.0, 16.0))
        h = 2 * L / N
        mix = random_mixture(rng, 4, 3, -L / 4, L / 4, 4 * h, 6 * h)
        p = Problem(f"batched_coulomb[{b}]", 3, (N, N, N), (2 * L,) * 3, COULOMB_3D, N, N // 2, N,
                    eps=1e-5, precision=MIXED)
        out.append((p, mix))
    return out


def dipole_grad_256(seed=5):
    """256^3 grid over [-16,16)^3, psi = 6 seeded wave packets, dipole kernel."""
    rng = np.random.default_rng(seed)
    packets = random_wave_packets(rng)
    axis = tuple(unit_vector(rng, 3))
    p = Problem("dipole_grad_256", 3, (256, 256, 256), (32.0, 32.0, 32.0), DIPOLE_3D, 256, 128, 256,
                theta_rule=COSTHETA_GL, axis=axis, eps=1e-5, precision=MIXED)
    return p, packets
