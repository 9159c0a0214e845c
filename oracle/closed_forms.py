"""Closed-form potentials and energies used to pin the oracle.  Test infrastructure only.

Sources (all in the paper's notation):
  * 3D Coulomb potential of a Gaussian charge exp(-|x|^2/a): Q erf(r/sqrt a)/(4 pi r)
    with Q = (pi a)^{3/2} (Green's function 1/(4 pi |x|) of eq. Cou3D).
  * 2.5D Coulomb potential of exp(-|x|^2/a): eq. 4.2 (Example 1),
    (sqrt(pi a)/2) exp(-r^2/2a) I0(r^2/2a).
  * Example 4: rho of eq. 4.10 has Coulomb potential -exp(-g).
  * Example 5: dipole potential -rho + 6 [2 g_n^2 - sum n_i^2/a_i] exp(-g).
  * Example 7: dipole energy of an anisotropic normalised Gaussian, with the
    three printed exact values.
  * Gaussian-mixture energies: the autocorrelation of two Gaussians is a
    Gaussian, (pi a_i a_j/(a_i+a_j))^{d/2} exp(-|z-(c_i-c_j)|^2/(a_i+a_j)), so
    E = (lambda/2) sum_ij A_i A_j (pi a_i a_j/(a_i+a_j))^{d/2} u_{a_i+a_j}(|c_i-c_j|).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf, i0e

# Example 7 exact energies as printed (lambda = 8 pi / 3, n = z-axis).
EXAMPLE7_PRINTED = {
    "I": {"gx": 0.25, "gz": 1.0, "E": 0.03867086140999021},
    "II": {"gx": 1.0, "gz": 1.0, "E": 0.0},
    "III": {"gx": 2.0, "gz": 1.0, "E": -0.1386449740987819},
}


def coulomb3d_gaussian(r, a=1.0):
    """Potential of exp(-|x|^2/a) under U = 1/(4 pi |x|)."""
    r = np.asarray(r, dtype=np.float64)
    Q = (np.pi * a) ** 1.5
    out = np.empty_like(r)
    small = r < 1e-8
    out[~small] = Q * erf(r[~small] / np.sqrt(a)) / (4 * np.pi * r[~small])
    out[small] = a / 2.0   # limit: Q * 2/(sqrt(pi a)) / (4 pi)
    return out


def coulomb2d_gaussian(r, a=1.0):
    """Eq. 4.2: potential of exp(-|x|^2/a) under U = 1/(2 pi |x|) in the plane."""
    r = np.asarray(r, dtype=np.float64)
    return 0.5 * np.sqrt(np.pi * a) * i0e(r * r / (2.0 * a))


def coulomb3d_gaussian_energy(a=1.0, lam=1.0):
    return lam * np.pi ** 1.5 * a ** 2.5 / (4.0 * np.sqrt(2.0))


def coulomb2d_gaussian_energy(a=1.0, lam=1.0):
    return lam * np.pi ** 1.5 * a ** 1.5 / (4.0 * np.sqrt(2.0))


def mixture_potential(mix, X, d):
    """u(x) = sum_g A_g u_{a_g}(|x - c_g|), a_g = sigma_g^2."""
    f = coulomb3d_gaussian if d == 3 else coulomb2d_gaussian
    out = 0.0
    for A, c, s in zip(mix.amps, mix.centers, mix.widths):
        r = np.sqrt(sum((Xi - ci) ** 2 for Xi, ci in zip(X, c)))
        out = out + A * f(r, s * s)
    return out


def mixture_energy(mix, d, lam=1.0):
    f = coulomb3d_gaussian if d == 3 else coulomb2d_gaussian
    E = 0.0
    for Ai, ci, si in zip(mix.amps, mix.centers, mix.widths):
        for Aj, cj, sj in zip(mix.amps, mix.centers, mix.widths):
            ai, aj = si * si, sj * sj
            dist = np.linalg.norm(np.asarray(ci) - np.asarray(cj))
            E += Ai * Aj * (np.pi * ai * aj / (ai + aj)) ** (d / 2.0) * float(f(np.array([dist]), ai + aj)[0])
    return 0.5 * lam * E


def example4_potential(X, a):
    """Coulomb potential of the eq. 4.10 density: -exp(-g), g = sum x_i^2/a_i."""
    g = sum(Xi ** 2 / ai for Xi, ai in zip(X, a))
    return -np.exp(-g)


def example5_potential(X, a, n):
    """Dipole potential of the eq. 4.10 density (Example 5)."""
    g = sum(Xi ** 2 / ai for Xi, ai in zip(X, a))
    gn = sum(Xi * ni / ai for Xi, ni, ai in zip(X, n, a))
    beta = sum(1.0 / ai for ai in a)
    q = sum(Xi ** 2 / ai ** 2 for Xi, ai in zip(X, a))
    rho = (-2.0 * beta + 4.0 * q) * np.exp(-g)
    s = sum(ni * ni / ai for ni, ai in zip(n, a))
    return -rho + 6.0 * (2.0 * gn * gn - s) * np.exp(-g)


def example7_energy(gx, gz, lam):
    """Example 7: dipole energy (n = z-axis) of pi^{-3/2} gx sqrt(gz) exp(-(gx(x^2+y^2)+gz z^2))."""
    kap2 = gz / gx
    pref = -lam * gx * np.sqrt(gz) / (4.0 * np.pi * np.sqrt(2.0 * np.pi))
    if abs(kap2 - 1.0) < 1e-15:
        return 0.0
    base = (1.0 + 2.0 * kap2) / (1.0 - kap2)
    if kap2 > 1.0:
        s = np.sqrt(kap2 - 1.0)
        return pref * (base - 3.0 * kap2 * np.arctan(s) / ((1.0 - kap2) * s))
    s = np.sqrt(1.0 - kap2)
    return pref * (base - 3.0 * kap2 / (2.0 * (1.0 - kap2) * s) * np.log((1.0 + s) / (1.0 - s)))
