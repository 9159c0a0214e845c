"""Time-splitting driver for the Gross-Pitaevskii / Schroedinger-Poisson equation
with the nonlocal potential of eq. gpe.  TEST INFRASTRUCTURE ONLY (see the
package header).

The equation (Section 1: the potential is needed on the grid many times, for
rho = |psi|^2 changing in time):

    i psi_t = [ -1/2 Lap + V(x) + beta |psi|^2 + lambda Phi ] psi,   Phi = U * |psi|^2,

on the grid of the potential's Problem, with the Laplacian periodic on the box
(psi and rho are negligible at its edges).  One step of length dt is Strang
splitting of the local and kinetic parts:

    N(dt/2):  psi <- exp(-i (dt/2) (V + beta |psi|^2 + lambda Phi)) psi   (|psi| unchanged)
    K(dt):    psi <- IDFT( exp(-i dt |k|^2 / 2) DFT(psi) ),  k_j = 2 pi q_j / R_j
    N(dt/2)   with Phi recomputed from the new |psi|^2.

Because N leaves |psi| unchanged, the Phi of a step's last half-step is the
Phi of the next step's first one, so a step needs one evaluation of Phi.  In
imaginary time (t = -i tau, the ground-state flow) the factors lose their i,
|psi| changes in N, Phi is evaluated before each half-step, and psi is
renormalised to H sum |psi|^2 = 1 after every step.

Energies (densities integrated by the trapezoid rule, the kinetic one by
Parseval on the periodic grid):
    E_kin = (H / (2 N)) sum_q |k_q|^2 |DFT(psi)_q|^2,   E_V = H sum V |psi|^2,
    E_loc = (beta/2) H sum |psi|^4,                      E_nl = (lambda/2) H sum Phi |psi|^2,
    E = E_kin + E_V + E_loc + E_nl,   mu = (E_kin + E_V + 2 E_loc + 2 E_nl) / norm.
"""
from __future__ import annotations

import numpy as np

from .direct import _axes, _cell_volume


def harmonic(n, box, trap):
    """V(x) = (1/2) sum_j gamma_j^2 x_j^2 on the grid."""
    x = _axes(n, box)
    X = np.meshgrid(*x, indexing="ij")
    return 0.5 * sum((float(g) ** 2) * Xi ** 2 for g, Xi in zip(trap, X))


def wavenumbers_squared(n, box):
    """|k|^2 on the periodic grid's DFT frequencies, k_j = 2 pi q_j / R_j (numpy FFT order)."""
    ks = [2.0 * np.pi * np.fft.fftfreq(int(N), d=1.0 / int(N)) / float(R) for N, R in zip(n, box)]
    K = np.meshgrid(*ks, indexing="ij")
    return sum(Ki ** 2 for Ki in K)


def kinetic_step(psi, box, dt, imaginary=False):
    k2 = wavenumbers_squared(psi.shape, box)
    f = np.exp(-0.5 * dt * k2) if imaginary else np.exp(-0.5j * dt * k2)
    return np.fft.ifftn(f * np.fft.fftn(psi))


def nonlinear_step(psi, V, phi, beta, lam, h, imaginary=False):
    theta = V + beta * np.abs(psi) ** 2 + lam * phi
    return psi * (np.exp(-h * theta) if imaginary else np.exp(-1j * h * theta))


def norm(psi, box):
    return _cell_volume(psi.shape, box) * float(np.sum(np.abs(psi) ** 2))


def strang(psi, box, V, beta, lam, dt, nsteps, potential, imaginary=False):
    """nsteps Strang steps from psi.  potential(rho) -> Phi = U * rho on the grid."""
    psi = np.asarray(psi, dtype=np.complex128).copy()
    if not imaginary:
        phi = potential(np.abs(psi) ** 2)
        for _ in range(nsteps):
            psi = nonlinear_step(psi, V, phi, beta, lam, 0.5 * dt)
            psi = kinetic_step(psi, box, dt)
            phi = potential(np.abs(psi) ** 2)
            psi = nonlinear_step(psi, V, phi, beta, lam, 0.5 * dt)
        return psi
    for _ in range(nsteps):
        phi = potential(np.abs(psi) ** 2)
        psi = nonlinear_step(psi, V, phi, beta, lam, 0.5 * dt, imaginary=True)
        psi = kinetic_step(psi, box, dt, imaginary=True)
        phi = potential(np.abs(psi) ** 2)
        psi = nonlinear_step(psi, V, phi, beta, lam, 0.5 * dt, imaginary=True)
        psi = psi / np.sqrt(norm(psi, box))
    return psi


def energies(psi, box, V, beta, lam, potential):
    """dict(norm, kinetic, trap, local, nonlocal, total, mu) of psi."""
    n = psi.shape
    H = _cell_volume(n, box)
    rho = np.abs(psi) ** 2
    phi = potential(rho)
    ph = np.fft.fftn(psi)
    ekin = H / (2.0 * psi.size) * float(np.sum(wavenumbers_squared(n, box) * np.abs(ph) ** 2))
    etrap = H * float(np.sum(V * rho))
    eloc = 0.5 * beta * H * float(np.sum(rho * rho))
    enl = 0.5 * lam * H * float(np.sum(phi * rho))
    nrm = H * float(np.sum(rho))
    return {"norm": nrm, "kinetic": ekin, "trap": etrap, "local": eloc, "nonlocal": enl,
            "total": ekin + etrap + eloc + enl, "mu": (ekin + etrap + 2 * eloc + 2 * enl) / nrm}
