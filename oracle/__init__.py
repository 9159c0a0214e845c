"""Oracle for the free-space Coulomb / dipole convolution -- TEST INFRASTRUCTURE ONLY.

A plain, slow, FP64 CPU evaluation of the discrete quantity the GPU library
computes faster: the trapezoid-rule transform of the density (eq. 3.2) at the
spherical / polar Fourier quadrature nodes (eqs. 3.5, 3.7), the weighted sum
back to the uniform grid (eq. 3.7, Algorithm 1), and the interaction energy
(eq. gpe2 and the energy remark after Algorithm 2).  No NUFFT is used: every
sum is evaluated directly, with per-axis phase tables and BLAS matrix products
as the only library primitives.  `split` holds Algorithm 2 (Section 3.3), whose
regular-grid part I1 is a padded FFT convolution (numpy's FFT as the library
step), pinned against the same trapezoid sum done directly.  `gpe` holds the
time-splitting driver for the Gross-Pitaevskii equation that repeatedly
evaluates the potential (Strang splitting, real and imaginary time).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import this package.  It shares no code with the HIP library: the two meet
only through the seeded inputs in `workloads`.

Pins (tests/test_oracle_*.py) tie every function here to something other than
itself: closed-form potentials and energies from the paper's examples, the
energies the paper prints for Example 7, exact quadrature identities, brute
force on tiny grids, and exact invariants (energy identity, scaling laws,
symmetry, self-adjointness).
"""
from .quadrature import (gauss_legendre, radial_rule, theta_rule, phi_rule,
                         spherical_nodes, polar_nodes, fourier_nodes)
from .symbols import symbol, coefficients
from .direct import (rho_hat, rho_hat_separable, rho_hat_separable_sum, sum_to_grid, sum_to_points,
                     sum_to_lattice, potential, energy_fourier,
                     energy_physical, Result, evaluate, energy_gradient_rho,
                     energy_gradient_psi, apply_operator)
from . import closed_forms
from . import split
from . import gpe

__all__ = [
    "gauss_legendre", "radial_rule", "theta_rule", "phi_rule", "spherical_nodes",
    "polar_nodes", "fourier_nodes", "symbol", "coefficients", "rho_hat", "rho_hat_separable", "rho_hat_separable_sum", "sum_to_grid",
    "sum_to_points", "sum_to_lattice", "potential", "energy_fourier", "energy_physical", "Result", "evaluate",
    "energy_gradient_rho", "energy_gradient_psi", "apply_operator", "closed_forms", "split", "gpe",
]
