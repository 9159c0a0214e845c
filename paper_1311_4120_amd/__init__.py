"""MI355X library for free-space Coulomb, dipole-dipole and 2D Poisson
convolutions by Fourier quadrature on spherical / polar nodes and NUFFTs
(Jiang, Greengard and Bao, arXiv:1311.4120: Algorithm 1, and the
partition-of-unity split of Algorithm 2), with a time-splitting
Gross-Pitaevskii driver built on it.  The compute path is libjgb.so (HIP,
gfx950); this package only marshals arguments."""
from .api import GPE, Batch, DipolarEnergy, InteractionEnergy, Plan  # noqa: F401
