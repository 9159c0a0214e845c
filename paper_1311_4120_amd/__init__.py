"""MI355X library for free-space Coulomb and dipole-dipole convolutions by
Fourier quadrature on spherical / polar nodes and NUFFTs (Jiang, Greengard and
Bao, arXiv:1311.4120, Algorithm 1).  The compute path is libjgb.so (HIP,
gfx950); this package only marshals arguments."""
from .api import GPE, Batch, DipolarEnergy, InteractionEnergy, Plan  # noqa: F401
