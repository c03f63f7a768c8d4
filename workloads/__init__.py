"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package produces *inputs only*: the synthetic RANS channel profiles that
stand in for the k-omega finite-volume solution the paper feeds to its
synthetic turbulence generator (Numerical setup section), the stretched
finite-volume y-grids those profiles live on, the lattice configurations, and
the seeded serving job mixes.  It holds none of the STG-LBM method's
arithmetic (no interpolation, Cholesky factor, spectrum, Fourier modes, unit
conversion or lattice-Boltzmann step); the oracle and the HIP library each
implement those on their own.
"""

from .rans import (
    KAPPA,
    reichardt_uplus,
    reichardt_duplus,
    k_plus,
    omega_plus,
    stretched_fv_grid,
    channel_rans_profile,
    bulk_velocity_fv,
)
from .configs import (channel_config, CONFIG_NAMES, perturbed_state, serving_jobs, job_config, small_channel,
                      periodic_channel)

__all__ = [
    "KAPPA",
    "reichardt_uplus",
    "reichardt_duplus",
    "k_plus",
    "omega_plus",
    "stretched_fv_grid",
    "channel_rans_profile",
    "bulk_velocity_fv",
    "channel_config",
    "CONFIG_NAMES",
    "perturbed_state",
    "serving_jobs",
    "job_config",
    "small_channel",
    "periodic_channel",
]
