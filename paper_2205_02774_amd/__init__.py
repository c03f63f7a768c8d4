"""STG-LBM on MI355X: a regularized D3Q19 lattice-Boltzmann LES of a turbulent
channel fed by a synthetic turbulence generator, as hand-written HIP kernels
behind the C ABI of libstglbm (include/stglbm.h).

The package holds the kernels (csrc/), their build, and a thin binding; the
serving loop batches several channels on one device.
"""

from .abi import StglbmError, load as load_library, LIB_PATH  # noqa: F401
from .lattice import (Lattice, channel_from_config, periodic_channel_from_config, derive_units,  # noqa: F401
                      acceleration_to_lattice,
                      footprint, make_desc)
