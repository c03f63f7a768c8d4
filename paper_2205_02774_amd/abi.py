"""ctypes declarations of libstglbm's C ABI (include/stglbm.h).

Argument marshalling only.  Loading fails loudly when the library has not
been built: there is no fallback implementation.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("STGLBM_LIB") or os.path.join(HERE, "libstglbm.so")

OK = 0
E_INVAL = -1
E_NOMEM = -2
E_HIP = -3
E_STATE = -4
E_UNSTABLE = -5
E_REALIZABILITY = -6

F32, F16, BF16 = 0, 1, 2
STORES = {"f32": F32, "f16": F16, "bf16": BF16}
COLLISIONS = {"regularized": 0, "bgk": 1}
ROW_FIELDS = 18

c_int32, c_int64, c_uint64, c_double = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
c_void_p = ctypes.c_void_p
P_double = ctypes.POINTER(ctypes.c_double)


class LatticeDesc(ctypes.Structure):
    _fields_ = [
        ("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("store", c_int32),
        ("periodic_x", c_int32), ("sponge_cells", c_int32), ("max_modes", c_int32), ("max_rans", c_int32),
        ("velocity_set", c_int32), ("collision", c_int32),
        ("nu_lb", c_double), ("cs_smag", c_double), ("force", c_double * 3), ("rho_out", c_double),
        ("sponge_K", c_double), ("sponge_p", c_double),
    ]


class RansInlet(ctypes.Structure):
    _fields_ = [
        ("n_rans", c_int32), ("n_modes", c_int32),
        ("y", P_double), ("U3", P_double), ("k", P_double), ("omega", P_double), ("R6", P_double),
        ("delta", c_double), ("nu_phys", c_double), ("c_x", c_double), ("c_t", c_double), ("U_b", c_double),
        ("alpha", c_double), ("seed", c_uint64), ("C_l", c_double), ("C_mu", c_double),
        ("strict", c_int32), ("reserved", c_int32),
    ]


class StglbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"stglbm error {code}: {msg}")
        self.code = code


_SIGS = {
    "stglbm_version": (c_int32, []),
    "stglbm_status_string": (ctypes.c_char_p, [c_int32]),
    "stglbm_derive_units": (c_int32, [c_double, c_int32, c_double, c_double, c_double, P_double, P_double, P_double]),
    "stglbm_footprint": (c_int32, [ctypes.POINTER(LatticeDesc), ctypes.POINTER(c_uint64)]),
    "stglbm_init_lattice": (c_int32, [ctypes.POINTER(LatticeDesc), c_void_p, c_uint64, c_void_p, ctypes.POINTER(c_void_p)]),
    "stglbm_set_rans_inlet": (c_int32, [c_void_p, ctypes.POINTER(RansInlet)]),
    "stglbm_stg_generate": (c_int32, [c_void_p, c_int64, c_void_p]),
    "stglbm_step": (c_int32, [c_void_p, c_int32]),
    "stglbm_step_noalloc": (c_int32, [c_void_p, c_int32]),
    "stglbm_stats_reset": (c_int32, [c_void_p]),
    "stglbm_stats_stop": (c_int32, [c_void_p]),
    "stglbm_get_stats": (c_int32, [c_void_p, P_double, c_uint64, ctypes.POINTER(c_int64)]),
    "stglbm_get_f": (c_int32, [c_void_p, P_double, c_uint64]),
    "stglbm_set_f": (c_int32, [c_void_p, P_double, c_uint64]),
    "stglbm_get_f_planes": (c_int32, [c_void_p, c_int32, c_int32, P_double, c_uint64]),
    "stglbm_set_equilibrium": (c_int32, [c_void_p, P_double, c_uint64]),
    "stglbm_set_equilibrium_physical": (c_int32, [c_void_p, P_double, c_uint64, c_double, c_double]),
    "stglbm_acceleration_to_lattice": (c_int32, [c_double, c_double, P_double, P_double]),
    "stglbm_set_probes": (c_int32, [c_void_p, c_int32, ctypes.POINTER(c_int32), c_void_p, c_int64]),
    "stglbm_probe_rows": (c_int32, [c_void_p, ctypes.POINTER(c_int64)]),
    "stglbm_state_view": (c_int32, [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_uint64)]),
    "stglbm_get_modes": (c_int32, [c_void_p, P_double, c_uint64]),
    "stglbm_get_inlet_rows": (c_int32, [c_void_p, P_double, c_uint64]),
    "stglbm_get_inlet_scalars": (c_int32, [c_void_p, P_double, c_uint64]),
    "stglbm_get_sqrtq": (c_int32, [c_void_p, P_double, c_uint64]),
    "stglbm_get_step": (c_int32, [c_void_p, ctypes.POINTER(c_int64)]),
    "stglbm_set_stream": (c_int32, [c_void_p, c_void_p]),
    "stglbm_sync": (c_int32, [c_void_p]),
    "stglbm_checkpoint_size": (c_int32, [c_void_p, ctypes.POINTER(c_uint64)]),
    "stglbm_checkpoint": (c_int32, [c_void_p, c_void_p, c_uint64]),
    "stglbm_restore": (c_int32, [c_void_p, c_void_p, c_uint64]),
    "stglbm_profile": (c_int32, [c_void_p, c_int32]),
    "stglbm_profile_read": (c_int32, [c_void_p, P_double, c_uint64]),
    "stglbm_copy_probe": (c_int32, [c_void_p, c_void_p, c_uint64, c_void_p]),
    "stglbm_bandwidth_probe": (c_int32, [c_void_p, c_void_p, c_uint64, c_int32, c_void_p]),
    "stglbm_destroy": (c_int32, [c_void_p]),
    "stglbm_last_error": (ctypes.c_char_p, [c_void_p]),
}

EXPORTED = tuple(_SIGS)
_lib = None


def load():
    """Load libstglbm.so from the package directory (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc, handle=None):
    if rc != OK:
        lib = load()
        msg = lib.stglbm_last_error(handle)
        raise StglbmError(rc, msg.decode() if msg else lib.stglbm_status_string(rc).decode())
    return rc
