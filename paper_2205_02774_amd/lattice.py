"""Python binding of libstglbm: one STG-LBM channel on one HIP device.

Marshalling only: torch supplies the device workspace and the stream,
NumPy arrays carry host data, and every step of the method runs in the
library's HIP kernels.  Method names follow the C entry points.
"""

import ctypes

import numpy as np
import torch

from . import abi


def _dptr(a):
    return a.ctypes.data_as(abi.P_double)


def derive_units(delta, ny, u_b_lb, U_b, nu_phys):
    """(c_x, c_t, nu_lb) of a channel run at lattice bulk velocity u_b_lb (library call)."""
    lib = abi.load()
    cx, ct, nu = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    abi.check(lib.stglbm_derive_units(delta, ny, u_b_lb, U_b, nu_phys,
                                      ctypes.byref(cx), ctypes.byref(ct), ctypes.byref(nu)))
    return cx.value, ct.value, nu.value


def acceleration_to_lattice(a_phys, c_x, c_t):
    """Guo acceleration in lattice units of a physical acceleration (library call)."""
    lib = abi.load()
    a = np.ascontiguousarray(a_phys, dtype=np.float64)
    if a.shape != (3,):
        raise ValueError("a_phys must hold 3 components")
    out = np.empty(3)
    abi.check(lib.stglbm_acceleration_to_lattice(c_x, c_t, _dptr(a), _dptr(out)))
    return tuple(float(v) for v in out)


def make_desc(nx, ny, nz, *, nu_lb, store="f32", periodic_x=False, cs_smag=0.1, force=(0.0, 0.0, 0.0),
              rho_out=1.0, sponge_cells=0, sponge_K=1000.0, sponge_p=3.0, max_modes=0, max_rans=0,
              velocity_set=19, collision="regularized"):
    d = abi.LatticeDesc()
    d.nx, d.ny, d.nz = nx, ny, nz
    d.store = abi.STORES[store] if isinstance(store, str) else int(store)
    d.periodic_x = 1 if periodic_x else 0
    d.sponge_cells = 0 if periodic_x else int(sponge_cells)
    d.max_modes = 0 if periodic_x else int(max_modes)
    d.max_rans = 0 if periodic_x else int(max_rans)
    d.nu_lb, d.cs_smag = float(nu_lb), float(cs_smag)
    for a in range(3):
        d.force[a] = float(force[a])
    d.rho_out, d.sponge_K, d.sponge_p = float(rho_out), float(sponge_K), float(sponge_p)
    d.velocity_set = int(velocity_set)
    d.collision = abi.COLLISIONS[collision] if isinstance(collision, str) else int(collision)
    return d


def footprint(desc):
    lib = abi.load()
    b = ctypes.c_uint64()
    abi.check(lib.stglbm_footprint(ctypes.byref(desc), ctypes.byref(b)))
    return b.value


class Lattice:
    """A handle on libstglbm with a torch-owned workspace and stream."""

    def __init__(self, nx, ny, nz, *, device="cuda", stream=None, **desc_kw):
        self.lib = abi.load()
        self.desc = make_desc(nx, ny, nz, **desc_kw)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.q = self.desc.velocity_set or 19
        self.device = torch.device(device)
        self.nbytes = footprint(self.desc)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.handle = ctypes.c_void_p()
        abi.check(self.lib.stglbm_init_lattice(ctypes.byref(self.desc), ctypes.c_void_p(self.workspace.data_ptr()),
                                               self.nbytes, ctypes.c_void_p(self.stream.cuda_stream),
                                               ctypes.byref(self.handle)))
        self.n_modes = 0

    # -- helpers -------------------------------------------------------
    def _chk(self, rc):
        return abi.check(rc, self.handle)

    @property
    def cells(self):
        return self.nx * self.ny * self.nz

    def close(self):
        if self.handle:
            self.lib.stglbm_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the C entry points ---------------------------------------------
    def set_rans_inlet(self, rans, *, delta, nu_phys, c_x, c_t, U_b, n_modes, alpha, seed,
                       C_l=3.0, C_mu=0.09, strict=False):
        y = np.ascontiguousarray(rans["y"], dtype=np.float64)
        U3 = np.ascontiguousarray(rans["U3"], dtype=np.float64)
        k = np.ascontiguousarray(rans["k"], dtype=np.float64)
        om = np.ascontiguousarray(rans["omega"], dtype=np.float64)
        R6 = np.ascontiguousarray(rans["R6"], dtype=np.float64)
        n = y.size
        if U3.shape != (n, 3) or R6.shape != (n, 6) or k.size != n or om.size != n:
            raise ValueError("RANS arrays have inconsistent shapes")
        inl = abi.RansInlet()
        inl.n_rans, inl.n_modes = n, int(n_modes)
        inl.y, inl.U3, inl.k, inl.omega, inl.R6 = _dptr(y), _dptr(U3), _dptr(k), _dptr(om), _dptr(R6)
        inl.delta, inl.nu_phys, inl.c_x, inl.c_t, inl.U_b = delta, nu_phys, c_x, c_t, U_b
        inl.alpha, inl.seed, inl.C_l, inl.C_mu = float(alpha), int(seed), C_l, C_mu
        inl.strict = 1 if strict else 0
        self._chk(self.lib.stglbm_set_rans_inlet(self.handle, ctypes.byref(inl)))
        self.n_modes = int(n_modes)

    def stg_generate(self, t_step, out=None):
        """Inlet plane at step index t_step; returns a (NY, NZ, 3) float32 device tensor."""
        if out is None:
            out = torch.empty((self.ny, self.nz, 3), dtype=torch.float32, device=self.device)
        if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() != self.ny * self.nz * 3:
            raise ValueError("out must be a contiguous float32 tensor of NY*NZ*3 elements")
        self._chk(self.lib.stglbm_stg_generate(self.handle, int(t_step), ctypes.c_void_p(out.data_ptr())))
        return out

    def step(self, n=1):
        self._chk(self.lib.stglbm_step(self.handle, int(n)))

    def step_noalloc(self, n=1):
        """stglbm_step_noalloc: the same steps with the inlet planes staged in the library's static scratch."""
        self._chk(self.lib.stglbm_step_noalloc(self.handle, int(n)))

    def stats_reset(self):
        self._chk(self.lib.stglbm_stats_reset(self.handle))

    def stats_stop(self):
        self._chk(self.lib.stglbm_stats_stop(self.handle))

    def get_stats(self):
        """(sums (NX, NY, 9) float64, number of sampled steps)."""
        out = np.empty((self.nx, self.ny, 9))
        ns = ctypes.c_int64()
        self._chk(self.lib.stglbm_get_stats(self.handle, _dptr(out), out.size, ctypes.byref(ns)))
        return out, ns.value

    def get_f(self):
        out = np.empty((self.q, self.nz, self.ny, self.nx))
        self._chk(self.lib.stglbm_get_f(self.handle, _dptr(out), out.size))
        return out

    def get_f_planes(self, x0, x1):
        out = np.empty((self.q, self.nz, self.ny, x1 - x0))
        self._chk(self.lib.stglbm_get_f_planes(self.handle, int(x0), int(x1), _dptr(out), out.size))
        return out

    def state_view(self):
        """Torch view (Q, NZ, NY, NX) of the current deviations g on the device.

        The device store is [NZ][Q][NY][NX]; the view permutes it (no copy).
        FP32 stores give float32; FP16/BF16 stores give float16/bfloat16.
        Valid until the next step or restore.
        """
        ptr, nb = ctypes.c_void_p(), ctypes.c_uint64()
        self._chk(self.lib.stglbm_state_view(self.handle, ctypes.byref(ptr), ctypes.byref(nb)))
        off = ptr.value - self.workspace.data_ptr()
        dt = {0: torch.float32, 1: torch.float16, 2: torch.bfloat16}[self.desc.store]
        raw = self.workspace[off: off + nb.value]
        return raw.view(dt).view(self.nz, self.q, self.ny, self.nx).permute(1, 0, 2, 3)

    def set_f(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (self.q, self.nz, self.ny, self.nx):
            raise ValueError("f must have shape (Q, NZ, NY, NX)")
        self._chk(self.lib.stglbm_set_f(self.handle, _dptr(f), f.size))

    def set_equilibrium(self, u):
        """Distributions = f_eq(rho = 1, u) for a velocity field u of shape (3, NZ, NY, NX), lattice units."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        if u.shape != (3, self.nz, self.ny, self.nx):
            raise ValueError("u must have shape (3, NZ, NY, NX)")
        self._chk(self.lib.stglbm_set_equilibrium(self.handle, _dptr(u), u.size))

    def set_equilibrium_physical(self, u, c_x, c_t):
        """f_eq(1, u c_t / c_x) for a physical velocity field u (3, NZ, NY, NX), converted by the library."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        if u.shape != (3, self.nz, self.ny, self.nx):
            raise ValueError("u must have shape (3, NZ, NY, NX)")
        self._chk(self.lib.stglbm_set_equilibrium_physical(self.handle, _dptr(u), u.size, float(c_x), float(c_t)))

    def set_probes(self, cells, capacity):
        """Record u at `cells` ((x, y, z) triples, at most 64) after each of the next `capacity` steps.

        Returns the device tensor (capacity, n, 3) float32 the library writes into.
        """
        import torch
        xyz = np.ascontiguousarray(np.asarray(cells, dtype=np.int32).reshape(-1, 3))
        series = torch.zeros((int(capacity), len(xyz), 3), dtype=torch.float32, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()   # the fill must land before the library's writes
        self._chk(self.lib.stglbm_set_probes(self.handle, len(xyz),
                                             xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                             ctypes.c_void_p(series.data_ptr()), int(capacity)))
        self._probe_series = series          # keep the buffer alive while the library writes it
        return series

    def probe_rows(self):
        rows = ctypes.c_int64()
        self._chk(self.lib.stglbm_probe_rows(self.handle, ctypes.byref(rows)))
        return rows.value

    def clear_probes(self):
        self._chk(self.lib.stglbm_set_probes(self.handle, 0, None, None, 0))
        self._probe_series = None

    def get_modes(self):
        out = np.empty((self.n_modes, 8))
        self._chk(self.lib.stglbm_get_modes(self.handle, _dptr(out), out.size))
        return out

    def get_inlet_rows(self):
        out = np.empty((self.ny, abi.ROW_FIELDS))
        self._chk(self.lib.stglbm_get_inlet_rows(self.handle, _dptr(out), out.size))
        return out

    def get_inlet_scalars(self):
        out = np.empty(8)
        self._chk(self.lib.stglbm_get_inlet_scalars(self.handle, _dptr(out), out.size))
        return out

    def get_sqrtq(self):
        out = np.empty((self.ny, self.n_modes))
        self._chk(self.lib.stglbm_get_sqrtq(self.handle, _dptr(out), out.size))
        return out

    def get_step(self):
        t = ctypes.c_int64()
        self._chk(self.lib.stglbm_get_step(self.handle, ctypes.byref(t)))
        return t.value

    def set_stream(self, stream):
        self.stream = stream
        self._chk(self.lib.stglbm_set_stream(self.handle, ctypes.c_void_p(stream.cuda_stream)))

    def sync(self):
        self._chk(self.lib.stglbm_sync(self.handle))

    def checkpoint(self):
        n = ctypes.c_uint64()
        self._chk(self.lib.stglbm_checkpoint_size(self.handle, ctypes.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        self._chk(self.lib.stglbm_checkpoint(self.handle, ctypes.c_void_p(buf.ctypes.data), n.value))
        return buf

    def restore(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._chk(self.lib.stglbm_restore(self.handle, ctypes.c_void_p(buf.ctypes.data), buf.size))

    def profile(self, enable=True, every=1):
        """Time the step kernel (one launch in `every`) and every STG launch with HIP events."""
        self._chk(self.lib.stglbm_profile(self.handle, int(every) if enable else 0))

    def profile_read(self):
        """{'step_ms', 'step_launches', 'stg_ms', 'stg_planes', 'stg_launches', 'tail_planes'} since the last
        read (tail_planes: planes made by the trailing blocks of step launches)."""
        out = np.zeros(6)
        self._chk(self.lib.stglbm_profile_read(self.handle, _dptr(out), 6))
        return {"step_ms": out[0], "step_launches": int(out[1]), "stg_ms": out[2], "stg_planes": int(out[3]),
                "stg_launches": int(out[4]), "tail_planes": int(out[5])}


def channel_from_config(cfg, *, store=None, device="cuda", stream=None, periodic_x=False, max_modes=None,
                        velocity_set=19, collision="regularized"):
    """Build an inlet/outlet channel from a configuration dictionary.

    cfg holds the lattice size, Re_tau-derived physical parameters and the
    RANS arrays (see the workloads package); units are derived by the library.
    """
    rans = cfg["rans"]
    c_x, c_t, nu_lb = derive_units(cfg["delta"], cfg["ny"], cfg["u_b_lb"], rans["U_b"], cfg["nu_phys"])
    n_modes = int(cfg["n_modes"])
    lat = Lattice(cfg["nx"], cfg["ny"], cfg["nz"], device=device, stream=stream,
                  store=store or cfg["store"], periodic_x=periodic_x, nu_lb=nu_lb, cs_smag=cfg["cs_smag"],
                  force=cfg["force"], rho_out=cfg["rho_out"], sponge_cells=cfg["sponge_cells"],
                  sponge_K=cfg["sponge_K"], sponge_p=cfg["sponge_p"],
                  max_modes=max_modes or n_modes, max_rans=len(rans["y"]), velocity_set=velocity_set,
                  collision=collision)
    lat.c_x, lat.c_t, lat.nu_lb = c_x, c_t, nu_lb
    if not periodic_x:
        lat.set_rans_inlet(rans, delta=cfg["delta"], nu_phys=cfg["nu_phys"], c_x=c_x, c_t=c_t, U_b=rans["U_b"],
                           n_modes=n_modes, alpha=cfg["alpha"], seed=cfg["seed"], C_l=cfg["C_l"],
                           C_mu=cfg["C_mu"])
    return lat


def periodic_channel_from_config(cfg, *, store=None, device="cuda", stream=None):
    """Build the force-driven periodic reference channel of a `workloads.periodic_channel` configuration.

    Units come from the library: `stglbm_derive_units`, the body force from the
    physical acceleration by `stglbm_acceleration_to_lattice`, and the start state
    f_eq of the physical start velocity by `stglbm_set_equilibrium_physical`.
    """
    rans = cfg["rans"]
    c_x, c_t, nu_lb = derive_units(cfg["delta"], cfg["ny"], cfg["u_b_lb"], rans["U_b"], cfg["nu_phys"])
    force = acceleration_to_lattice(cfg["force_phys"], c_x, c_t)
    lat = Lattice(cfg["nx"], cfg["ny"], cfg["nz"], device=device, stream=stream, store=store or cfg["store"],
                  periodic_x=True, nu_lb=nu_lb, cs_smag=cfg["cs_smag"], force=force)
    lat.c_x, lat.c_t, lat.nu_lb, lat.force = c_x, c_t, nu_lb, force
    lat.set_equilibrium_physical(cfg["start_velocity_phys"], c_x, c_t)
    return lat
