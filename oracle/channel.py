"""Algorithm 1 (STG-LBM) driven step by step, FP64 (test infrastructure).

State: post-collision distributions f[i, z, y, x], the step index t (the
number of completed steps), and per-(x, y) FP64 statistics sums.  One step
n -> n+1 generates the inlet plane at t = n+1 (Algorithm 1, steps 5-8),
streams, rebuilds the inlet and outlet planes (steps 9-11), collides every
cell (step 12) and, when sampling, adds the velocity the collision used to
the statistics.  The initial state is rest, f = w_i (Results section).
"""

import numpy as np

from . import lattice as L
from . import units
from .stg import InletGenerator


class OracleChannel:
    def __init__(self, nx, ny, nz, *, nu_lb, cs_smag=0.1, force=(0.0, 0.0, 0.0),
                 periodic_x=False, rho_out=1.0, sponge_cells=0, sponge_K=1000.0, sponge_p=3.0,
                 periodic_y=False, operator="regularized", velocity_set=19):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.nu_lb = nu_lb
        self.tau0 = units.tau_from_nu(nu_lb)
        self.cs_smag = cs_smag
        self.force = tuple(float(v) for v in force)
        self.periodic_x = periodic_x
        self.periodic_y = periodic_y        # oracle-only self-test option
        self.operator = operator            # "regularized" or "bgk" (plain BGK bulk, eq. lbe)
        self.vs = L.velocity_set(velocity_set)
        self.rho_out = rho_out
        self.sponge = L.sponge_factor(nx, 0 if periodic_x else sponge_cells, sponge_K, sponge_p)
        self.f = np.broadcast_to(self.vs.W[:, None, None, None], (self.vs.Q, nz, ny, nx)).copy()
        self.t = 0
        self.inlet = None
        self.stats = np.zeros((nx, ny, 9))
        self.n_samples = 0
        self.sampling = False
        self.guard_violations = 0

    @classmethod
    def from_config(cls, cfg, periodic_x=False, operator="regularized", velocity_set=19):
        """Build from a workloads configuration (units derived here, FP64)."""
        rans = cfg["rans"]
        c_x, c_t, nu_lb, _ = units.channel_units(cfg["delta"], cfg["ny"], cfg["u_b_lb"],
                                                 rans["U_b"], cfg["nu_phys"])
        ch = cls(cfg["nx"], cfg["ny"], cfg["nz"], nu_lb=nu_lb, cs_smag=cfg["cs_smag"],
                 force=cfg["force"], periodic_x=periodic_x, rho_out=cfg["rho_out"],
                 sponge_cells=cfg["sponge_cells"], sponge_K=cfg["sponge_K"], sponge_p=cfg["sponge_p"],
                 operator=operator, velocity_set=velocity_set)
        ch.c_x, ch.c_t = c_x, c_t
        if not periodic_x:
            ch.set_rans_inlet(rans, cfg["delta"], c_x, c_t, cfg["nu_phys"], rans["U_b"],
                              cfg["n_modes"], cfg["alpha"], cfg["seed"], cfg["C_l"], cfg["C_mu"])
        return ch

    @classmethod
    def periodic_from_config(cls, cfg):
        """The force-driven periodic reference channel (Numerical setup: periodic
        LES-LBM channel with a body force).  The physical acceleration and the
        start velocity are converted to lattice units (force F c_t^2/c_x,
        velocity u c_t/c_x) and the start state is f_eq(1, u) (eq. local_eq)."""
        rans = cfg["rans"]
        c_x, c_t, nu_lb, _ = units.channel_units(cfg["delta"], cfg["ny"], cfg["u_b_lb"],
                                                 rans["U_b"], cfg["nu_phys"])
        force = tuple(units.acceleration_to_lattice(a, c_t, c_x) for a in cfg["force_phys"])
        ch = cls(cfg["nx"], cfg["ny"], cfg["nz"], nu_lb=nu_lb, cs_smag=cfg["cs_smag"], force=force,
                 periodic_x=True)
        ch.c_x, ch.c_t = c_x, c_t
        u0 = units.velocity_to_lattice(np.asarray(cfg["start_velocity_phys"], dtype=np.float64), c_t, c_x)
        ch.set_f(L.equilibrium(np.ones(u0.shape[1:]), u0))
        return ch

    def set_rans_inlet(self, rans, delta, c_x, c_t, nu_phys, U_b, n_modes, alpha, seed,
                       C_l=3.0, C_mu=0.09):
        self.inlet = InletGenerator(rans, self.ny, self.nz, delta, c_x, c_t, nu_phys, U_b,
                                    n_modes, alpha, seed, C_l, C_mu)

    def set_f(self, f):
        self.f = np.array(f, dtype=np.float64, copy=True)

    def stats_reset(self):
        self.stats[:] = 0.0
        self.n_samples = 0
        self.sampling = True

    def inlet_plane(self, t_step):
        """u_bc (NY, NZ, 3) in lattice units for the state at step index t_step."""
        return self.inlet.plane(t_step)

    def step(self, n=1):
        for _ in range(n):
            u_bc = None
            if not self.periodic_x:
                plane = self.inlet_plane(self.t + 1)
                # density_bc: |u.n| < 0.3 c_s at the inlet
                self.guard_violations += int(np.sum(np.abs(plane[:, :, 0]) >= 0.3 * units.CS))
                u_bc = plane.transpose(2, 1, 0)          # (3, NZ, NY)
            self.f, rho, u = L.lattice_step(self.f, tau0=self.tau0, cs_smag=self.cs_smag,
                                            force=self.force, sponge=self.sponge,
                                            periodic_x=self.periodic_x, u_bc_zy=u_bc,
                                            rho_out=self.rho_out, periodic_y=self.periodic_y,
                                            operator=self.operator)
            self.last_rho, self.last_u = rho, u
            if self.sampling:
                self.stats += L.stats_bins(u)
                self.n_samples += 1
            self.t += 1
        return self
