"""Lattice configurations and seeded job mixes (inputs only).

Each configuration names a synthetic turbulent channel: lattice size
NX x NY x NZ (x streamwise with the inlet at x = 0 and the outlet at x = NX-1,
y wall-normal between two walls, z spanwise and periodic), the friction
Reynolds number, the storage type of the distributions, the STG mode count
and spacing, the seed of the mode draw, and the RANS input on its own y-grid.

Physical units follow the paper's channel: half-height delta = 1 m,
u_tau = 1 m/s, nu = 1/Re_tau.  The lattice half-height is NY/2 cells and the
lattice bulk velocity is fixed by u_b_lb (0.05 lattice units).
"""

import numpy as np

from .rans import channel_rans_profile, stretched_fv_grid, bulk_velocity_fv

CONFIG_NAMES = ("channel-64x32x32", "channel-512x128x256",
                "channel-512x128x256-f16", "channel-1024x256x512-f16")


def _rans_on_rows(ny, re_tau):
    """RANS fields evaluated directly at the lattice rows y_j = (j + 1/2) dx."""
    delta = 1.0
    dx = 2.0 * delta / ny
    y = (np.arange(ny) + 0.5) * dx
    prof = channel_rans_profile(y, re_tau, delta)
    prof["U_b"] = bulk_velocity_fv(prof["U3"][:, 0], np.full(ny, dx), delta)
    return prof


def _rans_on_fv_grid(n_cells, ratio, re_tau):
    centres, widths = stretched_fv_grid(n_cells, ratio, 1.0)
    prof = channel_rans_profile(centres, re_tau, 1.0)
    prof["U_b"] = bulk_velocity_fv(prof["U3"][:, 0], widths, 1.0)
    return prof


def channel_config(name_or_index, store=None):
    """Return the input dictionary of a named channel configuration."""
    names = {0: CONFIG_NAMES[0], 1: CONFIG_NAMES[1], 2: CONFIG_NAMES[2], 3: CONFIG_NAMES[3]}
    name = names.get(name_or_index, name_or_index)
    if name == "channel-64x32x32":
        cfg = dict(nx=64, ny=32, nz=32, store="f32", re_tau=180.0, n_modes=50,
                   alpha=0.05, seed=0, steps=200)
        cfg["rans"] = _rans_on_rows(cfg["ny"], cfg["re_tau"])
        cfg["rans_grid"] = "analytic at lattice rows"
    elif name in ("channel-512x128x256", "channel-512x128x256-f16"):
        cfg = dict(nx=512, ny=128, nz=256, store="f32" if name.endswith("256") else "f16",
                   re_tau=180.0, n_modes=600, alpha=0.0, seed=1, steps=1000, warmup=20000)
        cfg["rans"] = _rans_on_fv_grid(96, 1.04, cfg["re_tau"])
        cfg["rans_grid"] = "96-cell stretched FV grid, ratio 1.04"
    elif name == "channel-1024x256x512-f16":
        cfg = dict(nx=1024, ny=256, nz=512, store="f16", re_tau=550.0, n_modes=1000,
                   alpha=0.0, seed=3, steps=500, warmup=1000)
        cfg["rans"] = _rans_on_fv_grid(160, 1.04, cfg["re_tau"])
        cfg["rans_grid"] = "160-cell stretched FV grid, ratio 1.04"
    else:
        raise KeyError(name)
    if store is not None:
        cfg["store"] = store
    cfg["name"] = name
    _common(cfg)
    return cfg


def small_channel(nx, ny, nz, re_tau=180.0, n_modes=50, alpha=0.05, seed=0, store="f32"):
    """A channel of arbitrary size with the RANS input evaluated at its rows."""
    cfg = dict(nx=nx, ny=ny, nz=nz, store=store, re_tau=re_tau, n_modes=n_modes,
               alpha=alpha, seed=seed, name=f"channel-{nx}x{ny}x{nz}")
    cfg["rans"] = _rans_on_rows(ny, re_tau)
    _common(cfg)
    return cfg


def periodic_channel(nx, ny, nz, re_tau=180.0, store="f32", seed=0, amplitude=0.1):
    """Channel periodic in x and z, driven by the mean pressure gradient as a body force.

    This is the paper's LES-LBM reference set-up (periodic channel with a
    body force in place of the inlet and outlet).  The force is the physical
    acceleration u_tau^2 / delta = 1 m/s^2 along x that balances the wall
    shear in the mean.  The start state is the RANS mean velocity at the
    lattice rows plus a seeded perturbation, in physical units:
    `start_velocity_phys` (3, NZ, NY, NX) holds U(y) in the streamwise
    component plus U_b times uniform numbers in (-amplitude, amplitude) in
    every component.
    """
    cfg = dict(nx=nx, ny=ny, nz=nz, store=store, re_tau=re_tau, n_modes=0, alpha=0.0, seed=seed,
               name=f"periodic-{nx}x{ny}x{nz}", periodic_x=True)
    cfg["rans"] = _rans_on_rows(ny, re_tau)
    cfg["force_phys"] = (1.0, 0.0, 0.0)
    rng = np.random.default_rng(seed)
    u = cfg["rans"]["U_b"] * rng.uniform(-amplitude, amplitude, size=(3, nz, ny, nx))
    u[0] += cfg["rans"]["U3"][:, 0][None, :, None]
    cfg["start_velocity_phys"] = u
    _common(cfg)
    cfg["sponge_cells"] = 0
    return cfg


def _common(cfg):
    cfg.setdefault("delta", 1.0)
    cfg.setdefault("u_tau", 1.0)
    cfg["nu_phys"] = cfg["u_tau"] * cfg["delta"] / cfg["re_tau"]
    cfg.setdefault("u_b_lb", 0.05)
    cfg.setdefault("cs_smag", 0.1)
    cfg.setdefault("rho_out", 1.0)
    cfg.setdefault("sponge_K", 1000.0)
    cfg.setdefault("sponge_p", 3.0)
    # sponge zone 0.4 delta long, in whole cells (delta = NY/2 cells)
    cfg.setdefault("sponge_cells", int(round(0.4 * cfg["ny"] / 2)))
    cfg.setdefault("C_l", 3.0)
    cfg.setdefault("C_mu", 0.09)
    cfg.setdefault("force", (0.0, 0.0, 0.0))
    cfg["cells"] = cfg["nx"] * cfg["ny"] * cfg["nz"]
    return cfg


def perturbed_state(nx, ny, nz, seed, amplitude=1e-3):
    """Seeded random deviations g_i (19 x NZ x NY x NX), scaled per direction.

    g_i = a_i * amplitude * U(-1, 1) with a_i = 1/3, 1/18 or 1/36 for the rest,
    axis and diagonal directions respectively, so f_i = w_i + g_i stays positive.
    """
    rng = np.random.default_rng(seed)
    scale = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
    g = rng.uniform(-1.0, 1.0, size=(19, nz, ny, nx)) * amplitude
    return g * scale[:, None, None, None]


LADDER = ((64, 32, 32), (128, 64, 64), (256, 64, 128), (512, 128, 256))


def job_config(job):
    """Channel configuration of a serving job (RANS input evaluated at its lattice rows)."""
    cfg = small_channel(job["nx"], job["ny"], job["nz"], re_tau=job["re_tau"], n_modes=job["n_modes"],
                        alpha=job.get("alpha", 0.0), seed=job["seed"], store=job["store"])
    if "u_b_lb" in job:
        cfg["u_b_lb"] = job["u_b_lb"]
    return cfg


def serving_jobs(n_jobs=64, seed=4, rate_per_s=2.0, ladder=LADDER,
                 steps_range=(1000, 20000), modes_range=(50, 600)):
    """Seeded serving mix: Poisson arrivals and per-job channel parameters."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_jobs)
    arrivals = np.cumsum(gaps) - gaps[0]
    jobs = []
    for j in range(n_jobs):
        nx, ny, nz = ladder[int(rng.integers(len(ladder)))]
        jobs.append(dict(
            id=j,
            arrival_s=float(arrivals[j]),
            re_tau=float(rng.choice([180.0, 395.0, 550.0])),
            nx=nx, ny=ny, nz=nz,
            n_modes=int(rng.integers(modes_range[0], modes_range[1] + 1)),
            steps=int(rng.integers(steps_range[0], steps_range[1] + 1)),
            store=str(rng.choice(["f32", "f16"])),
            seed=1000 + j,
        ))
    return jobs
