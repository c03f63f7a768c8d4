"""Periodic, force-driven channel on the GPU: the start-state import, the
exact laminar solution, and parity with the oracle for the reference set-up."""

import numpy as np
import pytest

from oracle import OracleChannel
from oracle import lattice as OL
from workloads import periodic_channel

pytestmark = pytest.mark.gpu


def test_equilibrium_import_matches_oracle():
    """stglbm_set_equilibrium gives f_eq(1, u) of eq. local_eq, rounded once to the store."""
    from paper_2205_02774_amd import Lattice
    nx, ny, nz = 20, 6, 3
    rng = np.random.default_rng(8)
    u = rng.uniform(-0.08, 0.08, size=(3, nz, ny, nx))
    ref = OL.equilibrium(np.ones((nz, ny, nx)), u)
    # rounding unit and, for FP16, half its subnormal spacing (small |g| are subnormal there)
    for store, unit, floor in (("f32", 2.0 ** -24, 0.0), ("f16", 2.0 ** -11, 2.0 ** -25), ("bf16", 2.0 ** -8, 0.0)):
        print(f"[gpu] equilibrium import {store}", flush=True)
        lat = Lattice(nx, ny, nz, device="cuda:0", store=store, periodic_x=True, nu_lb=1e-2)
        lat.set_equilibrium(u)
        f = lat.get_f()
        lat.close()
        w = OL.W[:, None, None, None]
        # one rounding of g = f - w to the store (plus the FP64->FP32 step for 16-bit stores)
        bound = (unit + 2.0 ** -24) * np.abs(ref - w) + floor + 1e-15
        assert np.all(np.abs(f - ref) <= bound), store


def test_poiseuille_matches_closed_form():
    """Laminar forced channel: halfway bounce-back + Guo force + the regularized
    operator reproduce the parabola u = F/(2 nu) eta (NY - eta), eta = y + 1/2,
    exactly at tau = 7/8 (the oracle pins the same identity in FP64)."""
    from paper_2205_02774_amd import Lattice
    nx, ny, nz, F = 4, 16, 2, 1e-5
    tau = 0.875
    nu = (tau - 0.5) / 3.0
    lat = Lattice(nx, ny, nz, device="cuda:0", store="f32", periodic_x=True, nu_lb=nu, cs_smag=0.0,
                  force=(F, 0.0, 0.0))
    lat.step(int(5 * ny * ny / nu))
    lat.stats_reset()
    lat.step(10)
    st, n = lat.get_stats()
    lat.close()
    u = st[..., 0] / (n * nz)                    # (NX, NY) mean u_x
    eta = np.arange(ny) + 0.5
    exact = F / (2.0 * nu) * eta * (ny - eta)
    err = np.abs(u - exact[None, :]).max() / exact.max()
    print(f"[gpu] Poiseuille tau=7/8: max |u - exact| / u_max = {err:.3e} (u_max {exact.max():.3e})", flush=True)
    assert err < 1e-5
    assert np.abs(st[..., 1:3]).max() / (n * nz) < 1e-6 * exact.max()


@pytest.mark.parametrize("store,tol", [("f32", 1e-6)])
def test_periodic_reference_parity(store, tol):
    """The force-driven periodic reference channel from its perturbed start, 100 steps."""
    from paper_2205_02774_amd import periodic_channel_from_config
    cfg = periodic_channel(24, 16, 8, seed=3)
    print(f"[gpu] periodic reference {cfg['name']} {store}", flush=True)
    lat = periodic_channel_from_config(cfg, store=store, device="cuda:0")
    ora = OracleChannel.periodic_from_config(cfg)
    assert lat.force[0] == pytest.approx(ora.force[0], rel=1e-14)
    ora.set_f(lat.get_f())                         # compare from the same (rounded) start
    lat.stats_reset()
    ora.stats_reset()
    lat.step(100)
    ora.step(100)
    f = lat.get_f()
    rel = np.abs(f - ora.f) / np.abs(ora.f)
    print(f"[gpu] periodic reference: max rel err f after 100 steps {rel.max():.3e}", flush=True)
    assert rel.max() < tol
    st, n = lat.get_stats()
    nrm = np.linalg.norm(st - ora.stats) / np.linalg.norm(ora.stats)
    print(f"[gpu] periodic reference: stats normwise rel err {nrm:.3e}", flush=True)
    assert nrm < 1e-6
    lat.close()
