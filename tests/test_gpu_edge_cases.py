"""Degenerate sizes against the oracle: the smallest legal lattices, a single
spanwise slice (z - 1 = z = z + 1), and zero steps."""

import numpy as np
import pytest

from oracle import OracleChannel
from workloads.configs import small_channel

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return np.abs(a - b) / np.abs(b)


@pytest.mark.parametrize("shape", [(2, 2, 1), (3, 2, 1), (5, 3, 1), (2, 2, 3)])
def test_smallest_periodic_lattices(shape):
    from paper_2205_02774_amd import Lattice
    from oracle.lattice import W
    nx, ny, nz = shape
    nu, cs, force = 2e-2, 0.1, (1e-5, 0.0, 0.0)
    print(f"[gpu] edge periodic {shape}", flush=True)
    lat = Lattice(nx, ny, nz, device="cuda:0", periodic_x=True, nu_lb=nu, cs_smag=cs, force=force)
    ora = OracleChannel(nx, ny, nz, nu_lb=nu, cs_smag=cs, force=force, periodic_x=True)
    rng = np.random.default_rng(1)
    lat.set_f(W[:, None, None, None] * (1.0 + 1e-2 * rng.uniform(-1, 1, (19, nz, ny, nx))))
    ora.set_f(lat.get_f())
    lat.stats_reset()
    ora.stats_reset()
    lat.step(50)
    ora.step(50)
    rel = _rel(lat.get_f(), ora.f)
    st, n = lat.get_stats()
    print(f"[gpu] edge periodic {shape}: max rel err f {rel.max():.3e}", flush=True)
    assert rel.max() < 1e-6 and n == 50
    np.testing.assert_allclose(st, ora.stats, rtol=0, atol=1e-6 * np.abs(ora.stats).max() + 1e-12)
    lat.close()


@pytest.mark.parametrize("shape", [(2, 4, 1), (3, 6, 2), (65, 4, 1)])
def test_smallest_inlet_outlet_channels(shape):
    """Inlet and outlet planes adjacent (NX = 2) or one cell apart, single spanwise slice.

    Channels this small are far from resolved: the inlet drives the populations
    far from equilibrium (|f - w| up to 3 w, some f below zero), and FP32
    rounding grows by about 1e-7 per step, so a free run drifts past 1e-6 within
    ten steps however exact the kernel is.  The map itself is checked instead:
    both sides step in lockstep and the oracle restarts from the GPU state
    before every step, so each comparison holds one step of rounding.  The
    scale of population i is max(|f_i|, w_i): the store holds f - w and the
    arithmetic works on terms of size w_i, so f_i near zero has no smaller floor.
    """
    from paper_2205_02774_amd import channel_from_config
    from oracle.lattice import W
    nx, ny, nz = shape
    cfg = small_channel(nx, ny, nz, n_modes=5, seed=9)
    cfg["sponge_cells"] = min(cfg["sponge_cells"], nx - 2)   # the sponge must end before the inlet
    print(f"[gpu] edge channel {cfg['name']}", flush=True)
    lat = channel_from_config(cfg, device="cuda:0")
    ora = OracleChannel.from_config(cfg)
    scale_w = W[:, None, None, None]
    worst = 0.0
    for _ in range(30):
        lat.step(1)
        ora.step(1)
        f = lat.get_f()
        worst = max(worst, float((np.abs(f - ora.f) / np.maximum(np.abs(ora.f), scale_w)).max()))
        ora.set_f(f)
    print(f"[gpu] edge channel {cfg['name']}: max one-step rel err f {worst:.3e}", flush=True)
    assert worst < 1e-6
    assert ora.t == 30
    lat.close()


def test_zero_steps_is_a_no_op():
    from paper_2205_02774_amd import channel_from_config
    cfg = small_channel(16, 8, 4, n_modes=5, seed=2)
    lat = channel_from_config(cfg, device="cuda:0")
    lat.step(3)
    f0 = lat.get_f()
    lat.step(0)
    np.testing.assert_array_equal(lat.get_f(), f0)
    lat.close()


def test_profile_times_one_launch_in_every():
    """stglbm_profile(k): every STG launch and the step kernel on steps 0, k, 2k, ... after the call."""
    from paper_2205_02774_amd import abi, channel_from_config
    cfg = small_channel(24, 16, 8, n_modes=10, seed=3)
    lat = channel_from_config(cfg, device="cuda:0")
    lat.profile(True, every=4)
    lat.step(20)            # steps 0, 4, ..., 16 timed; planes made 16 at a time: 2 STG launches
    pr = lat.profile_read()
    assert pr["step_launches"] == 5 and pr["stg_launches"] == 2 and pr["stg_planes"] == 32
    assert pr["step_ms"] > 0.0 and pr["stg_ms"] > 0.0
    lat.profile(True)
    lat.step(5)
    pr = lat.profile_read()
    assert pr["step_launches"] == 5
    lat.profile(False)
    lat.step(2)
    assert lat.profile_read()["step_launches"] == 0
    with pytest.raises(abi.StglbmError) as e:
        lat._chk(lat.lib.stglbm_profile(lat.handle, -1))
    assert e.value.code == abi.E_INVAL
    lat.close()


@pytest.mark.parametrize("store,shape", [("f32", (581, 4, 6)), ("f16", (581, 4, 6)), ("f32", (1030, 4, 8))])
def test_rows_wider_than_one_block_with_idle_waves(store, shape):
    """Rows wider than one block, the last block of a row partly idle.

    NX = 581: 10 tiles of 64, whole-row blocks of 8 waves, so the second
    block of each row has 2 working waves and 6 that only keep step with
    them (statistics launches hold a barrier per z row; FP32 ones run two z
    waves per block).  NX = 1030: 17 tiles in three blocks per row, the
    third with one working wave; its 48 FP32 statistics blocks are renumbered
    so that the three blocks of a row share an XCD."""
    from paper_2205_02774_amd import Lattice
    from oracle.lattice import W
    nx, ny, nz = shape
    nu, cs, force = 2e-2, 0.1, (1e-5, 0.0, 0.0)
    print(f"[gpu] edge wide rows {store} {shape}", flush=True)
    lat = Lattice(nx, ny, nz, device="cuda:0", store=store, periodic_x=True, nu_lb=nu, cs_smag=cs, force=force)
    ora = OracleChannel(nx, ny, nz, nu_lb=nu, cs_smag=cs, force=force, periodic_x=True)
    rng = np.random.default_rng(11)
    lat.set_f(W[:, None, None, None] * (1.0 + 1e-2 * rng.uniform(-1, 1, (19, nz, ny, nx))))
    ora.set_f(lat.get_f())
    lat.stats_reset()
    ora.stats_reset()
    lat.step(30)
    ora.step(30)
    st, n = lat.get_stats()
    f = lat.get_f()
    lat.close()
    rel = _rel(f, ora.f)
    nrm = np.linalg.norm(st - ora.stats) / np.linalg.norm(ora.stats)
    print(f"[gpu] edge wide rows {store} {shape}: max rel err f {rel.max():.3e}, stats {nrm:.3e}", flush=True)
    assert n == 30
    if store == "f32":
        assert rel.max() < 1e-6 and nrm < 1e-6
    else:
        # 16-bit store: every step rounds g to 2^-11 relative; |g/f| <= 1e-2 here
        assert rel.max() < 4 * np.sqrt(30) * 2.0 ** -11 * 2e-2 and nrm < 1e-3


def test_statistics_without_per_row_barrier(monkeypatch):
    """The tuning override STGLBM_LOCKSTEP=0 drops the per-row barrier of the
    statistics launches (the two z waves of an FP32 block then run free and
    may leave the z loop at different trips); results stay those of the oracle."""
    from paper_2205_02774_amd import Lattice
    from oracle.lattice import W
    monkeypatch.setenv("STGLBM_LOCKSTEP", "0")
    nx, ny, nz = 581, 4, 7
    nu, cs, force = 2e-2, 0.1, (1e-5, 0.0, 0.0)
    print("[gpu] edge statistics without the per-row barrier", flush=True)
    lat = Lattice(nx, ny, nz, device="cuda:0", periodic_x=True, nu_lb=nu, cs_smag=cs, force=force)
    ora = OracleChannel(nx, ny, nz, nu_lb=nu, cs_smag=cs, force=force, periodic_x=True)
    rng = np.random.default_rng(12)
    lat.set_f(W[:, None, None, None] * (1.0 + 1e-2 * rng.uniform(-1, 1, (19, nz, ny, nx))))
    ora.set_f(lat.get_f())
    lat.stats_reset()
    ora.stats_reset()
    lat.step(20)
    ora.step(20)
    st, n = lat.get_stats()
    f = lat.get_f()
    lat.close()
    rel = _rel(f, ora.f)
    nrm = np.linalg.norm(st - ora.stats) / np.linalg.norm(ora.stats)
    print(f"[gpu] edge no barrier: max rel err f {rel.max():.3e}, stats {nrm:.3e}", flush=True)
    assert n == 20 and rel.max() < 1e-6 and nrm < 1e-6
