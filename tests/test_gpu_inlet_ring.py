"""Inlet planes made ahead: one STG launch writes the planes of 16 consecutive
steps, which stglbm_step keeps until used, also across calls.  The results
do not depend on how the steps are split into calls or streams, and a new
inlet takes effect at the next step although planes of the old one were
made ahead."""

import numpy as np
import pytest
import torch

from oracle import OracleChannel
from workloads.configs import small_channel

pytestmark = pytest.mark.gpu


def _channel(cfg):
    from paper_2205_02774_amd import channel_from_config
    return channel_from_config(cfg, device="cuda:0")


def test_planes_do_not_depend_on_call_split():
    cfg = small_channel(24, 16, 8, n_modes=20, seed=4)
    print(f"[gpu] ring split {cfg['name']}", flush=True)
    whole = _channel(cfg)
    whole.step(19)
    ref = whole.get_f()
    whole.close()
    ones = _channel(cfg)
    for _ in range(19):
        ones.step(1)
    np.testing.assert_array_equal(ones.get_f(), ref)
    ones.close()
    mixed = _channel(cfg)
    mixed.step(3)
    mixed.stg_generate(40)          # a plane for the caller between steps
    mixed.step(7)
    s = torch.cuda.Stream(device="cuda:0")
    mixed.set_stream(s)
    mixed.step(9)
    np.testing.assert_array_equal(mixed.get_f(), ref)
    mixed.close()


def test_inlet_replaced_mid_run():
    """A second set_rans_inlet between steps (new seed) takes effect at the next step."""
    cfg = small_channel(24, 16, 8, n_modes=20, seed=4)
    print(f"[gpu] ring new inlet {cfg['name']}", flush=True)
    lat = _channel(cfg)
    ora = OracleChannel.from_config(cfg)
    lat.step(5)
    ora.step(5)
    rans = cfg["rans"]
    lat.set_rans_inlet(rans, delta=cfg["delta"], nu_phys=cfg["nu_phys"], c_x=lat.c_x, c_t=lat.c_t, U_b=rans["U_b"],
                       n_modes=cfg["n_modes"], alpha=cfg["alpha"], seed=cfg["seed"] + 1, C_l=cfg["C_l"],
                       C_mu=cfg["C_mu"])
    ora.set_rans_inlet(rans, cfg["delta"], ora.c_x, ora.c_t, cfg["nu_phys"], rans["U_b"], cfg["n_modes"],
                       cfg["alpha"], cfg["seed"] + 1, cfg["C_l"], cfg["C_mu"])
    lat.step(6)
    ora.step(6)
    rel = np.abs(lat.get_f() - ora.f) / np.abs(ora.f)
    print(f"[gpu] ring new inlet: max rel err f {rel.max():.3e}", flush=True)
    assert rel.max() < 1e-6
    lat.close()


def test_restore_then_step_reproduces():
    cfg = small_channel(24, 16, 8, n_modes=20, seed=4)
    print(f"[gpu] ring restore {cfg['name']}", flush=True)
    lat = _channel(cfg)
    lat.step(2)
    ck = lat.checkpoint()
    lat.step(4)                     # the planes of steps 3 .. 10 are made
    ref = lat.get_f()
    lat.step(9)
    lat.restore(ck)                 # back to step 2
    lat.step(4)
    np.testing.assert_array_equal(lat.get_f(), ref)
    lat.close()


@pytest.mark.parametrize("store,shape", [("f16", (512, 8, 70, 37)), ("bf16", (512, 8, 70, 37)),
                                         ("f32", (512, 8, 70, 37)), ("f16", (520, 7, 33, 3)),
                                         ("f16", (512, 5, 64, 300))])
def test_planes_from_trailing_blocks(store, shape, monkeypatch):
    """16-bit statistics launches of rows of 512 cells (8-wave blocks) make
    the inlet plane of step t + 2 in trailing blocks once the ring's first
    batch is used up (from the 15th step on); FP32 launches never do.  Those
    planes are bit-identical to the plane kernel's (same mode order and the
    same explicit multiply/FMA chain per node), so f and the statistics match
    a run with the trailing blocks switched off (tuning override
    STGLBM_TAIL_STG=0) bit for bit over 40 steps, across calls of different
    lengths and a statistics restart.  Shapes: a ragged spanwise block (NZ =
    70 and 33), NY = 7 and 5 (the last row group of a block partly empty),
    fewer modes than waves (3: five waves sum nothing) and more modes than a
    wave's loads in flight cover in one round (300).  (The plane kernel's
    planes are checked against the oracle's STG in the inlet tests.)"""
    from paper_2205_02774_amd import channel_from_config
    nx, ny, nz, modes = shape
    cfg = small_channel(nx, ny, nz, n_modes=modes, seed=9)
    runs = {}
    for tail in ("1", "0"):
        monkeypatch.setenv("STGLBM_TAIL_STG", tail)
        print(f"[gpu] trailing plane blocks {tail} {store} {cfg['name']}", flush=True)
        lat = channel_from_config(cfg, store=store, device="cuda:0")
        lat.stats_reset()
        lat.profile(True)
        lat.step(13)
        lat.step(1)
        lat.step(11)
        lat.stats_reset()
        lat.step(15)
        prof = lat.profile_read()
        st, n = lat.get_stats()
        runs[tail] = (lat.get_f(), st, n, prof)
        lat.close()
    f1, st1, n1, prof1 = runs["1"]
    f0, st0, n0, prof0 = runs["0"]
    print(f"[gpu] planes: trailing blocks {prof1['tail_planes']} + plane kernel {prof1['stg_planes']}; "
          f"switched off {prof0['tail_planes']} + {prof0['stg_planes']}", flush=True)
    assert prof0["tail_planes"] == 0
    assert prof1["tail_planes"] > 20 if store != "f32" else prof1["tail_planes"] == 0
    assert n1 == n0 == 15
    np.testing.assert_array_equal(f1, f0)
    np.testing.assert_array_equal(st1, st0)
