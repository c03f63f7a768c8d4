"""Velocity probes (adaptation diagnostics) against the oracle, step by step."""

import numpy as np
import pytest

from oracle import OracleChannel
from workloads import channel_config

pytestmark = pytest.mark.gpu


def test_probe_series_matches_oracle():
    """Each probe row is the velocity the collision used at that cell in that step."""
    from paper_2205_02774_amd import channel_from_config, abi
    cfg = channel_config(0)
    cells = [(0, 5, 3), (1, 0, 7), (16, 12, 31), (32, 31, 0), (63, 20, 16), (62, 16, 16)]
    steps = 40
    print(f"[gpu] probes on {cfg['name']}: {len(cells)} cells, {steps} steps", flush=True)
    lat = channel_from_config(cfg, device="cuda:0")
    series = lat.set_probes(cells, capacity=steps)
    ora = OracleChannel.from_config(cfg)
    ref = np.empty((steps, len(cells), 3))
    for s in range(steps):
        ora.step(1)
        for k, (x, y, z) in enumerate(cells):
            ref[s, k] = ora.last_u[:, z, y, x]
    lat.step(steps + 5)                       # rows stop at the capacity
    lat.sync()
    assert lat.probe_rows() == steps
    got = series.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"[gpu] probes: max |u_gpu - u_oracle| / max|u| = {err:.3e}", flush=True)
    assert err < 1e-5
    with pytest.raises(abi.StglbmError) as e:
        lat.set_probes([(64, 0, 0)], capacity=4)
    assert e.value.code == abi.E_INVAL
    lat.clear_probes()
    lat.step(2)
    assert lat.probe_rows() == 0
    lat.close()
