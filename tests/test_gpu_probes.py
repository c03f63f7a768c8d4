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


@pytest.mark.parametrize("q,store", [(27, "f32"), (15, "f16"), (19, "bf16")])
def test_probe_rows_match_the_state(q, store):
    """Every velocity set and store: row s equals (sum c f - F/2) / rho of the
    state after step s at the probed cells (periodic box with a Guo force)."""
    from paper_2205_02774_amd import Lattice
    from oracle.lattice import velocity_set
    vs = velocity_set(q)
    nx, ny, nz, force = 20, 9, 6, (3e-5, -1e-5, 2e-5)
    cells = [(0, 0, 0), (19, 8, 5), (7, 4, 2), (13, 1, 3)]
    steps = 6
    print(f"[gpu] probes D3Q{q} {store}", flush=True)
    lat = Lattice(nx, ny, nz, device="cuda:0", periodic_x=True, nu_lb=2e-2, cs_smag=0.1, force=force,
                  store=store, velocity_set=q)
    rng = np.random.default_rng(q)
    W = vs.W[:, None, None, None]
    lat.set_f(W * (1.0 + 5e-2 * rng.uniform(-1, 1, (q, nz, ny, nx))))
    series = lat.set_probes(cells, capacity=steps)
    ref = np.empty((steps, len(cells), 3))
    for s in range(steps):
        lat.step(1)
        f = lat.get_f()
        for k, (x, y, z) in enumerate(cells):
            fc = f[:, z, y, x]
            ref[s, k] = (vs.C.T @ fc - 0.5 * np.asarray(force)) / fc.sum()
    lat.sync()
    got = series.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"[gpu] probes D3Q{q} {store}: max |u_probe - u_state| / max|u| = {err:.3e}", flush=True)
    assert err < 1e-5
    lat.close()
