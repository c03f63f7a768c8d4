"""Precision pattern: FP16/BF16 deviation stores against the FP64 oracle's
long-run channel statistics (64x32x32, 10k warm-up steps, 40k sampled).

The reference is `tests/golden/oracle_stats_64x32x32_w10000_s40000.npz`,
written by `tests/golden/make_oracle_stats.py` with the oracle only.  The
flow is chaotic, so a run in any precision is a different realisation after a
few thousand steps (an accepted reading: results are judged on statistics).
Profiles are the z- and time-means over 2 <= x/delta < 3.5 of U, u_rms,
v_rms, w_rms and uv; the error of a profile is its largest deviation over y
divided by the reference profile's largest magnitude.  The realisation noise
of that comparison is measured, not assumed: a second FP32 run started from
a state perturbed by 1e-9 gives the spread between two equally valid FP32
realisations.
"""

import os

import numpy as np
import pytest

from workloads import channel_config, perturbed_state

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "oracle_stats_64x32x32_w10000_s40000.npz")
WARMUP, STEPS = 10_000, 40_000


def _profiles(st, n, nz, x0, x1):
    s = st[x0:x1] / (n * nz)
    U, V, W = s[..., 0], s[..., 1], s[..., 2]
    P = {"U": U,
         "urms": np.sqrt(np.maximum(s[..., 3] - U * U, 0.0)),
         "vrms": np.sqrt(np.maximum(s[..., 4] - V * V, 0.0)),
         "wrms": np.sqrt(np.maximum(s[..., 5] - W * W, 0.0)),
         "uv": s[..., 6] - U * V}
    return {k: v.mean(axis=0) for k, v in P.items()}


def _err(a, b):
    return {k: float(np.abs(a[k] - b[k]).max() / np.abs(b[k]).max()) for k in b}


def _run(cfg, store, perturb=0.0):
    from paper_2205_02774_amd import channel_from_config
    from oracle.lattice import W
    print(f"[gpu] precision run {cfg['name']} {store} perturb={perturb}", flush=True)
    lat = channel_from_config(cfg, store=store, device="cuda:0")
    if perturb:
        lat.set_f(W[:, None, None, None] + perturb * perturbed_state(cfg["nx"], cfg["ny"], cfg["nz"], seed=11,
                                                                     amplitude=1.0))
    lat.step(WARMUP)
    lat.stats_reset()
    lat.step(STEPS)
    st, n = lat.get_stats()
    lat.close()
    assert n == STEPS
    return st, n


def test_half_stores_against_oracle_statistics():
    cfg = channel_config(0)
    d = cfg["ny"] // 2
    x0, x1 = 2 * d, int(3.5 * d)
    ref = np.load(GOLDEN)
    assert int(ref["n_samples"]) == STEPS and int(ref["warmup"]) == WARMUP
    P_ora = _profiles(ref["stats"], STEPS, cfg["nz"], x0, x1)
    P = {store: _profiles(*_run(cfg, store), cfg["nz"], x0, x1) for store in ("f32", "f16", "bf16")}
    P_alt = _profiles(*_run(cfg, "f32", perturb=1e-9), cfg["nz"], x0, x1)
    noise = _err(P_alt, P["f32"])
    errs = {store: _err(p, P_ora) for store, p in P.items()}
    for name, e in (("FP32 vs FP32 realisation", noise), *((f"{s} vs FP64 oracle", errs[s]) for s in P)):
        print(f"[gpu] {name}: " + ", ".join(f"{k} {100 * v:.2f}%" for k, v in e.items()), flush=True)
    # mean profile: within 1 % of the FP64 oracle for the FP32 and FP16 stores
    assert errs["f32"]["U"] < 0.01 and errs["f16"]["U"] < 0.01
    # second moments: FP32 and FP16 stay within the measured realisation noise
    # band (FP32-vs-FP64 spread or the FP32-vs-FP32 spread, whichever is
    # larger, times 3, and never tighter than 1 %)
    for k in ("urms", "vrms", "wrms", "uv"):
        band = max(0.01, 3.0 * max(noise[k], errs["f32"][k]))
        assert errs["f16"][k] < band, (k, errs["f16"][k], band)
