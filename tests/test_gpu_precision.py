"""Precision pattern: the FP16 deviation store against FP32 and the FP64 oracle,
compared on long-run channel statistics (64x32x32, 10k warm-up steps, 40k sampled).

The flow is chaotic, so a run in any precision is a different realisation
after a few thousand steps (an accepted reading: results are compared as
statistics), and a single run cannot resolve a 1 % bound on the second
moments: equally valid FP32 realisations differ by several per cent there.
The stores are therefore compared as ensembles.  Each member starts from
rest plus a seeded deviation a w_i U(-1, 1) and shares the inlet.  The
window statistics of this small channel also depend on the size of that
start deviation: ensembles started with a = 1e-9, 1e-4 and 1e-2 have means
whose w_rms, u_rms and uv differ by up to 8 % (measured on MI355X), far more
than their standard errors.  So each comparison is made within one class of
start states:

* FP16 against FP32: M members each with a = 1e-4 (seed 100 + m; the
  smallest class the FP16 import keeps), the same start states for both
  stores.  Bar: every profile of the FP16 ensemble mean within 1 % of the
  FP32 ensemble mean (L2 over y), with a standard error of that difference
  below 1 %.
* FP32 against the FP64 oracle: the oracle's long run starts from rest
  (`tests/golden/oracle_stats_64x32x32_w10000_s40000.npz`, written by
  `tests/golden/make_oracle_stats.py` with the oracle only); the FP32 members
  of its class start from rest or with a = 1e-9 (seed 200 + m).  Its profiles
  must lie within the spread of those members around their mean.

Profiles are the z- and time-means over 2 <= x/delta < 3.5 of U, u_rms,
v_rms, w_rms and uv.  Errors are L2-relative over y, ||P - P_ref|| /
||P_ref||, reported beside the max-norm; the standard error of a difference
of two ensemble means is the L2 norm of their per-row standard errors
combined in quadrature, relative to ||P_ref||.  BF16 runs one member of the
first class for the record.
"""

import os

import numpy as np
import pytest
import torch

from workloads import channel_config, perturbed_state

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "oracle_stats_64x32x32_w10000_s40000.npz")
WARMUP, STEPS = 10_000, 40_000
MEMBERS = 48       # per store, start deviation 1e-4
REST_MEMBERS = 24  # FP32, from rest and with start deviation 1e-9
GROUP = 8          # members stepped concurrently, one stream each
CHUNK = 1000
KEYS = ("U", "urms", "vrms", "wrms", "uv")


def _profiles(st, n, nz, x0, x1):
    s = st[x0:x1] / (n * nz)
    U, V, W = s[..., 0], s[..., 1], s[..., 2]
    P = {"U": U,
         "urms": np.sqrt(np.maximum(s[..., 3] - U * U, 0.0)),
         "vrms": np.sqrt(np.maximum(s[..., 4] - V * V, 0.0)),
         "wrms": np.sqrt(np.maximum(s[..., 5] - W * W, 0.0)),
         "uv": s[..., 6] - U * V}
    return {k: v.mean(axis=0) for k, v in P.items()}


def _l2(a, ref):
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))


def _maxrel(a, ref):
    return float(np.abs(a - ref).max() / np.abs(ref).max())


def _members(cfg, store, starts, x0, x1):
    """Profiles of one run per (seed, amplitude) start (seed None: rest), GROUP runs at a time on their own streams."""
    from paper_2205_02774_amd import channel_from_config
    from oracle.lattice import W
    out = []
    for g0 in range(0, len(starts), GROUP):
        group = starts[g0:g0 + GROUP]
        print(f"[gpu] precision ensemble {store}: members {g0}..{g0 + len(group) - 1}", flush=True)
        runs = []
        for seed, amp in group:
            stream = torch.cuda.Stream(device="cuda:0")
            lat = channel_from_config(cfg, store=store, device="cuda:0", stream=stream)
            if seed is not None:
                lat.set_f(W[:, None, None, None] + perturbed_state(cfg["nx"], cfg["ny"], cfg["nz"], seed=seed,
                                                                   amplitude=amp))
            runs.append(lat)
        for phase, total in (("warm-up", WARMUP), ("sampled", STEPS)):
            if phase == "sampled":
                for lat in runs:
                    lat.stats_reset()
            for _ in range(0, total, CHUNK):
                for lat in runs:
                    lat.step(CHUNK)
            for lat in runs:
                lat.sync()
        for lat in runs:
            st, n = lat.get_stats()
            assert n == STEPS
            out.append(_profiles(st, n, cfg["nz"], x0, x1))
            lat.close()
    return {k: np.stack([p[k] for p in out]) for k in KEYS}


def test_fp16_store_ensemble_statistics():
    cfg = channel_config(0)
    d = cfg["ny"] // 2
    x0, x1 = 2 * d, int(3.5 * d)
    ref = np.load(GOLDEN)
    assert int(ref["n_samples"]) == STEPS and int(ref["warmup"]) == WARMUP
    P_ora = _profiles(ref["stats"], STEPS, cfg["nz"], x0, x1)
    starts = [(100 + m, 1e-4) for m in range(MEMBERS)]
    ens = {store: _members(cfg, store, starts, x0, x1) for store in ("f32", "f16")}
    rest = _members(cfg, "f32", [(None, 0.0)] + [(200 + m, 1e-9) for m in range(REST_MEMBERS - 1)], x0, x1)
    bf16 = _members(cfg, "bf16", starts[:1], x0, x1)
    failures = []
    for k in KEYS:
        m32, m16, mrest = ens["f32"][k].mean(0), ens["f16"][k].mean(0), rest[k].mean(0)
        se32, se16 = (ens[s][k].std(0, ddof=1) / np.sqrt(MEMBERS) for s in ("f32", "f16"))
        err = _l2(m16, m32)
        se_diff = float(np.linalg.norm(np.hypot(se16, se32)) / np.linalg.norm(m32))
        spread = np.array([_l2(m, mrest) for m in rest[k]])
        d_ora = _l2(P_ora[k], mrest)
        print(f"[gpu] {k}: FP16 vs FP32 ensemble mean L2 {100 * err:.2f}% (max-norm {100 * _maxrel(m16, m32):.2f}%), "
              f"standard error {100 * se_diff:.2f}%; FP32 members around their mean L2 "
              f"{100 * np.mean([_l2(m, m32) for m in ens['f32'][k]]):.2f}%; from-rest class: members around their "
              f"mean {100 * spread.mean():.2f}% (max {100 * spread.max():.2f}%), FP64 oracle run "
              f"{100 * d_ora:.2f}%, first member (exact rest) vs oracle {100 * _l2(rest[k][0], P_ora[k]):.2f}%; "
              f"class means differ by {100 * _l2(m32, mrest):.2f}%; one BF16 run vs FP32 mean "
              f"{100 * _l2(bf16[k][0], m32):.2f}%", flush=True)
        if not err < 0.01:
            failures.append(f"{k}: FP16 ensemble {100 * err:.2f}% off FP32")
        if not se_diff < 0.01:
            failures.append(f"{k}: standard error {100 * se_diff:.2f}% does not resolve 1 %")
        if not d_ora <= spread.max():
            failures.append(f"{k}: oracle run {100 * d_ora:.2f}% outside the FP32 spread {100 * spread.max():.2f}%")
    assert not failures, failures
