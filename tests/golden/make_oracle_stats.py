"""Write the FP64 oracle's long-run channel statistics used by the precision study.

Runs the 64x32x32 STG channel (Re_tau = 180, 50 modes, seed 0) from rest with
the oracle only: `warmup` steps, then FP64 statistics sampled every step for
`steps` more.  Stores the per-(x, y) sums of u, v, w, uu, vv, ww, uv, uw, vw
and the sample count, plus the final distributions' mass.

    python tests/golden/make_oracle_stats.py [warmup] [steps]
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import OracleChannel  # noqa: E402
from workloads import channel_config  # noqa: E402


def main():
    warmup = int(sys.argv[1]) if len(sys.argv) > 1 else 10_000
    steps = int(sys.argv[2]) if len(sys.argv) > 2 else 40_000
    cfg = channel_config(0)
    ch = OracleChannel.from_config(cfg)
    t0 = time.time()
    for done in range(0, warmup, 1000):
        ch.step(min(1000, warmup - done))
        print(f"warm-up {ch.t} steps, {time.time() - t0:.0f} s", flush=True)
    ch.stats_reset()
    for done in range(0, steps, 1000):
        ch.step(min(1000, steps - done))
        print(f"sampled {ch.n_samples} steps, {time.time() - t0:.0f} s", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                       f"oracle_stats_64x32x32_w{warmup}_s{steps}.npz")
    np.savez_compressed(out, stats=ch.stats, n_samples=ch.n_samples, warmup=warmup, steps=steps,
                        mass=ch.f.sum(), guard_violations=ch.guard_violations)
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main()
