"""Device bandwidth through libstglbm's probe kernels.

Gives the achievable HBM ceilings next to the 8 TB/s peak: the plain copy
(also the kernel of known traffic for calibrating the FETCH_SIZE / WRITE_SIZE
counters: a copy of B bytes reads B and writes B), a copy with four 16-byte
loads in flight per lane and non-temporal stores, a read-only sweep and a
write-only fill.

    python -m paper_2205_02774_amd.bandwidth [--gib 2] [--reps 20] [--modes 0,1,2,3]
"""

import argparse
import ctypes
import json

import torch

from . import abi

MODES = {0: "copy", 1: "copy, 4 loads in flight, non-temporal stores", 2: "read only", 3: "write only"}


def probe_bandwidth(nbytes, mode=0, reps=20, device="cuda:0"):
    lib = abi.load()
    nbytes -= nbytes % 16
    src = torch.empty(nbytes, dtype=torch.uint8, device=device)
    dst = torch.empty(nbytes, dtype=torch.uint8, device=device)
    src.fill_(1)
    stream = torch.cuda.current_stream(device)

    def run():
        abi.check(lib.stglbm_bandwidth_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                             nbytes, mode, ctypes.c_void_p(stream.cuda_stream)))
    for _ in range(3):
        run()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        run()
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    moved = 2 * nbytes if mode in (0, 1) else nbytes
    if mode in (0, 1):
        assert bool((dst[:1024] == 1).all())
    return {"mode": mode, "kind": MODES[mode], "bytes": nbytes, "ms": ms, "gbs": moved / (ms * 1e-3) / 1e9}


def copy_bandwidth(nbytes, reps=20, device="cuda:0"):
    """The plain copy (mode 0): bytes copied, ms per copy, read + write GB/s."""
    r = probe_bandwidth(nbytes, 0, reps, device)
    return {"bytes_copied": r["bytes"], "ms_per_copy": r["ms"], "gbs_read_plus_write": r["gbs"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gib", type=float, default=2.0)
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--modes", default="0")
    a = ap.parse_args()
    for m in (int(v) for v in a.modes.split(",")):
        print(json.dumps(probe_bandwidth(int(a.gib * 2 ** 30), m, a.reps)), flush=True)


if __name__ == "__main__":
    main()
