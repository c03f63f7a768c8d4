"""Device copy bandwidth through libstglbm's plain copy kernel.

Gives the achievable HBM ceiling next to the 8 TB/s peak, and a kernel of
known traffic for calibrating the FETCH_SIZE / WRITE_SIZE counters (the copy
of B bytes reads B and writes B).

    python -m paper_2205_02774_amd.bandwidth [--gib 2] [--reps 20]
"""

import argparse
import ctypes
import json

import torch

from . import abi


def copy_bandwidth(nbytes, reps=20, device="cuda:0"):
    lib = abi.load()
    nbytes -= nbytes % 16
    src = torch.empty(nbytes, dtype=torch.uint8, device=device)
    dst = torch.empty(nbytes, dtype=torch.uint8, device=device)
    src.fill_(1)
    stream = torch.cuda.current_stream(device)
    for _ in range(3):
        abi.check(lib.stglbm_copy_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                        nbytes, ctypes.c_void_p(stream.cuda_stream)))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        abi.check(lib.stglbm_copy_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                        nbytes, ctypes.c_void_p(stream.cuda_stream)))
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    assert bool((dst[:1024] == 1).all())
    return {"bytes_copied": nbytes, "ms_per_copy": ms, "gbs_read_plus_write": 2 * nbytes / (ms * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gib", type=float, default=2.0)
    ap.add_argument("--reps", type=int, default=20)
    a = ap.parse_args()
    print(json.dumps(copy_bandwidth(int(a.gib * 2 ** 30), a.reps)), flush=True)


if __name__ == "__main__":
    main()
