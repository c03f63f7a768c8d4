"""Benchmark of the STG-LBM step on one MI355X.

One step = the STG inlet plane + the fused stream-collide pass over every
cell (inlet rebuild, outlet, sponge, Smagorinsky, regularized collision,
FP64 statistics), on the 512x128x256 Re_tau = 180 channel (600 modes, RANS
input on a 96-cell stretched grid).  Inputs are resident in HBM; W warm-up
steps run first, then exactly K steps are timed between two device
synchronizations.  The FP16- and BF16-store variants of the same workload
and the 1024x256x512 FP16 lattice are timed the same way; optional legs
compare long-run FP16/BF16 statistics with FP32 (--precision-steps) and run
the 64-job serving mix.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                       # MI355X HBM3E
# The step kernel's duration comes from HIP events on one timed launch in
# PROFILE_EVERY (every launch is the same work); recording events costs a few
# microseconds per launch, which would otherwise land in ms_per_step.
PROFILE_EVERY = 8
PROFILES = os.path.join(ROOT, "profiles")
# What makes the step kernels: the units that instantiate them, the headers
# they include and the build script (it sets the FP32 unit's scheduler).
KERNEL_SRCS = [os.path.join(ROOT, "paper_2205_02774_amd", "csrc", f)
               for f in ("lattice_step.h", "stg_block.h", "stglbm_internal.h", "lattice_kernels.hip",
                         "lattice_f32.hip")] + [os.path.join(ROOT, "paper_2205_02774_amd", "build.py")]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


_CODE_TOKENS = re.compile(r'"(?:\\.|[^"\\])*"|//[^\n]*|/\*.*?\*/', re.S)


def code_text(source):
    """C++ source without its comments, white space collapsed (string literals kept)."""
    text = _CODE_TOKENS.sub(lambda m: m.group(0) if m.group(0).startswith('"') else " ", source)
    return " ".join(text.split())


def kernel_hash():
    """Hash of the code of the stream-collide kernel (the unit that instantiates it and every
    header of the library that unit includes).

    Comments are dropped and white space collapsed first, so that a change of
    wording alone keeps the counter record of an unchanged kernel valid.
    """
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        h.update(code_text(open(path).read()).encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


def measured_traffic(workload, store):
    """HBM bytes per step-kernel launch from committed counter runs, if the kernel is unchanged."""
    path = os.path.join(PROFILES, f"traffic_{workload}_{store}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_sha256_16") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def run_variant(cfg, store, steps, warmup, stats=True, velocity_set=19, collision="regularized"):
    import torch
    from paper_2205_02774_amd import channel_from_config

    t0 = time.perf_counter()
    lat = channel_from_config(cfg, store=store, device="cuda:0", velocity_set=velocity_set, collision=collision)
    try:
        if stats:
            # warm up the launch that is timed (statistics on; the sums are cleared below), so
            # that the inlet planes are made as in a long statistics run when timing starts
            lat.stats_reset()
        lat.step(warmup)
        lat.sync()
    except Exception:
        lat.close()
        raise
    log(f"[bench] {cfg['name']} {store}: setup + {warmup} warm-up steps in {time.perf_counter() - t0:.1f} s")
    if stats:
        lat.stats_reset()
    lat.profile(True, every=PROFILE_EVERY)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat.step(steps)
    lat.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    prof = lat.profile_read()
    lat.profile(False)
    st, ns = lat.get_stats()
    assert ns == (steps if stats else 0)
    cells = cfg["cells"]
    bytes_per_cell = 2 * velocity_set * (4 if store == "f32" else 2)
    k_ms = prof["step_ms"] / prof["step_launches"]
    out = {
        "store": store,
        "ms_per_step": 1e3 * elapsed / steps,
        "mlups": cells * steps / elapsed / 1e6,
        "step_kernel_ms": k_ms,
        "stg_ms_per_plane": prof["stg_ms"] / max(1, prof["stg_planes"]),
        # 16-bit statistics steps make most inlet planes in trailing blocks of the
        # step kernel, whose time then includes them
        "planes_in_step_kernel": prof["tail_planes"],
        "bytes_per_launch": bytes_per_cell * cells,
        "achieved_gbs": bytes_per_cell * cells / (k_ms * 1e-3) / 1e9,
        "mean_u_lb": float(st[..., 0].sum() / (ns * cells)),
    }
    log(f"[bench] {store} D3Q{velocity_set} {collision}: {out['ms_per_step']:.4f} ms/step, {out['mlups']:.0f} MLUPS, step kernel "
        f"{k_ms:.4f} ms = {out['achieved_gbs']:.0f} GB/s, STG {out['stg_ms_per_plane'] * 1e3:.1f} us per plane"
        f" ({out['planes_in_step_kernel']} planes made in the step kernel)")
    lat.close()
    del lat
    torch.cuda.empty_cache()
    return out


def precision_study(cfg, steps, warmup):
    """Long runs of the FP16 and BF16 stores against the FP32 store: profile errors over 2 <= x/delta < 3.5."""
    import torch
    from paper_2205_02774_amd import channel_from_config
    from paper_2205_02774_amd.statistics import profiles, profile_errors
    d = cfg["ny"] // 2
    prof = {}
    for store in ("f32", "f16", "bf16"):
        t0 = time.perf_counter()
        lat = channel_from_config(cfg, store=store, device="cuda:0")
        for k in range(0, warmup, 5000):
            lat.step(min(5000, warmup - k))
            lat.sync()
        lat.stats_reset()
        for k in range(0, steps, 5000):
            lat.step(min(5000, steps - k))
            lat.sync()
        st, n = lat.get_stats()
        lat.close()
        del lat
        torch.cuda.empty_cache()
        prof[store] = profiles(st, n, cfg["nz"], 2 * d, int(3.5 * d))
        log(f"[bench] precision run {store}: {warmup} + {steps} steps in {time.perf_counter() - t0:.1f} s")
    out = {"warmup": warmup, "sampled_steps": steps, "x_range_delta": [2.0, 3.5], "reference": "f32"}
    for store in ("f16", "bf16"):
        out[store] = {k: round(v, 5) for k, v in profile_errors(prof[store], prof["f32"]).items()}
    log(f"[bench] precision: {out}")
    return out


def periodic_reference(nx, ny, nz, steps, warmup):
    """The force-driven periodic reference channel (no inlet plane), FP32, statistics every timed step."""
    import torch
    from paper_2205_02774_amd import periodic_channel_from_config
    from workloads import periodic_channel
    cfg = periodic_channel(nx, ny, nz, seed=5)
    lat = periodic_channel_from_config(cfg, device="cuda:0")
    lat.step(warmup)
    lat.sync()
    lat.stats_reset()
    lat.profile(True, every=PROFILE_EVERY)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat.step(steps)
    lat.sync()
    elapsed = time.perf_counter() - t1
    prof = lat.profile_read()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    cells = nx * ny * nz
    k_ms = prof["step_ms"] / prof["step_launches"]
    gbs = 152 * cells / (k_ms * 1e-3) / 1e9
    log(f"[bench] periodic {cfg['name']}: {1e3 * elapsed / steps:.4f} ms/step, step kernel {k_ms:.4f} ms = {gbs:.0f} GB/s")
    return {"workload": cfg["name"], "store": "f32", "force": "Guo, 1 m/s^2 along x", "steps": steps,
            "warmup": warmup, "value": round(cells * steps / elapsed / 1e6, 1), "unit": "MLUPS",
            "ms_per_step": round(1e3 * elapsed / steps, 5), "step_kernel_ms": round(k_ms, 5),
            "achieved_gbs": round(gbs, 1), "roofline_frac": round(gbs / HBM_PEAK_GBS, 4)}


def adaptation_study(cfg, steps, warmup):
    """Adaptation diagnostics of the FP32 STG channel: u_tau(x) / u_theory from the FP64
    statistics (eq. u_shear), the adaptation length (first x/delta from which it stays within
    +-3 % up to the sponge), and the integral time scale T_t (eq. time-integral) of u at
    y+ ~ 100 probes at x/delta = 0, 1, 2, 4, ... (z = NZ/2), in units of t* = delta / U_bulk."""
    import torch
    from paper_2205_02774_amd import channel_from_config
    from paper_2205_02774_amd.statistics import friction_velocity, adaptation_length, autocorrelation, \
        integral_time
    d = cfg["ny"] // 2
    yplus_per_cell = cfg["re_tau"] / d
    j100 = int(round(100.0 / yplus_per_cell - 0.5))
    stations = [s for s in (0, 1, 2, 4, 8, 16) if s * d < cfg["nx"] - cfg["sponge_cells"]]
    cells = [(s * d, j100, cfg["nz"] // 2) for s in stations]
    t0 = time.perf_counter()
    lat = channel_from_config(cfg, store="f32", device="cuda:0")
    for k in range(0, warmup, 5000):
        lat.step(min(5000, warmup - k))
        lat.sync()
    lat.stats_reset()
    series = lat.set_probes(cells, steps)
    for k in range(0, steps, 5000):
        lat.step(min(5000, steps - k))
        lat.sync()
    st, n = lat.get_stats()
    u = series.cpu().numpy().astype(np.float64)
    u_theory = lat.c_t / lat.c_x                       # u_tau = 1 m/s in lattice units
    ratio = friction_velocity(st, n, cfg["nz"], lat.nu_lb) / u_theory
    lat.close()
    del lat
    torch.cuda.empty_cache()
    x_d = np.arange(cfg["nx"]) / d
    t_star = d / cfg["u_b_lb"]                         # t* = delta / U_bulk, in steps
    out = {"warmup": warmup, "sampled_steps": steps, "u_theory_lb": u_theory,
           "adaptation_length_delta": adaptation_length(ratio, x_d, 0.03, (cfg["nx"] - cfg["sponge_cells"]) / d),
           "u_tau_ratio_at": {f"{s}": round(float(ratio[min(s * d, cfg['nx'] - 1)]), 4) for s in (1, 2, 3, 4, 6)
                              if s * d < cfg["nx"]},
           "probe_y_plus": round((j100 + 0.5) * yplus_per_cell, 1),
           "t_star_steps": t_star,
           "T_t_over_t_star": {f"{s}": round(float(integral_time(autocorrelation(u[:, k, 0]), 1.0)) / t_star, 4)
                               for k, s in enumerate(stations)},
           "record_t_star": round(steps / t_star, 3)}
    log(f"[bench] adaptation: {out} ({time.perf_counter() - t0:.1f} s)")
    return out


def large_lattice(name, steps, warmup):
    """The largest single-GPU lattice (FP16 store), timed like the main workload."""
    from workloads import channel_config
    cfg = channel_config(name)
    r = run_variant(cfg, cfg["store"], steps, warmup)
    return {"workload": cfg["name"], "store": cfg["store"], "cells": cfg["cells"], "steps": steps,
            "warmup": warmup, "value": round(r["mlups"], 1), "unit": "MLUPS",
            "ms_per_step": round(r["ms_per_step"], 5), "step_kernel_ms": round(r["step_kernel_ms"], 5),
            "stg_ms_per_plane": round(r["stg_ms_per_plane"], 5), "achieved_gbs": round(r["achieved_gbs"], 1),
            "roofline_frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
            "planes_in_step_kernel": r["planes_in_step_kernel"]}


def serving_mix(scale, budget_gib, max_active, chunk):
    """The 64-job serving mix with step budgets scaled by `scale` (Poisson arrivals, 2/s)."""
    from paper_2205_02774_amd.serve import Server, DeviceExecutor
    from workloads import serving_jobs, job_config
    jobs = []
    for spec in serving_jobs(64, seed=4):
        steps = max(1, int(round(spec["steps"] * scale)))
        jobs.append({"id": spec["id"], "arrival_s": spec["arrival_s"], "steps": steps, "cfg": job_config(spec)})
    srv = Server(int(budget_gib * 2 ** 30), max_active=max_active, chunk_steps=chunk,
                 executor=DeviceExecutor("cuda:0"))
    res, summ = srv.run(jobs)
    queue = [r.admitted_s - r.arrival_s for r in res]
    summ.update({"step_scale": scale, "budget_gib": round(budget_gib, 2), "max_active": max_active,
                 "chunk_steps": chunk, "peak_active": srv.peak_active, "peak_gib": round(srv.peak_bytes / 2 ** 30, 2),
                 "max_queue_s": float(max(queue)), "jobs_queued": int(sum(q > 0.05 for q in queue)),
                 "cell_updates": int(sum(r.cells * r.steps for r in res if r.status == "ok"))})
    log(f"[bench] serving: {summ}")
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in summ.items()}


def _cpu_info():
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


_ORACLE_RUN = """
import json, os, sys, time
sys.path.insert(0, {root!r})
from workloads import channel_config
from oracle import OracleChannel
cfg = channel_config({name!r})
if {nz} > 0:
    cfg['nz'] = {nz}
cfg['cells'] = cfg['nx'] * cfg['ny'] * cfg['nz']
ch = OracleChannel.from_config(cfg)
ch.stats_reset()
ch.step({untimed})
t0 = time.perf_counter()
ch.step({steps})
dt = time.perf_counter() - t0
print(json.dumps({{"cells": cfg['cells'], "steps": {steps}, "seconds": dt}}))
"""


def _oracle_procs(name, nz, steps, untimed, n_procs):
    """Run n_procs independent 1-thread oracle processes at once; their timing records."""
    env = dict(os.environ, OMP_NUM_THREADS="1", MKL_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1")
    code = _ORACLE_RUN.format(root=ROOT, name=name, nz=nz, steps=steps, untimed=untimed)
    procs = [subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                              text=True, env=env) for _ in range(n_procs)]
    recs = []
    for p in procs:
        out, err = p.communicate(timeout=900)
        if p.returncode != 0:
            log(err[-2000:])
            return None
        recs.append(json.loads(out.strip().splitlines()[-1]))
    return recs


def cpu_baseline(cfg, nz_sample, steps, all_core_max=16):
    """The FP64 oracle on the host: one thread on a spanwise slab of the workload (the value),
    the same slab in as many concurrent one-thread processes as the machine's CPU share allows
    (at most `all_core_max`), and the 64x32x32 channel's 200 steps in full."""
    model, nproc, usable = _cpu_info()
    one = _oracle_procs(cfg["name"], nz_sample, steps, 1, 1)
    if one is None:
        return None
    rec = one[0]
    n_all = max(1, min(usable, all_core_max))
    t0 = time.perf_counter()
    many = _oracle_procs(cfg["name"], nz_sample, steps, 1, n_all)
    wall_all = time.perf_counter() - t0
    small = _oracle_procs("channel-64x32x32", 0, 200, 0, 1)
    out = {
        "value": rec["cells"] * rec["steps"] / rec["seconds"] / 1e6,
        "unit": "MLUPS",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{cfg['nx']}x{cfg['ny']}x{nz_sample} spanwise slab of {cfg['name']} (same inlet), "
                  f"{steps} steps after 1 untimed, FP64 NumPy, 1 thread; {rec['seconds']:.1f} s",
        "cpu_model": model,
        "nproc": nproc,
        "usable_cpus": usable,
    }
    if many is not None:
        cells_steps = sum(r["cells"] * r["steps"] for r in many)
        slowest = max(r["seconds"] for r in many)
        out["all_core"] = {"processes": n_all, "aggregate_mlups": round(cells_steps / slowest / 1e6, 3),
                           "slowest_process_s": round(slowest, 2), "wall_s": round(wall_all, 2),
                           "note": f"{n_all} concurrent one-thread oracle processes on the same slab "
                                   f"(the box's CPU share for one GPU is {all_core_max} cores)"}
    if small is not None:
        r = small[0]
        out["channel_64x32x32_200_steps"] = {"seconds": round(r["seconds"], 2),
                                             "mlups": round(r["cells"] * r["steps"] / r["seconds"] / 1e6, 3),
                                             "threads": 1}
    log(f"[bench] cpu baseline: {out}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20000)
    ap.add_argument("--workload", default="channel-512x128x256")
    ap.add_argument("--variants", default="f16,bf16", help="extra store types timed on the same workload")
    ap.add_argument("--variant-warmup", type=int, default=2000)
    ap.add_argument("--variant-steps", type=int, default=500,
                    help="timed steps of each store and lattice variant (a window of a few steps is dominated by "
                         "the fixed latency at its start and end)")
    ap.add_argument("--lattice-variants", default="15:regularized,27:regularized,19:bgk",
                    help="velocity-set:operator pairs timed (FP32) on the same workload ('' = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="step budgets of the 64-job serving mix are scaled by this (1.0 = full mix; 0 = skip)")
    ap.add_argument("--serve-budget-gib", type=float, default=0.0,
                    help="memory budget of the first serving leg (0 = 90 %% of the device's free memory)")
    ap.add_argument("--serve-capped-gib", type=float, default=8.0,
                    help="memory budget of the second serving leg, where admission binds (0 = skip)")
    ap.add_argument("--serve-max-active", type=int, default=16)
    ap.add_argument("--serve-chunk", type=int, default=250)
    ap.add_argument("--large", default="channel-1024x256x512-f16", help="large lattice timed after the main one ('' = skip)")
    ap.add_argument("--large-steps", type=int, default=500)
    ap.add_argument("--large-warmup", type=int, default=1000)
    ap.add_argument("--periodic-steps", type=int, default=500,
                    help="timed steps of the periodic force-driven 512x128x256 reference channel (0 = skip)")
    ap.add_argument("--adaptation-steps", type=int, default=0,
                    help="if > 0: sampled steps of the u_tau(x) / probe autocorrelation study (after 20k warm-up)")
    ap.add_argument("--precision-steps", type=int, default=0,
                    help="if > 0: sampled steps of the FP16/BF16-vs-FP32 profile comparison (after 20k warm-up)")
    ap.add_argument("--cpu-nz", type=int, default=32)
    ap.add_argument("--cpu-steps", type=int, default=12)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the x-slab multi-GPU "
              f"decomposition is a design, not part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    from paper_2205_02774_amd import abi
    if not os.path.exists(abi.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    from workloads import channel_config

    cfg = channel_config(args.workload)
    main_run = run_variant(cfg, cfg["store"], args.steps, args.warmup)
    variants = {}
    for v in [s for s in args.variants.split(",") if s]:
        r = run_variant(cfg, v, args.variant_steps, args.variant_warmup)
        variants[v] = {
            "value": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 5),
            "step_kernel_ms": round(r["step_kernel_ms"], 5),
            "roofline_frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
            "planes_in_step_kernel": r["planes_in_step_kernel"],
            "speedup_vs_f32": round(r["mlups"] / main_run["mlups"], 3),
            "steps": args.variant_steps, "warmup": args.variant_warmup,
        }
    lattice_variants = {}
    for spec in [v for v in args.lattice_variants.split(",") if v]:
        q, op = spec.split(":")
        try:
            r = run_variant(cfg, "f32", args.variant_steps, args.variant_warmup, velocity_set=int(q), collision=op)
        except abi.StglbmError as e:            # e.g. plain BGK going unstable at tau0 - 1/2 = 3.4e-3
            log(f"[bench] D3Q{q} {op}: {e}")
            import torch
            torch.cuda.empty_cache()
            lattice_variants[f"D3Q{q}-{op}"] = {"status": "unstable", "message": str(e)}
            continue
        lattice_variants[f"D3Q{q}-{op}"] = {
            "value": round(r["mlups"], 1), "unit": "MLUPS", "ms_per_step": round(r["ms_per_step"], 5),
            "step_kernel_ms": round(r["step_kernel_ms"], 5), "algorithmic_bytes_per_cell": 2 * int(q) * 4,
            "achieved_gbs": round(r["achieved_gbs"], 1), "roofline_frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
            "steps": args.variant_steps, "warmup": args.variant_warmup}
    large = large_lattice(args.large, args.large_steps, args.large_warmup) if args.large else None
    periodic = periodic_reference(cfg["nx"], cfg["ny"], cfg["nz"], args.periodic_steps, 500) \
        if args.periodic_steps > 0 else None
    precision = precision_study(cfg, args.precision_steps, 20000) if args.precision_steps > 0 else None
    adaptation = adaptation_study(cfg, args.adaptation_steps, 20000) if args.adaptation_steps > 0 else None
    serving = None
    if args.serve_scale > 0:
        budget = args.serve_budget_gib or 0.9 * torch.cuda.mem_get_info(0)[0] / 2 ** 30
        serving = {"hbm_budget": serving_mix(args.serve_scale, budget, args.serve_max_active, args.serve_chunk)}
        if args.serve_capped_gib > 0:
            serving["capped_budget"] = serving_mix(args.serve_scale, args.serve_capped_gib, args.serve_max_active,
                                                   args.serve_chunk)
    traffic = measured_traffic(args.workload, cfg["store"])
    for v, rec in variants.items():
        rec["traffic"] = measured_traffic(args.workload, v)
    cpu = None if args.no_cpu_baseline else cpu_baseline(cfg, args.cpu_nz, args.cpu_steps)
    line = {
        "metric": "MLUPS + % HBM roofline (FP32 vs FP16-store STG-LBM); p50/p99 job latency",
        "value": round(main_run["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": cfg["name"], "lattice": [cfg["nx"], cfg["ny"], cfg["nz"]], "cells": cfg["cells"],
            "re_tau": cfg["re_tau"], "n_modes": cfg["n_modes"], "rans_grid": cfg["rans_grid"],
            "store": cfg["store"], "statistics": "FP64, every timed step", "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "step_kernel (fused stream-collide)",
            "achieved": round(main_run["achieved_gbs"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(main_run["achieved_gbs"] / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": main_run["bytes_per_launch"],
            "step_kernel_ms": round(main_run["step_kernel_ms"], 5),
            "stg_ms_per_plane": round(main_run["stg_ms_per_plane"], 5),
        },
        "variants": variants,
        "lattice_variants": lattice_variants,
        "large": large,
        "periodic": periodic,
        "precision": precision,
        "adaptation": adaptation,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
