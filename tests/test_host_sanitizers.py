"""Host code of libstglbm under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds the library's host code (api.hip) with the sanitizers on the host side
only, the kernel units unchanged, links tests/host_abi_check.c against them,
and runs it: descriptor validation, footprint (the launch-shape,
statistics-slot and z-chunk rules over 11,340 lattice descriptors), unit
derivation, status strings and the argument checks that return before any
HIP call.  The
two-buffer pull scheme of the kernels is race-free by construction (each
launch reads one buffer and writes the other); determinism is checked on the
GPU by the parity tests.
"""

import concurrent.futures
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2205_02774_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(not os.path.exists(HIPCC) or shutil.which("gcc") is None, reason="needs hipcc and gcc")
def test_host_abi_under_asan_ubsan(tmp_path):
    flags = ["--offload-arch=gfx950", "-O1", "-fPIC", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    units = [("lattice_kernels.hip", []), ("lattice_variants.hip", []), ("lattice_f32.hip", []),
             ("inlet_kernels.hip", []), ("api.hip", SAN)]
    cmds = [[HIPCC, *flags, *extra, "-c", os.path.join(CSRC, src), "-o", str(tmp_path / (src + ".o"))]
            for src, extra in units]
    with concurrent.futures.ThreadPoolExecutor(len(cmds)) as pool:
        for res in pool.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds):
            assert res.returncode == 0, res.stderr[-3000:]
    check_o = tmp_path / "check.o"
    subprocess.run(["gcc", "-std=c99", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-I", os.path.join(ROOT, "include"), "-c", os.path.join(ROOT, "tests", "host_abi_check.c"),
                    "-o", str(check_o)], check=True)
    exe = tmp_path / "check"
    res = subprocess.run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                          "-fsanitize=undefined", str(check_o), *[str(tmp_path / (s + ".o")) for s, _ in units],
                          "-o", str(exe), "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"],
                         capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0 and run.stdout.strip() == "ok", run.stdout + run.stderr[-3000:]
