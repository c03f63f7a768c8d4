"""bench.py command-line contract on the CPU: one GPU only, JSON helpers."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_kernel_hash_covers_the_stream_collide_sources():
    """The hash covers the units that instantiate the step kernels of the
    channel workloads, every library header they include, directly or not,
    and the build script that sets their compile flags."""
    import re
    sys.path.insert(0, ROOT)
    import bench
    csrc = os.path.join(ROOT, "paper_2205_02774_amd", "csrc")
    seen, todo = set(), ["lattice_kernels.hip", "lattice_f32.hip"]
    while todo:
        f = todo.pop()
        if f in seen or not os.path.exists(os.path.join(csrc, f)):
            continue
        seen.add(f)
        todo += re.findall(r'#include "([^"]+)"', open(os.path.join(csrc, f)).read())
    assert "stg_block.h" in seen and "lattice_step.h" in seen
    assert {os.path.basename(p) for p in bench.KERNEL_SRCS} == seen | {"build.py"}
    h = bench.kernel_hash()
    assert len(h) == 16 and h == bench.kernel_hash()


def test_kernel_hash_ignores_comments_but_not_code():
    sys.path.insert(0, ROOT)
    import bench
    norm = bench.code_text

    a = 'int f(int x) { // the input\n  return x + 1; /* one */ }\nconst char* s = "a//b";\n'
    b = 'int f(int x) {\n  // reworded comment\n  return x + 1;   }\nconst char* s = "a//b";\n'
    c = 'int f(int x) { return x + 2; }\nconst char* s = "a//b";\n'
    assert norm(a) == norm(b)
    assert norm(a) != norm(c)
    assert '"a//b"' in norm(a)
