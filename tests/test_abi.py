"""CPU checks of the C ABI: the library loads, exports what the header
declares, the ctypes mirrors match the C struct layout, and the host-only
logic (descriptor validation, footprint, unit derivation) behaves."""

import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stglbm.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2205_02774_amd import abi
    if not os.path.exists(abi.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return abi.load()


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(stglbm_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    from paper_2205_02774_amd import abi
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(abi.EXPORTED) == names


def test_struct_layout_matches_header():
    """Compile a host-only C probe of sizeof/offsetof and compare with ctypes."""
    from paper_2205_02774_amd import abi
    fields = {
        "stglbm_lattice_desc": [f[0] for f in abi.LatticeDesc._fields_],
        "stglbm_rans_inlet": [f[0] for f in abi.RansInlet._fields_],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "stglbm.h"', "int main(void){"]
    for st, fl in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fl:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout
    got = dict(l.rsplit(" ", 1) for l in out.strip().splitlines())
    for cls, st in ((abi.LatticeDesc, "stglbm_lattice_desc"), (abi.RansInlet, "stglbm_rans_inlet")):
        assert int(got[st]) == ctypes.sizeof(cls)
        for f, _ in cls._fields_:
            assert int(got[f"{st}.{f}"]) == getattr(cls, f).offset, f


def test_descriptor_validation_and_footprint(lib):
    from paper_2205_02774_amd import abi, make_desc, footprint
    d = make_desc(512, 128, 256, nu_lb=1.1458e-3, max_modes=600, max_rans=96)
    fp = footprint(d)
    g32 = 2 * 19 * 512 * 128 * 256 * 4
    bins = 9 * 512 * 128 * 8                          # the FP64 statistics totals (twice a window slot's bytes)
    ring = 16 * 128 * 256 * 3 * 4                     # inlet planes of 16 steps, FP32
    ptab = 16 * 600 * 128 * 8                         # row phasors of 16 steps, [mode][row] FP32 pairs
    assert fp >= g32 + ring + ptab
    # two distribution buffers + FP64 statistics slots (at most 16) + the plane ring and row-phasor
    # table + the small inlet tables
    assert fp - g32 <= 16 * bins + ring + ptab + 4 * 2 ** 20
    d16 = make_desc(512, 128, 256, nu_lb=1.1458e-3, store="f16", max_modes=600, max_rans=96)
    assert 0 <= footprint(d16) - g32 // 2 <= 16 * bins + ring + ptab + 4 * 2 ** 20
    bad = make_desc(1, 128, 256, nu_lb=1e-3, max_modes=10, max_rans=10)
    with pytest.raises(abi.StglbmError) as e:
        footprint(bad)
    assert e.value.code == abi.E_INVAL
    with pytest.raises(abi.StglbmError):
        footprint(make_desc(64, 32, 32, nu_lb=-1.0, max_modes=10, max_rans=10))
    with pytest.raises(abi.StglbmError):
        footprint(make_desc(64, 32, 32, nu_lb=1e-3, max_modes=0, max_rans=10))
    # periodic lattices need no inlet tables
    dp = make_desc(64, 32, 32, nu_lb=1e-3, periodic_x=True)
    assert footprint(dp) < footprint(make_desc(64, 32, 32, nu_lb=1e-3, max_modes=50, max_rans=32))
    # init without a workspace fails on the host before touching a device
    h = ctypes.c_void_p()
    rc = lib.stglbm_init_lattice(ctypes.byref(d), None, 0, None, ctypes.byref(h))
    assert rc == abi.E_INVAL and not h.value


def test_derive_units_matches_oracle(lib):
    from paper_2205_02774_amd import derive_units
    from oracle import units
    got = derive_units(1.0, 128, 0.05, 15.37, 1 / 180)
    c_x, c_t, nu_lb, _ = units.channel_units(1.0, 128, 0.05, 15.37, 1 / 180)
    assert got == pytest.approx((c_x, c_t, nu_lb), rel=1e-15)


@pytest.mark.parametrize("shape,store,qset,slots", [
    ((512, 128, 256), "f32", 19, 2),     # two z waves per block, 2 x 128 x 16 waves = 4096
    ((512, 128, 256), "f32", 15, 2),
    ((512, 128, 256), "f32", 27, 4),     # one z wave: 4 slots
    ((512, 128, 256), "f16", 19, 12),    # 16-bit, 8-wave blocks: two rounds of 768 resident blocks, 6 slots each
    ((512, 128, 256), "bf16", 19, 12),
    ((512, 256, 256), "f16", 19, 6),     # 256 blocks per slot: 3 slots per round
    ((512, 64, 96), "f16", 19, 24),      # 64 blocks per slot: 12 per round, 24 chunks of 5, 4 or 3 and 2 rows
    ((512, 64, 64), "f16", 19, 32),      # too few rows for 24 chunks: the uniform rule's 32, cut unequal
    ((1024, 256, 512), "f16", 19, 4),    # 512 blocks per slot (768 is no multiple): slots for 16384 waves
    ((448, 128, 256), "f16", 19, 19),    # 7-wave rows: uniform chunks (16384 waves: 19 slots of 14 rows)
    ((64, 32, 32), "f32", 19, 16),       # capped at NZ / 2 for two z waves
    ((64, 32, 32), "f16", 19, 32),       # capped at NZ
])
def test_statistics_slots_of_the_launch_shape(lib, shape, store, qset, slots):
    """The statistics slots the layout reserves follow the launch-shape rule:
    periodic lattices hold the two distribution buffers, the statistics and
    under 1 MiB of small tables, so the slot count is read off the footprint.
    Every store keeps one set of FP64 totals and FP32 window sums per slot."""
    from paper_2205_02774_amd import make_desc, footprint
    nx, ny, nz = shape
    fp = footprint(make_desc(nx, ny, nz, nu_lb=1e-3, store=store, periodic_x=True, velocity_set=qset))
    g = 2 * qset * nx * ny * nz * (4 if store == "f32" else 2)
    bins = 9 * nx * ny
    need = bins * 8 + slots * bins * 4
    assert need <= fp - g < need + 2 ** 20


def test_velocity_set_and_collision_validation(lib):
    from paper_2205_02774_amd import abi, make_desc, footprint
    base = footprint(make_desc(64, 32, 32, nu_lb=1e-3, periodic_x=True))
    f27 = footprint(make_desc(64, 32, 32, nu_lb=1e-3, periodic_x=True, velocity_set=27))
    f15 = footprint(make_desc(64, 32, 32, nu_lb=1e-3, periodic_x=True, velocity_set=15))
    g19 = 2 * 19 * 64 * 32 * 32 * 4
    # FP32 statistics launches of D3Q15 / D3Q19 run two z waves per block, so
    # this lattice has 16 slots of 9 x 64 x 32 FP32 window sums where D3Q27
    # (one z wave per block) has 32.
    slot = 9 * 64 * 32 * 4
    assert f27 - base == pytest.approx(g19 * 8 / 19 + 16 * slot, abs=1024)
    assert base - f15 == pytest.approx(g19 * 4 / 19, abs=1024)
    assert footprint(make_desc(64, 32, 32, nu_lb=1e-3, periodic_x=True, velocity_set=0)) == base
    for bad in (dict(velocity_set=21), dict(collision=2), dict(collision="bgk", velocity_set=13)):
        with pytest.raises(abi.StglbmError) as e:
            footprint(make_desc(64, 32, 32, nu_lb=1e-3, periodic_x=True, **bad))
        assert e.value.code == abi.E_INVAL
