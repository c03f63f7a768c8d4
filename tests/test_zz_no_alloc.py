"""stglbm_step_noalloc through the C ABI against stglbm_step (GPU).

The allocation-free variant runs the same kernels with its inlet planes staged
in the library's static device scratch; its lattice and statistics must equal
those of stglbm_step bit for bit.  Two calls in a row on different lattices,
the second smaller, check that nothing carries over in the shared scratch.
"""

import numpy as np
import pytest

from workloads import channel_config
from workloads.configs import small_channel

pytestmark = pytest.mark.gpu


def _pair(cfg):
    from paper_2205_02774_amd import channel_from_config
    print(f"[gpu] no-alloc case {cfg['name']}", flush=True)
    return channel_from_config(cfg, device="cuda:0"), channel_from_config(cfg, device="cuda:0")


def _compare(ref, na, chunks):
    ref.stats_reset()
    na.stats_reset()
    for n in chunks:
        ref.step(n)
        na.step_noalloc(n)
    f_ref, f_na = ref.get_f(), na.get_f()
    (s_ref, n_ref), (s_na, n_na) = ref.get_stats(), na.get_stats()
    diff = np.abs(f_na - f_ref).max()
    print(f"[gpu] no-alloc vs step: {sum(chunks)} steps, max |f diff| {diff:.3e}, "
          f"stats equal {np.array_equal(s_na, s_ref)}", flush=True)
    assert n_ref == n_na == sum(chunks)
    assert np.array_equal(f_na, f_ref)
    assert np.array_equal(s_na, s_ref)


def test_step_noalloc_matches_step_twice():
    # first call: the 64x32x32 channel, chunks that cross the 16-plane batches at odd offsets
    ref, na = _pair(channel_config(0))
    _compare(ref, na, (23, 17, 1))
    ref.close()
    na.close()
    # second call: a smaller lattice with fewer modes; the scratch holds the first call's planes
    ref, na = _pair(small_channel(40, 12, 8, n_modes=20, seed=2))
    _compare(ref, na, (5, 16))
    # the two entry points interleave on one handle without changing the result
    ref.step(9)
    na.step_noalloc(4)
    na.step(5)
    assert np.array_equal(na.get_f(), ref.get_f())
    ref.close()
    na.close()


@pytest.mark.parametrize("store", ["f16", "bf16"])
def test_step_noalloc_matches_step_16bit(store):
    # 16-bit statistics launches of 512-cell rows: stglbm_step makes the inlet
    # planes in the step kernel's trailing blocks from the 15th step on, the
    # allocation-free variant with the plane kernel into the scratch; the two
    # give the same planes, so f and the statistics agree bit for bit
    ref, na = _pair(small_channel(512, 8, 40, n_modes=30, seed=5, store=store))
    ref.profile(True)
    _compare(ref, na, (23, 17, 2))
    assert ref.profile_read()["tail_planes"] > 0
    ref.close()
    na.close()


def test_step_noalloc_rejects_planes_beyond_the_scratch():
    from paper_2205_02774_amd import Lattice, abi
    # one inlet plane of 2 x 700,000 nodes is 16.8 MB, above the 16 MiB scratch
    lat = Lattice(2, 2, 700_000, device="cuda:0", nu_lb=1e-2, max_modes=1, max_rans=2, sponge_cells=0)
    with pytest.raises(abi.StglbmError) as e:
        lat.step_noalloc(1)
    assert e.value.code == abi.E_INVAL and "scratch" in str(e.value)
    with pytest.raises(abi.StglbmError) as e:
        lat.step_noalloc(-1)
    assert e.value.code == abi.E_INVAL
    lat.close()
