"""GPU: the allocation-free entry point mslm_leiden_static against mslm_leiden.

Two calls in a row on one device, the second on a smaller graph (the static scratch keeps the
first call's contents), each compared with the existing entry point's result: memberships and
Q components identical, statistics equal.  A counting allocator installed through
mslm_set_allocator shows that the allocation-free call requests no device memory at all.
"""
import ctypes as C
from fractions import Fraction as F

import numpy as np
import pytest

from paper_2608_03695_amd import gen

pytestmark = pytest.mark.gpu

STAT_KEYS = ["sweeps", "moves", "sweep_cap_hits", "refine_rounds", "merges", "splits",
             "levels_run", "iterations_run", "n_communities", "exact_fallbacks"]


def test_static_entry_equals_plain_on_two_calls_in_a_row():
    import torch
    from paper_2608_03695_amd import mslm
    lib = mslm.load()
    calls = {"alloc": 0}

    @mslm._ALLOC_T
    def counting_alloc(nbytes, ctx):
        calls["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(int(nbytes))

    @mslm._RELEASE_T
    def counting_release(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    mslm._allocators.append((counting_alloc, counting_release))
    cases = [(gen.config1(), F(1), F(1)),                                    # 4000 supra-nodes
             (gen.planted_partition(300, 3, 5, 0.1, 0.01, 0.1, seed=31), F(2), F(1, 10))]
    for tg, gamma, omega in cases:
        g = mslm.Graph(tg, omega)
        want_m, want_r = g.leiden(gamma, max_levels=32, max_iterations=2, seed=0)
        assert lib.mslm_set_allocator(counting_alloc, counting_release, None) == 0
        try:
            before = calls["alloc"]
            got_m, got_r = g.leiden(gamma, max_levels=32, max_iterations=2, seed=0, no_alloc=True)
            assert calls["alloc"] == before, "the allocation-free call allocated device memory"
        finally:
            mslm.use_hip_allocator()
        assert np.array_equal(got_m, want_m), tg.name
        assert np.array_equal(got_r["q_components"], want_r["q_components"]), tg.name
        for k in STAT_KEYS:
            assert got_r[k] == want_r[k], (tg.name, k)
        g.close()


def test_static_entry_device_output_and_limits():
    import torch
    from paper_2608_03695_amd import mslm
    tg = gen.planted_partition(300, 3, 5, 0.1, 0.01, 0.1, seed=31)
    g = mslm.Graph(tg, 1)
    want_m, want_r = g.leiden(1)
    out = torch.empty(tg.n_supra, dtype=torch.int32, device="cuda")
    _, got_r = g.leiden(1, out=out, no_alloc=True)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), want_m)
    assert np.array_equal(got_r["q_components"], want_r["q_components"])
    with pytest.raises(mslm.MslmError) as e:        # it records no HIP events
        g.leiden(1, profile=True, no_alloc=True)
    assert e.value.status == mslm.MSLM_EINVAL
    g.close()
