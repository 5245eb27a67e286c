"""GPU: the boundary's memory hook and error paths.

* mslm_set_allocator: with PyTorch's caching allocator installed, the graph's and the solve's
  device buffers come from it (torch's allocated-bytes counter rises while a graph lives and
  falls back when it is destroyed), and results still equal the oracle's.
* mslm_leiden refuses a solve whose int64 gain head-room fails (EOVERFLOW) and leaves the
  handle usable.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from paper_2608_03695_amd import gen

pytestmark = pytest.mark.gpu


def _mslm():
    from paper_2608_03695_amd import mslm
    return mslm


def test_torch_allocator_routes_device_memory():
    import torch
    mslm = _mslm()
    tg = gen.planted_partition(400, 4, 6, 0.08, 0.004, 0.1, seed=12, name="pp400")
    torch.cuda.synchronize()
    mslm.use_torch_allocator()
    try:
        before = torch.cuda.memory_allocated()
        g = mslm.Graph(tg, F(1, 2))
        with_graph = torch.cuda.memory_allocated()
        m, r = g.leiden(F(1), max_levels=32, max_iterations=2, seed=0)
        after_solve = torch.cuda.memory_allocated()
        g.close()
        torch.cuda.synchronize()
        after_close = torch.cuda.memory_allocated()
    finally:
        mslm.use_hip_allocator()
    assert with_graph > before                 # the supra-CSR lives in torch's pool
    assert after_solve > with_graph            # so do the solve's work buffers
    assert after_close == before               # and all of it goes back when the graph goes
    om, oc, _ = oracle.OracleGraph(tg, F(1, 2)).leiden(F(1), max_levels=32, max_iterations=2,
                                                       seed=0)
    assert np.array_equal(m, om)
    assert np.array_equal(r["q_components"], oc)
    # back on hipMalloc: torch's counter no longer moves
    base = torch.cuda.memory_allocated()
    g = mslm.Graph(tg, F(1, 2))
    assert torch.cuda.memory_allocated() == base
    g.close()


def test_leiden_refuses_gain_overflow_and_keeps_the_handle():
    mslm = _mslm()
    tg = gen.erdos_renyi(400, 1, 0.45, seed=5, name="dense400")   # 2m_0 > 2^16
    g = mslm.Graph(tg, 1)
    with pytest.raises(mslm.MslmError) as e:
        g.leiden(F(1 << 30))                   # p*b*S^2 >= 2^62
    assert e.value.status == mslm.MSLM_EOVERFLOW
    m, r = g.leiden(F(1))                      # the handle still works
    g.close()
    om, oc, _ = oracle.OracleGraph(tg, 1).leiden(F(1), max_levels=32, max_iterations=2, seed=0)
    assert np.array_equal(m, om)
    assert np.array_equal(r["q_components"], oc)
