"""GPU: execution choices (mslm_tuning) never change a result, and the autotuner keeps that.

Every tuning below is applied to the same solves, whose memberships, Q components and schedule
statistics must equal the default tuning's bit for bit; those are also compared with the
oracle.  The autotuner returns a valid tuning, installs it on the handle, and the tuned handle
reproduces the result.  Out-of-range values are refused and leave the handle's tuning alone.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from paper_2608_03695_amd import gen

pytestmark = pytest.mark.gpu

STAT_KEYS = ["sweeps", "moves", "sweep_cap_hits", "refine_rounds", "merges", "splits",
             "levels_run", "iterations_run", "n_communities"]

TUNINGS = [
    dict(graphs=1),
    dict(graphs=1, latency_units=64),
    dict(latency_units=4096, lat_parts_max=1),
    dict(latency_units=256, lat_parts_max=16),
    dict(split_group_units=0),
    dict(split_group_units=1 << 30),
    dict(copy_moves=1),
    dict(copy_moves=1 << 30),
    dict(graphs=1, split_group_units=0, copy_moves=1, latency_units=65536, lat_parts_max=4),
]

GRAPHS = [
    ("dcsbm_levels", lambda: gen.dcsbm(20000, 4, 10, 40, 0.3, 2.3, 0.03, seed=10), F(1), F(1, 2)),
    ("dcsbm_weighted", lambda: gen.dcsbm(3000, 6, 8, 20, 0.3, 2.5, 0.05, weights_max=8, seed=8),
     F(1), F(1)),
    ("planted", lambda: gen.planted_partition(600, 5, 8, 0.08, 0.004, 0.1, seed=3), F(2), F(10)),
]


def _mslm():
    from paper_2608_03695_amd import mslm
    return mslm


def _same(a, b, case):
    assert np.array_equal(a[0], b[0]), case
    assert np.array_equal(a[1]["q_components"], b[1]["q_components"]), case
    for k in STAT_KEYS:
        assert a[1][k] == b[1][k], f"{case}: {k}"


@pytest.mark.parametrize("name,make,gamma,omega", GRAPHS, ids=[x[0] for x in GRAPHS])
def test_tunings_never_change_results(name, make, gamma, omega):
    mslm = _mslm()
    tg = make()
    g = mslm.Graph(tg, omega)
    base = g.leiden(gamma)
    default = g.tuning()
    om, oc, _ = oracle.OracleGraph(tg, omega).leiden(gamma)
    assert np.array_equal(base[0], om)
    assert np.array_equal(base[1]["q_components"], oc)
    for tu in TUNINGS:
        g.set_tuning(**default)
        g.set_tuning(**tu)
        for rep in range(2):   # graph replays after eager sweeps, twice over
            _same(g.leiden(gamma), base, f"{name} {tu} run {rep}")
    g.set_tuning(**default)
    glob = g.leiden(gamma, null_model=1)
    g.set_tuning(graphs=1, split_group_units=0, copy_moves=1)
    _same(g.leiden(gamma, null_model=1), glob, f"{name} global")
    g.close()


def test_autotune_installs_a_tuning_with_the_same_result():
    mslm = _mslm()
    tg = gen.dcsbm(20000, 4, 10, 40, 0.3, 2.3, 0.03, seed=10)
    g = mslm.Graph(tg, F(1, 2))
    base = g.leiden(F(1))
    tuned, ms0, ms1 = g.autotune(F(1), rounds=1)
    assert ms0 > 0 and 0 < ms1 <= ms0 * 1.5
    assert g.tuning() == tuned
    assert tuned["graphs"] in (0, 1) and 1 <= tuned["lat_parts_max"] <= 16
    _same(g.leiden(F(1)), base, f"tuned {tuned}")
    g.close()


def test_set_tuning_refuses_out_of_range_values():
    mslm = _mslm()
    g = mslm.Graph(gen.erdos_renyi(100, 2, 0.05, seed=1), 1)
    before = g.tuning()
    for bad in (dict(graphs=2), dict(latency_units=32), dict(latency_units=1 << 20),
                dict(copy_moves=0), dict(lat_parts_max=17), dict(batch_units=0),
                dict(split_group_units=-1)):
        with pytest.raises(mslm.MslmError) as e:
            g.set_tuning(**bad)
        assert e.value.status == mslm.MSLM_EINVAL, bad
        assert g.tuning() == before
    g.close()


def test_batch_with_small_union_chunks_equals_plain_calls():
    """batch_units = 1 (2^20 supra-nodes per union) cuts a batch into several unions; every
    solve still equals its plain call."""
    mslm = _mslm()
    tgs = [gen.dcsbm(300000, 2, 8, 30, 0.3, 2.5, 0.05, seed=41),
           gen.dcsbm(250000, 3, 8, 30, 0.3, 2.5, 0.05, seed=42),
           gen.planted_partition(300, 3, 5, 0.1, 0.01, 0.1, seed=31)]
    handles = [mslm.Graph(tg, 1) for tg in tgs]
    handles[0].set_tuning(batch_units=1, graphs=1)
    solves = [(0, F(1), F(1), 32, 2, 0), (1, F(1), F(1, 10), 32, 2, 0), (2, F(2), F(1), 32, 2, 0),
              (0, F(1, 2), F(10), 32, 2, 0)]
    got = mslm.batch_leiden(handles, solves)
    for (gi, gamma, omega, lv, it, seed), out in zip(solves, got):
        _same(out, handles[gi].leiden(gamma, omega, max_levels=lv, max_iterations=it, seed=seed),
              f"graph {gi} gamma={gamma} omega={omega}")
    for h in handles:
        h.close()
