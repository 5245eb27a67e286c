"""Pins of the oracle's windowed optimisation (oracle/windows.py; Section 4 names windowing for
sequences too long for one supra-graph):

* one window covering the sequence is the plain solve;
* disjoint windows (no overlap) are independent plain solves of the window graphs;
* with overlap, copies that a window puts in one community share one label, and a window's
  start partition holds the earlier labels of its overlapping snapshots;
* the window ranges cover every snapshot and step by W - o.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from oracle import windows as WN
from paper_2608_03695_amd import gen


def _same_partition(a, b):
    return np.array_equal(WN.first_appearance(list(a)), WN.first_appearance(list(b)))


@pytest.mark.parametrize("T,W,o", [(10, 4, 0), (10, 4, 1), (10, 4, 3), (7, 7, 2), (65, 64, 5),
                                   (1, 3, 2)])
def test_window_ranges_cover_the_sequence(T, W, o):
    r = WN.window_ranges(T, W, o)
    assert r[0][0] == 0 and r[-1][1] == T
    for (a0, a1), (b0, b1) in zip(r, r[1:]):
        assert b0 == a1 - o and a1 - a0 == W
    assert all(1 <= s1 - s0 <= W for s0, s1 in r)


def test_one_window_is_the_plain_solve():
    g = gen.planted_partition(120, 6, 4, 0.1, 0.01, 0.1, seed=2)
    m, nw = WN.leiden_windowed(g, F(1), 8, 2)
    pm, _, _ = oracle.OracleGraph(g, F(1)).leiden(F(1))
    assert nw == 1 and np.array_equal(m, pm)


@pytest.mark.parametrize("nm", [0, 2])
def test_disjoint_windows_are_independent_solves(nm):
    g = gen.planted_partition(80, 9, 4, 0.12, 0.01, 0.1, seed=3)
    gamma = F(1) if nm == 0 else F(1, 20)
    m, nw = WN.leiden_windowed(g, F(1, 2), 3, 0, gamma=gamma, null_model=nm)
    assert nw == 3
    N = g.n_nodes
    labels_seen = set()
    for s0, s1 in WN.window_ranges(9, 3, 0):
        pm, _, _ = oracle.OracleGraph(WN.sub_graph(g, s0, s1), F(1, 2)).leiden(gamma, null_model=nm)
        part = m[s0 * N:s1 * N]
        assert _same_partition(part, pm)
        assert not (set(part.tolist()) & labels_seen)   # windows share no community
        labels_seen |= set(part.tolist())


@pytest.mark.parametrize("o", [1, 3])
def test_overlapping_windows_keep_communities_together(o):
    g = gen.dcsbm(100, 12, 8, 5, 0.2, 2.5, 0.05, seed=4)
    m, nw = WN.leiden_windowed(g, F(1), 5, o)
    N = g.n_nodes
    ranges = WN.window_ranges(12, 5, o)
    assert nw == len(ranges)
    # re-run each window from the labels it started from: copies it puts in one community
    # (outside its overlap) carry one label
    for k, (s0, s1) in enumerate(ranges):
        ov = 0 if k == 0 else ranges[k - 1][1] - s0
        init = None
        if ov:
            init = np.arange((s1 - s0) * N, dtype=np.int32)
            seen = {}
            for v in range(ov * N):
                lab = int(m[s0 * N + v])
                init[v] = seen.setdefault(lab, v)
        wm, _, _ = oracle.OracleGraph(WN.sub_graph(g, s0, s1), F(1)).leiden(F(1), initial=init)
        # final labels refine nothing: one window community -> one label on its own snapshots
        lab_of = {}
        for v in range(ov * N, (s1 - s0) * N):
            c = int(wm[v])
            assert lab_of.setdefault(c, int(m[s0 * N + v])) == int(m[s0 * N + v])
