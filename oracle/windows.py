"""Windowed optimisation of a long snapshot sequence, plainly (test infrastructure only).

This file belongs to the oracle: only tests, the smoke check and the benchmark's CPU baseline
may use it.  Section 4 (the School case, 7375 snapshots) names windowed optimisation as the
approximate strategy for sequences too long for one supra-graph; the steps below are this
project's reading of it, stated once here and once in the library:

* Windows of W consecutive snapshots, each starting W - o snapshots after the previous one
  (o overlapping snapshots, 0 <= o < W); the last window ends at the last snapshot (it may be
  shorter).
* Each window is solved on its own supra-graph (the same coupling, the same parameters).  The
  first window starts from singletons; a later window starts from the previous windows'
  labels on its overlapping snapshots (equal labels stay together) and singletons elsewhere.
* Labels: a community of a window that holds overlapping copies takes the global label of its
  first such copy (smallest supra-node index); any other community takes a new label.  Copies
  of the overlapping snapshots keep the labels they already have; the window labels its other
  snapshots.  At the end labels are renumbered by first appearance in v = s*N + i.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

import oracle
from paper_2608_03695_amd import gen


def window_ranges(T, W, o):
    """[(s0, s1)] of the windows covering snapshots 0..T-1."""
    out, s0 = [], 0
    while True:
        s1 = min(T, s0 + W)
        out.append((s0, s1))
        if s1 == T:
            return out
        s0 = s1 - o


def sub_graph(g, s0, s1):
    a, b = int(g.offsets[s0]), int(g.offsets[s1])
    return gen.TemporalGraph(g.n_nodes, s1 - s0, (g.offsets[s0:s1 + 1] - a).astype(np.int64),
                             g.src[a:b], g.dst[a:b], None if g.weight is None else g.weight[a:b],
                             None, f"{g.name}[{s0}:{s1}]")


def first_appearance(labels):
    first = {}
    out = np.empty(len(labels), np.int32)
    for v, c in enumerate(labels):
        if c not in first:
            first[c] = len(first)
        out[v] = first[c]
    return out


def leiden_windowed(g, omega, W, o, gamma=Fraction(1), max_levels=32, max_iterations=2,
                    seed=0, null_model=0, gamma_slices=None, present_only=False):
    """(membership int32[T*N], number of windows)."""
    T, N = g.n_slices, g.n_nodes
    glob = np.full(T * N, -1, np.int64)
    fresh = 0
    ranges = window_ranges(T, W, o)
    for k, (s0, s1) in enumerate(ranges):
        sub = sub_graph(g, s0, s1)
        nw = (s1 - s0) * N
        ov = 0 if k == 0 else ranges[k - 1][1] - s0     # overlapping snapshots
        init = None
        if ov > 0:
            init = np.arange(nw, dtype=np.int32)
            seen = {}
            for v in range(ov * N):                      # overlap copies: their labels so far
                lab = int(glob[s0 * N + v])
                if lab not in seen:
                    seen[lab] = v
                init[v] = seen[lab]
        gs = None if gamma_slices is None else list(gamma_slices[s0:s1])
        og = oracle.OracleGraph(sub, omega, present_only=present_only)
        m, _, _ = og.leiden(gamma, max_levels=max_levels, max_iterations=max_iterations, seed=seed,
                            null_model=null_model, gamma_slices=gs, initial=init)
        label_of = {}
        for v in range(ov * N):                          # communities holding overlap copies
            c = int(m[v])
            if c not in label_of:
                label_of[c] = int(glob[s0 * N + v])
        for v in range(ov * N, nw):
            c = int(m[v])
            if c not in label_of:
                label_of[c] = fresh
                fresh += 1
            glob[s0 * N + v] = label_of[c]
    return first_appearance(glob), len(ranges)
