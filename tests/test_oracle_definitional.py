"""Pins of the definitional tier of the oracle (Eq. 3 and Eq. 6 in exact rationals).

Each check ties the oracle to something other than itself: a hand-derived example, a
closed form, a textbook special case (Eq. 5 at T = 1), a decomposition that must hold
for omega = 0, or brute force.  A dropped term, a wrong sign or a transposed index in
any of the three Q evaluators fails at least one of them.
"""
import json
import os
import random
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import definitional as D
from paper_2608_03695_amd import gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _h2():
    return gen.from_edge_lists(2, [[(0, 1)], [(0, 1)]])


def _random_graph(rng, n, t, p=0.6, wmax=3):
    slices = []
    for _ in range(t):
        edges = []
        for i in range(n):
            for j in range(i + 1, n):
                if rng.random() < p:
                    a, b = (i, j) if rng.random() < 0.5 else (j, i)
                    edges.append((a, b, rng.randint(1, wmax)))
        slices.append(edges)
    return gen.from_edge_lists(n, slices, weighted=True)


def _random_partition(rng, size):
    k = rng.randint(1, size)
    return [rng.randrange(k) for _ in range(size)]


def test_h2_hand_example_values():
    spec = json.load(open(os.path.join(GOLDEN, "h2_hand_example.json")))
    g = _h2()
    gamma, omega = F(spec["gamma"]), F(spec["omega"])
    assert D.two_mu(g, omega) == 8
    for name, case in spec["partitions"].items():
        want = F(case["Q"])
        m = case["membership"]
        assert D.q_quadruple_sum(g, gamma, omega, m) == want, name
        assert D.q_trace_form(g, gamma, omega, m) == want, name
        assert D.q_component_form(g, gamma, omega, m) == want, name


def test_h2_brute_force_optimum_unique():
    spec = json.load(open(os.path.join(GOLDEN, "h2_hand_example.json")))
    best, arg = D.brute_force_max(_h2(), F(1), F(1))
    assert best == F(spec["optimum"]["Q"])
    assert len(arg) == 1 and len(set(arg[0])) == 1


def test_supra_adjacency_block_structure():
    rng = random.Random(3)
    g = _random_graph(rng, 4, 3)
    om = F(3, 7)
    A = D.supra_adjacency(g, om)
    mats = D.slice_matrices(g)
    n, t = 4, 3
    for s in range(t):
        for r in range(t):
            for i in range(n):
                for j in range(n):
                    v = A[s * n + i][r * n + j]
                    if s == r:
                        assert v == mats[s][i][j]
                    elif abs(s - r) == 1 and i == j:
                        assert v == om
                    else:
                        assert v == 0
    assert all(A[u][v] == A[v][u] for u in range(n * t) for v in range(n * t))
    assert sum(sum(row) for row in A) == D.two_mu(g, om)


@pytest.mark.parametrize("seed", range(12))
def test_three_forms_of_eq6_agree(seed):
    rng = random.Random(seed)
    n, t = rng.randint(2, 4), rng.randint(1, 3)
    g = _random_graph(rng, n, t, p=rng.choice([0.3, 0.6, 0.9]))
    gamma = F(rng.randint(0, 5), rng.randint(1, 3))
    omega = F(rng.randint(0, 5), rng.randint(1, 4))
    for _ in range(3):
        m = _random_partition(rng, n * t)
        q1 = D.q_quadruple_sum(g, gamma, omega, m)
        assert q1 == D.q_trace_form(g, gamma, omega, m)
        assert q1 == D.q_component_form(g, gamma, omega, m)


@pytest.mark.parametrize("seed", range(6))
def test_closed_forms(seed):
    rng = random.Random(100 + seed)
    n, t = rng.randint(2, 4), rng.randint(1, 3)
    g = _random_graph(rng, n, t)
    gamma = F(rng.randint(1, 4), rng.randint(1, 3))
    omega = F(rng.randint(0, 4), rng.randint(1, 3))
    size = n * t
    assert D.q_quadruple_sum(g, gamma, omega, list(range(size))) == D.q_all_singletons(g, gamma, omega)
    assert D.q_quadruple_sum(g, gamma, omega, [0] * size) == D.q_one_community(g, gamma, omega)
    # gamma = 1: the one-community value is the coupling share of the total weight
    tm = D.two_mu(g, omega)
    if tm:
        assert D.q_one_community(g, 1, omega) == 2 * omega * n * (t - 1) / tm


@pytest.mark.parametrize("seed", range(6))
def test_single_snapshot_is_newman_modularity(seed):
    rng = random.Random(200 + seed)
    n = rng.randint(3, 6)
    g = _random_graph(rng, n, 1)
    gamma = F(rng.randint(1, 3), rng.randint(1, 2))
    for _ in range(3):
        m = _random_partition(rng, n)
        assert D.q_quadruple_sum(g, gamma, F(5), m) == D.q_newman_static(g, gamma, m)


@pytest.mark.parametrize("seed", range(4))
def test_zero_coupling_decomposes_by_slice(seed):
    rng = random.Random(300 + seed)
    n, t = 4, 3
    g = _random_graph(rng, n, t)
    gamma = F(rng.randint(1, 3), 2)
    m = _random_partition(rng, n * t)
    tm = D.two_mu(g, 0)
    want = F(0)
    for s in range(t):
        u, x, w = g.slice_edges(s)
        gs = gen.from_edge_lists(n, [[(int(u[e]), int(x[e]), int(w[e])) for e in range(u.size)]],
                                 weighted=True)
        two_m_s = 2 * int(w.sum())
        want += F(two_m_s) / tm * D.q_newman_static(gs, gamma, m[s * n:(s + 1) * n])
    assert D.q_quadruple_sum(g, gamma, 0, m) == want


def test_brute_force_on_two_triangles():
    # two triangles joined by one edge, single snapshot: the optimum is the two triangles
    edges = [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (2, 3)]
    g = gen.from_edge_lists(6, [edges])
    best, arg = D.brute_force_max(g, F(1), F(1))
    assert best == F(5, 14)
    assert arg == [[0, 0, 0, 1, 1, 1]]


def test_relabelling_does_not_change_q():
    rng = random.Random(9)
    g = _random_graph(rng, 3, 2)
    m = [0, 1, 1, 2, 0, 2]
    perm = {0: 7, 1: 3, 2: 11}
    assert D.q_quadruple_sum(g, 1, 1, m) == D.q_quadruple_sum(g, 1, 1, [perm[x] for x in m])
