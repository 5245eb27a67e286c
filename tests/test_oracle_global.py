"""Pins of the global null-model mode of the oracle (the objective the paper's GPU path
optimised on the supra-graph as a stand-in for Eq. 6): Eq. 5 with d_out = d_in = kappa over
every supra-node of Eq. 3.

* The definitional tier: the literal pair sum equals the trace form with the global
  modularity matrix; closed forms (all singletons, one community); for one snapshot the global
  and the multislice objective are both textbook Newman modularity; a hand value.
* The C oracle's global Q components reproduce the definitional Q on random partitions.
* The C oracle's global schedule equals the literal tier (every decision on the exact change
  of Q_G) level by level, with its refinement bookkeeping, on random tiny graphs.
* Named cases reach the brute-force optimum of Q_G; random tiny graphs stay below it, with
  connected communities.
"""
import random
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from oracle import definitional as D
from oracle import schedule as S
from paper_2608_03695_amd import gen

import test_oracle_literal as L


def _rand(seed, max_nodes=4):
    rng = random.Random(seed)
    n, t = rng.randint(2, max_nodes), rng.randint(1, 3)
    g = gen.erdos_renyi(n, t, rng.uniform(0.3, 0.8), seed=rng.randrange(1 << 30),
                        weights_max=rng.choice([1, 3]))
    return rng, g, F(rng.randint(0, 3), rng.randint(1, 3)), F(rng.randint(1, 4), rng.randint(1, 3))


@pytest.mark.parametrize("seed", range(8))
def test_global_pair_sum_equals_trace_form_and_closed_forms(seed):
    rng, g, omega, gamma = _rand(seed)
    size = g.n_supra
    for _ in range(3):
        m = [rng.randrange(size) for _ in range(size)]
        assert D.q_global_pair_sum(g, gamma, omega, m) == D.q_global_trace_form(g, gamma, omega, m)
    assert D.q_global_pair_sum(g, gamma, omega, list(range(size))) == \
        D.q_global_all_singletons(g, gamma, omega)
    assert D.q_global_pair_sum(g, gamma, omega, [0] * size) == \
        D.q_global_one_community(g, gamma, omega)


@pytest.mark.parametrize("seed", range(4))
def test_one_snapshot_global_is_newman_modularity(seed):
    rng = random.Random(100 + seed)
    g = gen.erdos_renyi(5, 1, 0.6, seed=seed, weights_max=3)
    gamma = F(rng.randint(1, 3), 2)
    for _ in range(4):
        m = np.array([rng.randrange(3) for _ in range(5)])
        assert D.q_global_pair_sum(g, gamma, 1, m) == D.q_newman_static(g, gamma, m) == \
            D.q_quadruple_sum(g, gamma, 1, m)


def test_global_hand_value():
    """Hand example: N=2, T=2, edge 0-1 of weight 1 in both slices, omega = gamma = 1, so
    kappa = 2 for every supra-node and 2mu = 8.  By node ({0,2}, {1,3}): the weight inside is
    the 4 directed coupling entries, the null term (16 + 16) / 8 = 4, Q = 0.  By slice
    ({0,1}, {2,3}): 4 directed intra entries inside, null 4, Q = 0.  One community:
    1 - gamma = 0.  Singletons: -gamma * 4 * 2^2 / 8^2 = -1/4."""
    g = gen.from_edge_lists(2, [[(0, 1)], [(0, 1)]])
    assert D.q_global_pair_sum(g, 1, 1, [0, 1, 0, 1]) == 0
    assert D.q_global_pair_sum(g, 1, 1, [0, 0, 1, 1]) == 0
    assert D.q_global_pair_sum(g, 1, 1, [0, 0, 0, 0]) == 0
    assert D.q_global_pair_sum(g, 1, 1, [0, 1, 2, 3]) == F(-1, 4)


@pytest.mark.parametrize("seed", range(8))
def test_oracle_global_components_equal_definition(seed):
    rng, g, omega, gamma = _rand(50 + seed)
    og = oracle.OracleGraph(g, omega)
    for _ in range(4):
        m = np.array([rng.randrange(g.n_supra) for _ in range(g.n_supra)], dtype=np.int32)
        comps = og.q_components(m, null_model=1)
        assert oracle.q_global_from_components(comps, g.n_nodes, g.n_slices, gamma, omega) == \
            D.q_global_pair_sum(g, gamma, omega, m)


def _global_differences(seed, max_nodes=6):
    g, omega, gamma, lv, it, sw, sd = L.random_case(seed, max_nodes)
    m1, st1, tr1 = S.leiden(g, gamma, omega, lv, it, sw, sd, null_model=1)
    og = oracle.OracleGraph(g, omega)
    oracle.trace_enable(True)
    try:
        m2, _, st2 = og.leiden(gamma, lv, it, sw, sd, null_model=1)
        tr2 = oracle.trace_levels(g.n_supra)
    finally:
        oracle.trace_enable(False)
    diffs = [] if list(m2) == m1 else ["membership"]
    diffs += [k for k in st1 if st1[k] != int(st2[k])]
    if len(tr1) != len(tr2):
        return diffs + ["levels"]
    b = omega.denominator
    for a, rec in zip(tr1, tr2):
        for k in ("colour", "p_in", "p_lm"):
            if a[k] != [int(x) for x in rec[k]]:
                diffs.append(k)
        ra, rb = a.get("r"), rec["r"]
        if (ra is None) != (rb is None) or (ra is not None and ra != [int(x) for x in rb]):
            diffs.append("r")
        if rb is not None:
            for T, (_, ext, wc) in a["subs"].items():
                if rec["ext"][T] != ext * b or bool(rec["wc"][T]) != wc:
                    diffs.append("bookkeeping")
    return diffs


@pytest.mark.parametrize("chunk", range(4))
def test_c_oracle_global_equals_literal_schedule(chunk):
    for seed in range(2000 + chunk * 40, 2000 + chunk * 40 + 40):
        assert _global_differences(seed) == [], f"case {seed}"


CASES = [
    ("h2", lambda: gen.from_edge_lists(2, [[(0, 1)], [(0, 1)]]), F(1), F(1)),
    ("two_triangles", lambda: gen.from_edge_lists(6, [[(0, 1), (1, 2), (0, 2), (3, 4), (4, 5),
                                                       (3, 5), (2, 3)]]), F(1), F(1)),
    ("path5_T2", lambda: gen.from_edge_lists(5, [[(0, 1), (1, 2), (2, 3), (3, 4)],
                                                 [(0, 1), (1, 2), (3, 4), (2, 4)]]), F(1), F(1, 2)),
]


@pytest.mark.parametrize("name,make,gamma,omega", CASES)
def test_global_named_cases_reach_brute_force_optimum(name, make, gamma, omega):
    g = make()
    best, _ = D.brute_force_max_global(g, gamma, omega)
    m, comps, _ = oracle.OracleGraph(g, omega).leiden(gamma, max_iterations=0, null_model=1)
    assert oracle.q_global_from_components(comps, g.n_nodes, g.n_slices, gamma, omega) == best


@pytest.mark.parametrize("seed", range(12))
def test_global_tiny_random_below_optimum_and_connected(seed):
    rng, g, omega, gamma = _rand(300 + seed, max_nodes=3)
    if g.n_supra > 10:
        pytest.skip("brute force is for at most 10 supra-nodes")
    best, _ = D.brute_force_max_global(g, gamma, omega)
    m, comps, _ = oracle.OracleGraph(g, omega).leiden(gamma, max_iterations=0, null_model=1)
    q = oracle.q_global_from_components(comps, g.n_nodes, g.n_slices, gamma, omega)
    assert q <= best
    assert D.communities_connected(g, omega, m)
