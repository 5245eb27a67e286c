"""GPU parity of the global null-model mode (the modularity of Eq. 5 over the whole supra-graph
of Eq. 3, which the paper's GPU path optimised in place of Q_MS) against the C oracle run with
the same null model: identical memberships, Q components and schedule statistics; Q_G from the
library's reduction equals the oracle's rational value.  Also: batches and the serving loop
that mix the two null models give every solve its plain-call result, the allocation-free
entry point agrees, and the global head-room is checked before any work.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from paper_2608_03695_amd import gen

pytestmark = pytest.mark.gpu

STAT_KEYS = ["sweeps", "moves", "sweep_cap_hits", "refine_rounds", "merges", "splits",
             "levels_run", "iterations_run", "n_communities"]
GLOBAL = 1


def _mslm():
    from paper_2608_03695_amd import mslm
    return mslm


def assert_same_global(tg, gamma, omega, **kw):
    mslm = _mslm()
    om, oc, ost = oracle.OracleGraph(tg, omega).leiden(gamma, null_model=GLOBAL, **kw)
    g = mslm.Graph(tg, omega)
    gm, gr = g.leiden(gamma, null_model=GLOBAL, **kw)
    g.close()
    case = f"{tg.name} N={tg.n_nodes} T={tg.n_slices} gamma={gamma} omega={omega} {kw}"
    bad = np.nonzero(gm != om)[0]
    assert bad.size == 0, f"{case}: {bad.size} memberships differ, first at {bad[:5]}"
    assert np.array_equal(gr["q_components"], oc), case
    for k in STAT_KEYS:
        assert gr[k] == ost[k], f"{case}: {k} gpu={gr[k]} oracle={ost[k]}"
    q = mslm.q_exact_global(gr["q_components"], tg.n_slices, tg.n_nodes, gamma, omega)
    assert q == oracle.q_global_from_components(oc, tg.n_nodes, tg.n_slices, gamma, omega), case
    return gm, gr


CASES = [
    ("er_sparse", lambda: gen.erdos_renyi(300, 3, 0.01, seed=1), F(1), F(1)),
    ("er_weighted", lambda: gen.erdos_renyi(200, 4, 0.03, seed=2, weights_max=8), F(1), F(1, 2)),
    ("planted_T5", lambda: gen.planted_partition(400, 5, 8, 0.08, 0.004, 0.1, seed=3), F(1), F(1, 10)),
    ("planted_gamma2", lambda: gen.planted_partition(300, 3, 6, 0.1, 0.01, 0.2, seed=4), F(2), F(10)),
    ("static_T1", lambda: gen.planted_partition(500, 1, 5, 0.05, 0.005, 0.0, seed=6), F(1), F(1)),
    ("omega_zero", lambda: gen.planted_partition(200, 4, 4, 0.1, 0.01, 0.1, seed=7), F(1), F(0)),
    ("dcsbm_small", lambda: gen.dcsbm(2000, 6, 8, 20, 0.3, 2.5, 0.05, weights_max=8, seed=8), F(1), F(1)),
    ("dcsbm_hubs", lambda: gen.dcsbm(3000, 3, 12, 10, 0.4, 2.1, 0.02, seed=9), F(1), F(1, 2)),
    ("dcsbm_many_tiles", lambda: gen.dcsbm(20000, 4, 10, 40, 0.3, 2.3, 0.03, seed=10), F(1), F(1, 2)),
]


@pytest.mark.parametrize("name,make,gamma,omega", CASES, ids=[c[0] for c in CASES])
def test_global_null_model_full_parity(name, make, gamma, omega):
    assert_same_global(make(), gamma, omega, max_levels=32, max_iterations=2, seed=0)


@pytest.mark.parametrize("kw", [
    dict(max_levels=1, max_iterations=1, max_sweeps=1),
    dict(max_levels=2, max_iterations=1),
    dict(max_levels=32, max_iterations=0),
    dict(max_levels=32, max_iterations=3, seed=777),
])
def test_global_schedule_knobs(kw):
    tg = gen.planted_partition(500, 4, 10, 0.06, 0.004, 0.1, seed=11)
    assert_same_global(tg, F(1), F(1), **kw)


def test_global_degenerate_graphs():
    assert_same_global(gen.from_edge_lists(3, [[], [], []]), F(1), F(1), max_iterations=0)
    assert_same_global(gen.from_edge_lists(4, [[]]), F(1), F(1))
    assert_same_global(gen.from_edge_lists(1, [[]] * 5), F(2), F(1, 3))
    assert_same_global(gen.from_edge_lists(3, [[], [], []]), F(1), F(0))
    assert_same_global(gen.from_edge_lists(4, [[(0, 1, 2), (1, 0, 3), (2, 3, 1)], [(0, 2, 5)]],
                                           weighted=True), F(1), F(1))


def test_global_hand_example_reaches_brute_force_optimum():
    from oracle import definitional as D
    mslm = _mslm()
    tg = gen.from_edge_lists(5, [[(0, 1), (1, 2), (2, 3), (3, 4)],
                             [(0, 1), (1, 2), (3, 4), (2, 4)]])
    best, _ = D.brute_force_max_global(tg, F(1), F(1, 2))
    g = mslm.Graph(tg, F(1, 2))
    m, r = g.leiden(F(1), null_model=GLOBAL, max_iterations=0)
    g.close()
    assert mslm.q_exact_global(r["q_components"], 2, 5, F(1), F(1, 2)) == best


def test_batch_mixing_null_models_equals_plain_calls():
    mslm = _mslm()
    tgs = [gen.planted_partition(300, 3, 5, 0.1, 0.01, 0.1, seed=31),
           gen.dcsbm(1500, 5, 10, 12, 0.3, 2.5, 0.05, weights_max=8, seed=32),
           gen.from_edge_lists(3, [[], []])]
    handles = [mslm.Graph(tg, 1) for tg in tgs]
    solves = []
    for gi in range(len(tgs)):
        for gamma, omega in ((F(1), F(1, 10)), (F(2), F(1))):
            for nm in (0, GLOBAL):
                solves.append((gi, gamma, omega, 32, 2, 0, nm))
    got = mslm.batch_leiden(handles, solves)
    for (gi, gamma, omega, lv, it, seed, nm), (m, r) in zip(solves, got):
        pm, pr = handles[gi].leiden(gamma, omega, max_levels=lv, max_iterations=it, seed=seed,
                                    null_model=nm)
        case = f"graph {gi} gamma={gamma} omega={omega} null_model={nm}"
        assert np.array_equal(m, pm), case
        assert np.array_equal(r["q_components"], pr["q_components"]), case
        for k in STAT_KEYS:
            assert r[k] == pr[k], f"{case}: {k}"
    for h in handles:
        h.close()
    # one of the global solves against the oracle directly
    om, oc, _ = oracle.OracleGraph(tgs[1], F(1)).leiden(F(2), null_model=GLOBAL)
    m, r = got[[s[:3] + (s[6],) for s in solves].index((1, F(2), F(1), GLOBAL))]
    assert np.array_equal(m, om)
    assert np.array_equal(r["q_components"], oc)


def test_server_serves_global_requests():
    mslm = _mslm()
    tgs = [gen.planted_partition(300, 3, 5, 0.1, 0.01, 0.1, seed=31),
           gen.erdos_renyi(200, 2, 0.03, seed=33)]
    srv = mslm.Server(8 << 30, max_slots=2)
    reqs = [(tgs[i % 2], F(1), F(1, 2), (0, GLOBAL)[(i // 2) % 2]) for i in range(6)]
    tickets = [srv.submit(tg, gamma, omega, null_model=nm) for tg, gamma, omega, nm in reqs]
    outs = [srv.wait(t) for t in tickets]
    srv.close()
    for (tg, gamma, omega, nm), (m, r, _) in zip(reqs, outs):
        om, oc, ost = oracle.OracleGraph(tg, omega).leiden(gamma, null_model=nm)
        assert np.array_equal(m, om), (tg.name, nm)
        assert np.array_equal(r["q_components"], oc), (tg.name, nm)
        for k in STAT_KEYS:
            assert r[k] == ost[k], (tg.name, nm, k)


def test_global_allocation_free_entry_agrees():
    mslm = _mslm()
    tg = gen.dcsbm(3000, 3, 12, 10, 0.4, 2.1, 0.02, seed=9)
    g = mslm.Graph(tg, F(1, 2))
    a, ra = g.leiden(F(1), null_model=GLOBAL)
    b, rb = g.leiden(F(1), null_model=GLOBAL, no_alloc=True)
    g.close()
    assert np.array_equal(a, b)
    assert np.array_equal(ra["q_components"], rb["q_components"])


def test_global_headroom_refused_before_work():
    """2mu' = b * sum 2m_s + 2 a N (T-1) must stay below 2^31 and max(p,q) * 2mu'^2 below
    2^62: gamma = 2^30 on 2mu' > 2^16 is refused (EOVERFLOW) by the plain call and at submit,
    and the handle stays usable."""
    mslm = _mslm()
    tg = gen.erdos_renyi(400, 1, 0.45, seed=5, name="dense400")
    g = mslm.Graph(tg, 1)
    with pytest.raises(mslm.MslmError) as e:
        g.leiden(F(1 << 30), null_model=GLOBAL)
    assert e.value.status == mslm.MSLM_EOVERFLOW
    m, r = g.leiden(F(1), null_model=GLOBAL)
    g.close()
    om, oc, _ = oracle.OracleGraph(tg, 1).leiden(F(1), null_model=GLOBAL)
    assert np.array_equal(m, om)
    assert np.array_equal(r["q_components"], oc)
    srv = mslm.Server(8 << 30, max_slots=1)
    with pytest.raises(mslm.MslmError) as e:
        srv.submit(tg, F(1 << 30), F(1), null_model=GLOBAL)
    assert e.value.status == mslm.MSLM_EOVERFLOW
    srv.close()
