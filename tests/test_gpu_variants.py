"""GPU parity of the variants of the objective and the input against the C oracle run with the
same variant: a resolution gamma^(s) per slice (Eq. 6), the multislice CPM (null term
gamma^(s) n_i n_j, node weight 1 per supra-node), and a start partition for the first
iteration (warm start / resume).  Identical memberships, Q components and schedule
statistics; the exact value from the library's reduction equals the oracle's rational one.
Also: batches, the serving loop, the allocation-free entry point and every tuning give each
variant its plain-call result; invalid variants are refused before any work.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from paper_2608_03695_amd import gen

pytestmark = pytest.mark.gpu

STAT_KEYS = ["sweeps", "moves", "sweep_cap_hits", "refine_rounds", "merges", "splits",
             "levels_run", "iterations_run", "n_communities"]
MS, GLOBAL, CPM = 0, 1, 2


def _mslm():
    from paper_2608_03695_amd import mslm
    return mslm


def _q_oracle(oc, tg, gamma, omega, nm, gs):
    gam = gs if gs is not None else gamma
    if nm == CPM:
        return oracle.q_cpm_from_components(oc, tg.n_nodes, tg.n_slices, gam, omega)
    if nm == GLOBAL:
        return oracle.q_global_from_components(oc, tg.n_nodes, tg.n_slices, gam, omega)
    return oracle.q_from_components(oc, tg.n_nodes, tg.n_slices, gam, omega)


def assert_same(tg, gamma, omega, null_model=MS, gamma_slices=None, initial=None, **kw):
    mslm = _mslm()
    om, oc, ost = oracle.OracleGraph(tg, omega).leiden(gamma, null_model=null_model,
                                                      gamma_slices=gamma_slices,
                                                      initial=initial, **kw)
    g = mslm.Graph(tg, omega)
    gm, gr = g.leiden(gamma, null_model=null_model, gamma_slices=gamma_slices, initial=initial,
                      **kw)
    g.close()
    case = (f"{tg.name} N={tg.n_nodes} T={tg.n_slices} gamma={gamma} omega={omega} "
            f"null_model={null_model} gamma_slices={gamma_slices} "
            f"initial={'yes' if initial is not None else 'no'} {kw}")
    bad = np.nonzero(gm != om)[0]
    assert bad.size == 0, f"{case}: {bad.size} memberships differ, first at {bad[:5]}"
    assert np.array_equal(gr["q_components"], oc), case
    for k in STAT_KEYS:
        assert gr[k] == ost[k], f"{case}: {k} gpu={gr[k]} oracle={ost[k]}"
    q = mslm.q_exact_variant(gr["q_components"], tg.n_slices, tg.n_nodes, gamma, omega,
                             null_model, gamma_slices)
    assert q == _q_oracle(oc, tg, gamma, omega, null_model, gamma_slices), case
    assert abs(gr["q"] - float(q)) <= 1e-12 * max(1.0, abs(float(q))), case
    return gm, gr


CASES = [
    ("er_sparse", lambda: gen.erdos_renyi(300, 3, 0.01, seed=1), F(1)),
    ("er_weighted", lambda: gen.erdos_renyi(200, 4, 0.03, seed=2, weights_max=8), F(1, 2)),
    ("planted_T5", lambda: gen.planted_partition(400, 5, 8, 0.08, 0.004, 0.1, seed=3), F(1, 10)),
    ("planted_omega10", lambda: gen.planted_partition(300, 3, 6, 0.1, 0.01, 0.2, seed=4), F(10)),
    ("static_T1", lambda: gen.planted_partition(500, 1, 5, 0.05, 0.005, 0.0, seed=6), F(1)),
    ("omega_zero", lambda: gen.planted_partition(200, 4, 4, 0.1, 0.01, 0.1, seed=7), F(0)),
    ("dcsbm_weighted", lambda: gen.dcsbm(2000, 6, 8, 20, 0.3, 2.5, 0.05, weights_max=8, seed=8), F(1)),
    ("dcsbm_hubs", lambda: gen.dcsbm(3000, 3, 12, 10, 0.4, 2.1, 0.02, seed=9), F(1, 2)),
    ("dcsbm_many_tiles", lambda: gen.dcsbm(20000, 4, 10, 40, 0.3, 2.3, 0.03, seed=10), F(1, 2)),
]
IDS = [c[0] for c in CASES]

RES = [F(1, 2), F(1), F(3, 2), F(2), F(3), F(2, 3)]
CPM_RES = [F(1, 50), F(1, 20), F(1, 100), F(1, 30), F(3, 100), F(1, 40)]


def _per_slice(T, base):
    return [base[(s * 5 + 1) % len(base)] for s in range(T)]


@pytest.mark.parametrize("name,make,omega", CASES, ids=IDS)
def test_per_slice_resolutions_parity(name, make, omega):
    tg = make()
    assert_same(tg, F(1), omega, gamma_slices=_per_slice(tg.n_slices, RES))


@pytest.mark.parametrize("name,make,omega", CASES, ids=IDS)
def test_multislice_cpm_parity(name, make, omega):
    assert_same(make(), F(1, 40), omega, null_model=CPM)


@pytest.mark.parametrize("name,make,omega", CASES[2:4] + CASES[6:], ids=IDS[2:4] + IDS[6:])
def test_multislice_cpm_per_slice_parity(name, make, omega):
    tg = make()
    assert_same(tg, F(1), omega, null_model=CPM, gamma_slices=_per_slice(tg.n_slices, CPM_RES))


@pytest.mark.parametrize("nm", [MS, GLOBAL, CPM])
@pytest.mark.parametrize("name,make,omega", CASES[2:3] + CASES[6:], ids=IDS[2:3] + IDS[6:])
def test_start_partition_parity(name, make, omega, nm):
    """Warm starts: the oracle's partition at another resolution, and a random partition."""
    tg = make()
    gamma = F(1) if nm != CPM else F(1, 40)
    warm, _, _ = oracle.OracleGraph(tg, omega).leiden(gamma * 2, null_model=nm)
    assert_same(tg, gamma, omega, null_model=nm, initial=warm)
    rng = np.random.default_rng(len(name) + nm)
    rand = rng.integers(0, tg.n_supra // 7 + 1, tg.n_supra) * 7   # labels in [0, N*T)
    assert_same(tg, gamma, omega, null_model=nm, initial=rand, max_iterations=1)


@pytest.mark.parametrize("nm", [MS, CPM])
def test_stable_start_comes_back_after_one_iteration(nm):
    mslm = _mslm()
    tg = gen.dcsbm(3000, 3, 12, 10, 0.4, 2.1, 0.02, seed=9)
    g = mslm.Graph(tg, F(1, 2))
    gamma = F(1) if nm == MS else F(1, 40)
    m, r = g.leiden(gamma, null_model=nm, max_iterations=0)
    perm = np.random.default_rng(3).permutation(tg.n_supra).astype(np.int32)
    for init in (m, perm[m]):
        m2, r2 = g.leiden(gamma, null_model=nm, max_iterations=0, initial=init)
        assert np.array_equal(m2, m)
        assert np.array_equal(r2["q_components"], r["q_components"])
        assert r2["iterations_run"] == 1
    g.close()


def _variant_solves(tgs):
    T = [tg.n_slices for tg in tgs]
    warm = oracle.OracleGraph(tgs[1], F(1)).leiden(F(2))[0]
    return [
        (0, F(1), F(1), 32, 2, 0),
        (0, F(1), F(1), 32, 2, 0, MS, _per_slice(T[0], RES)),
        (1, F(1, 40), F(1), 32, 2, 0, CPM),
        (1, F(1), F(1), 32, 2, 0, MS, None, warm),
        (2, F(1), F(1, 2), 32, 0, 5, GLOBAL, None, np.zeros(tgs[2].n_supra, np.int32)),
        (2, F(1), F(1, 2), 32, 2, 0, CPM, _per_slice(T[2], CPM_RES)),
        (0, F(1, 40), F(1), 32, 2, 0, CPM),
        (1, F(1), F(10), 32, 1, 3, MS, _per_slice(T[1], RES), warm),
    ]


def test_batch_of_variants_equals_plain_calls_and_the_oracle():
    mslm = _mslm()
    tgs = [gen.planted_partition(300, 3, 6, 0.1, 0.01, 0.2, seed=4),
           gen.dcsbm(2000, 4, 8, 20, 0.3, 2.5, 0.05, weights_max=4, seed=8),
           gen.dcsbm(3000, 3, 12, 10, 0.4, 2.1, 0.02, seed=9)]
    handles = [mslm.Graph(tg, 1) for tg in tgs]
    solves = _variant_solves(tgs)
    got = mslm.batch_leiden(handles, solves)
    for sv, (bm, br) in zip(solves, got):
        gi, gamma, omega, lv, it, seed = sv[:6]
        nm = sv[6] if len(sv) > 6 else MS
        gs = sv[7] if len(sv) > 7 else None
        ini = sv[8] if len(sv) > 8 else None
        pm, pr = handles[gi].leiden(gamma, omega, max_levels=lv, max_iterations=it, seed=seed,
                                    null_model=nm, gamma_slices=gs, initial=ini)
        case = f"graph {gi} {sv[1:6]} nm={nm} gs={gs is not None} init={ini is not None}"
        assert np.array_equal(bm, pm), case
        assert np.array_equal(br["q_components"], pr["q_components"]), case
        for k in STAT_KEYS:
            assert br[k] == pr[k], f"{case}: {k}"
        om, oc, ost = oracle.OracleGraph(tgs[gi], omega).leiden(
            gamma, max_levels=lv, max_iterations=it, seed=seed, null_model=nm, gamma_slices=gs,
            initial=ini)
        assert np.array_equal(bm, om) and np.array_equal(br["q_components"], oc), case
    for h in handles:
        h.close()


def test_server_and_static_entry_run_the_variants():
    mslm = _mslm()
    tg = gen.dcsbm(2000, 4, 8, 20, 0.3, 2.5, 0.05, weights_max=4, seed=8)
    warm = oracle.OracleGraph(tg, F(1)).leiden(F(2))[0]
    reqs = [dict(gamma=F(1), gamma_slices=_per_slice(4, RES)),
            dict(gamma=F(1, 40), null_model=CPM),
            dict(gamma=F(1), initial=warm),
            dict(gamma=F(1), null_model=CPM, gamma_slices=_per_slice(4, CPM_RES), initial=warm)]
    srv = mslm.Server(1 << 30, max_slots=2)
    tickets = [srv.submit(tg, omega=F(1), **r) for r in reqs]
    g = mslm.Graph(tg, F(1))
    for r, t in zip(reqs, tickets):
        sm, sr, _ = srv.wait(t)
        pm, pr = g.leiden(**r)
        am, ar = g.leiden(no_alloc=True, **r)
        for m, res, how in ((sm, sr, "server"), (am, ar, "static")):
            assert np.array_equal(m, pm), f"{how} {r.keys()}"
            assert np.array_equal(res["q_components"], pr["q_components"]), how
            for k in STAT_KEYS:
                assert res[k] == pr[k], f"{how}: {k}"
    srv.close()
    g.close()


def test_tunings_never_change_a_variant_result():
    mslm = _mslm()
    tg = gen.dcsbm(20000, 4, 10, 40, 0.3, 2.3, 0.03, seed=10)
    g = mslm.Graph(tg, F(1, 2))
    warm = oracle.OracleGraph(tg, F(1, 2)).leiden(F(2), max_iterations=1)[0]
    kws = [dict(gamma=F(1, 40), null_model=CPM),
           dict(gamma=F(1), gamma_slices=_per_slice(4, RES), initial=warm)]
    base = [g.leiden(**kw) for kw in kws]
    default = g.tuning()
    for tu in (dict(graphs=1, split_group_units=0, copy_moves=1),
               dict(latency_units=4096, lat_parts_max=1, copy_moves=1 << 30)):
        g.set_tuning(**default)
        g.set_tuning(**tu)
        for kw, (bm, br) in zip(kws, base):
            m, r = g.leiden(**kw)
            assert np.array_equal(m, bm), f"{tu} {kw.keys()}"
            assert np.array_equal(r["q_components"], br["q_components"])
            for k in STAT_KEYS:
                assert r[k] == br[k], f"{tu}: {k}"
    g.close()


def test_invalid_variants_are_refused_and_the_handle_stays_valid():
    mslm = _mslm()
    tg = gen.planted_partition(100, 3, 4, 0.1, 0.01, 0.1, seed=2)
    g = mslm.Graph(tg, F(1))
    n = tg.n_supra
    bad = [
        (dict(gamma_slices=[F(1)] * 3, null_model=GLOBAL), mslm.MSLM_EINVAL),
        (dict(gamma_slices=[F(1), F(0), F(1)]), mslm.MSLM_EINVAL),
        (dict(null_model=3), mslm.MSLM_EINVAL),
        (dict(initial=np.full(n, n, np.int32)), mslm.MSLM_EINVAL),
        (dict(initial=np.full(n, -1, np.int32)), mslm.MSLM_EINVAL),
        # coprime resolution denominators whose common multiple passes 2^31
        (dict(gamma_slices=[F(1, 65521), F(1, 65519), F(1, 65497)]), mslm.MSLM_EOVERFLOW),
    ]
    for kw, code in bad:
        with pytest.raises(mslm.MslmError) as e:
            g.leiden(F(1), **kw)
        assert e.value.status == code, kw
    m, r = g.leiden(F(1))
    om, oc, _ = oracle.OracleGraph(tg, F(1)).leiden(F(1))
    assert np.array_equal(m, om) and np.array_equal(r["q_components"], oc)
    g.close()
