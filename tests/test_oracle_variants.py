"""Pins of the oracle's variants of the objective and the input (Eq. 6 in its full generality,
Section 3.2): a resolution gamma^(s) per slice, the multislice CPM (null term gamma^(s) n_i n_j
with node weight 1 per supra-node, same 1/2mu normalisation), and a start partition for the
first iteration (warm start / resume).

* Definitional tier: the literal quadruple sum, the trace form and the component form agree
  for per-slice resolutions and for the CPM; closed forms (all singletons, one community); a
  hand value of the CPM.
* The C oracle's Q components reproduce the definitional Q under every variant.
* The C oracle equals the literal schedule (every decision on the exact change of the
  objective) level by level on random tiny graphs under every variant, and planted mistakes in
  the variant code are caught by that comparison.
* Reductions to textbook cases: equal per-slice resolutions are the single-gamma solve; the
  CPM at gamma = 0 gives the connected components of the supra-graph (a library routine); a
  CPM resolution above every weight leaves singletons; an identity start is the cold start; a
  stable partition given as the start comes back after one iteration, under any relabelling.
* Named cases reach the brute-force optimum; random tiny graphs stay below it with connected
  communities and no improving single move at a stable stop; a warm start never lowers Q.
"""
import os
import random
import subprocess
import sys
from fractions import Fraction as F

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle
from oracle import definitional as D
from oracle import schedule as S
from paper_2608_03695_amd import gen

import test_oracle_literal as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KINDS = ["per_slice", "cpm", "cpm_per_slice", "warm", "warm_cpm", "warm_per_slice"]


def variant_case(seed, max_nodes=6):
    """A random tiny case of the literal tests plus one variant: per-slice resolutions, the
    CPM, and/or a random start partition."""
    g, omega, gamma, lv, it, sw, sd = L.random_case(seed, max_nodes)
    rng = random.Random(seed * 7919 + 11)
    kind = KINDS[seed % len(KINDS)]
    kw = {}
    if "per_slice" in kind:
        kw["gamma_slices"] = [rng.choice([F(1, 8), F(1, 3), F(1), F(3, 2), F(4), F(9)])
                              for _ in range(g.n_slices)]
    if "cpm" in kind:
        kw["null_model"] = 2
        # CPM resolutions are on the scale of one edge weight
        if "gamma_slices" in kw:
            kw["gamma_slices"] = [x / 4 for x in kw["gamma_slices"]]
        gamma = gamma / 4
    if "warm" in kind:
        n = g.n_supra
        k = rng.randint(1, n)
        kw["initial"] = [rng.randrange(k) * (n // k) for _ in range(n)]   # labels in [0, n)
    return g, omega, gamma, lv, it, sw, sd, kw


def run_variant(seed, max_nodes=6):
    g, omega, gamma, lv, it, sw, sd, kw = variant_case(seed, max_nodes)
    m1, st1, tr1 = S.leiden(g, gamma, omega, lv, it, sw, sd, **kw)
    og = oracle.OracleGraph(g, omega)
    oracle.trace_enable(True)
    try:
        m2, c2, st2 = og.leiden(gamma, lv, it, sw, sd, **kw)
        tr2 = oracle.trace_levels(g.n_supra)
    finally:
        oracle.trace_enable(False)
    return (g, omega, gamma, kw), (m1, st1, tr1), (m2, {k: int(v) for k, v in st2.items()}, tr2)


def variant_differences(seed, max_nodes=6):
    (g, omega, gamma, kw), (m1, st1, tr1), (m2, st2, tr2) = run_variant(seed, max_nodes)
    diffs = [] if list(m2) == m1 else ["membership"]
    diffs += [k for k in st1 if st1[k] != st2[k]]
    if len(tr1) != len(tr2):
        return diffs + ["levels"]
    b = omega.denominator
    for a, rec in zip(tr1, tr2):
        where = f"@it{a['it']}/lvl{a['lvl']}"
        for k in ("colour", "p_in", "p_lm"):
            if a[k] != [int(x) for x in rec[k]]:
                diffs.append(k + where)
        ra, rb = a.get("r"), rec["r"]
        if (ra is None) != (rb is None) or (ra is not None and ra != [int(x) for x in rb]):
            diffs.append("r" + where)
            continue
        if rb is not None and "subs" in a:
            for T, (_, ext, wc) in a["subs"].items():
                if rec["ext"][T] != ext * b or bool(rec["wc"][T]) != wc:
                    diffs.append("bookkeeping" + where)
    return diffs


def first_caught_variant(seeds):
    for s in seeds:
        if variant_differences(s):
            return s
    return None


def _q(g, gamma, omega, memb, cpm):
    return D.q_quadruple_sum(g, gamma, omega, np.asarray(memb), cpm=cpm)


# --------------------------------------------------------------------------- definitional tier

@pytest.mark.parametrize("seed", range(8))
def test_three_forms_agree_per_slice_and_cpm(seed):
    rng = random.Random(400 + seed)
    n, t = rng.randint(2, 4), rng.randint(1, 3)
    g = gen.erdos_renyi(n, t, 0.7, seed=seed, weights_max=3)
    omega = F(rng.randint(0, 3), rng.randint(1, 3))
    gam = [F(rng.randint(1, 5), rng.randint(1, 3)) for _ in range(t)]
    for cpm in (False, True):
        for _ in range(3):
            m = np.array([rng.randrange(n * t) for _ in range(n * t)])
            a = D.q_quadruple_sum(g, gam, omega, m, cpm=cpm)
            assert a == D.q_trace_form(g, gam, omega, m, cpm=cpm)
            assert a == D.q_component_form(g, gam, omega, m, cpm=cpm)
        assert D.q_quadruple_sum(g, gam, omega, np.arange(n * t), cpm=cpm) == \
            D.q_all_singletons(g, gam, omega, cpm=cpm)
        assert D.q_quadruple_sum(g, gam, omega, np.zeros(n * t, int), cpm=cpm) == \
            D.q_one_community(g, gam, omega, cpm=cpm)


def test_per_slice_gamma_weights_each_slice_by_its_own_resolution():
    """With omega = 0 the objective splits by slice: 2mu Q = sum_s 2m_s Q_s with Q_s the
    Newman modularity of slice s at its own resolution."""
    g = gen.erdos_renyi(5, 3, 0.6, seed=3, weights_max=2)
    gam = [F(1, 2), F(1), F(3)]
    rng = random.Random(1)
    for _ in range(5):
        m = np.array([rng.randrange(4) for _ in range(15)])
        total = F(0)
        two_mu = F(0)
        for s in range(3):
            u, x, w = g.slice_edges(s)
            w = np.ones_like(u) if w is None else w
            sub = gen.from_edge_lists(5, [[(int(a), int(b), int(c)) for a, b, c in zip(u, x, w)]],
                                      weighted=True)
            tm = sum(sum(r) for r in D.slice_matrices(sub)[0])
            two_mu += tm
            total += tm * D.q_newman_static(sub, gam[s], m[5 * s:5 * s + 5])
        assert D.q_quadruple_sum(g, gam, 0, m) == total / two_mu


def test_cpm_hand_values():
    """A triangle, T = 1, unit weights, gamma = 1/2: 2mu = 6.  One community: W = 6 (both
    directions), SS = 3^2 = 9, Q = (6 - 9/2) / 6 = 1/4.  Singletons: Q = -3/2 / 6 = -1/4.
    {0,1},{2}: W = 2, SS = 4 + 1, Q = (2 - 5/2) / 6 = -1/12."""
    g = gen.from_edge_lists(3, [[(0, 1), (1, 2), (0, 2)]])
    assert _q(g, F(1, 2), 1, [0, 0, 0], True) == F(1, 4)
    assert _q(g, F(1, 2), 1, [0, 1, 2], True) == F(-1, 4)
    assert _q(g, F(1, 2), 1, [0, 0, 1], True) == F(-1, 12)


@pytest.mark.parametrize("seed", range(8))
def test_oracle_components_equal_definition_under_variants(seed):
    rng = random.Random(500 + seed)
    n, t = rng.randint(2, 4), rng.randint(1, 3)
    g = gen.erdos_renyi(n, t, 0.7, seed=seed, weights_max=3)
    omega = F(rng.randint(0, 3), rng.randint(1, 3))
    gam = [F(rng.randint(1, 5), rng.randint(1, 3)) for _ in range(t)]
    og = oracle.OracleGraph(g, omega)
    for _ in range(4):
        m = np.array([rng.randrange(n * t) for _ in range(n * t)], dtype=np.int32)
        c0 = og.q_components(m)
        assert oracle.q_from_components(c0, n, t, gam, omega) == _q(g, gam, omega, m, False)
        c2 = og.q_components(m, null_model=2)
        assert oracle.q_cpm_from_components(c2, n, t, gam, omega) == _q(g, gam, omega, m, True)
        # the CPM components differ from Eq. 6's only in SS_s: squared community sizes
        for s in range(t):
            sizes = np.bincount(m[s * n:(s + 1) * n])
            assert c2[t + s] == int((sizes * sizes).sum())
        assert list(c2[:t]) == list(c0[:t]) and list(c2[2 * t:]) == list(c0[2 * t:])


# --------------------------------------------------------------------------- C oracle == literal

@pytest.mark.parametrize("chunk", range(6))
def test_c_oracle_equals_literal_schedule_under_variants(chunk):
    for seed in range(chunk * 30, chunk * 30 + 30):
        assert variant_differences(seed) == [], f"case {seed} ({KINDS[seed % len(KINDS)]})"


def test_c_oracle_equals_literal_schedule_under_variants_larger():
    for seed in range(20_000, 20_024):
        assert variant_differences(seed, max_nodes=11) == [], f"case {seed}"


# one plausible mistake per case in the variant code of mslm_oracle.c
VARIANT_MUTATIONS = [
    ("first slice's resolution everywhere",
     "out->small = (i128)cf->gq[s] * cf->S[s] * W - (i128)(cf->gp[s] * cf->b) * ((i128)pk[0] * y[0]);",
     "out->small = (i128)cf->gq[0] * cf->S[s] * W - (i128)(cf->gp[0] * cf->b) * ((i128)pk[0] * y[0]);"),
    ("resolution numerator dropped on multi-slice units",
     "bn_mul_u64(&t1, (uint64_t)cf->gp[s]);", ""),
    ("CPM node weight 2", "g.ps[q] = (int32_t)(v / G->N); g.pk[q] = 1; q++;",
     "g.ps[q] = (int32_t)(v / G->N); g.pk[q] = 2; q++;"),
    ("CPM keeps 2m_s", "S[s] = null_model == 2 ? 1 : (G->twom[s] > 0 ? G->twom[s] : 1);",
     "S[s] = G->twom[s] > 0 ? G->twom[s] : 1;"),
    ("start partition not canonical",
     "for (int64_t v = 0; v < n0; v++) Pcur[v] = (int32_t)c0[v];",
     "for (int64_t v = 0; v < n0; v++) Pcur[v] = initial[v];"),
]


@pytest.mark.parametrize("what,old,new", VARIANT_MUTATIONS, ids=[m[0] for m in VARIANT_MUTATIONS])
def test_planted_variant_mistake_is_caught(tmp_path, what, old, new):
    src = open(os.path.join(ROOT, "oracle", "mslm_oracle.c")).read()
    assert src.count(old) == 1, what
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-o", str(lib), str(path)])
    code = ("import sys; sys.path.insert(0, %r); sys.path.insert(0, %r); "
            "import test_oracle_variants as t; print(t.first_caught_variant(range(300)))"
            % (ROOT, os.path.join(ROOT, "tests")))
    env = dict(os.environ, MSLM_ORACLE_LIB=str(lib), OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=600)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() != "None", f"planted mistake not caught: {what}"


# --------------------------------------------------------------------------- reductions

@pytest.mark.parametrize("seed", range(6))
def test_equal_per_slice_resolutions_are_the_single_gamma_solve(seed):
    g = gen.dcsbm(60, 3, 4, 6, 0.3, 2.5, 0.05, weights_max=3, seed=seed)
    gamma = [F(1, 2), F(1), F(3, 2)][seed % 3]
    og = oracle.OracleGraph(g, F(1, 2))
    for nm in (0, 2):
        gg = gamma if nm == 0 else gamma / 8
        a = og.leiden(gg, null_model=nm)
        b = og.leiden(F(7), null_model=nm, gamma_slices=[gg] * g.n_slices)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def _supra_components(g, omega):
    edges = D.supra_edges(g, omega)
    n = g.n_supra
    if not edges:
        return n, np.arange(n)
    r = [a for a, b, _ in edges]
    c = [b for a, b, _ in edges]
    A = coo_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
    return connected_components(A, directed=False)


@pytest.mark.parametrize("seed", range(6))
def test_cpm_at_zero_resolution_gives_connected_components(seed):
    rng = random.Random(600 + seed)
    g = gen.erdos_renyi(rng.randint(8, 30), rng.randint(1, 4), rng.uniform(0.02, 0.15),
                        seed=seed, weights_max=rng.choice([1, 3]))
    omega = rng.choice([F(0), F(1, 2), F(1)])
    m, comps, st = oracle.OracleGraph(g, omega).leiden(0, null_model=2, max_iterations=0)
    ncomp, lab = _supra_components(g, omega)
    # the same partition: labels by first appearance on both sides
    assert list(m) == S.canonical(list(lab))
    assert st["n_communities"] == ncomp


@pytest.mark.parametrize("seed", range(4))
def test_cpm_above_every_weight_leaves_singletons(seed):
    # the CPM null term acts inside a slice only (coupling entries always attract), so the
    # slices are left uncoupled; every intra weight is below every resolution
    g = gen.erdos_renyi(12, 3, 0.3, seed=seed, weights_max=3)
    omega = F(0)
    gam = [F(7), F(13, 2), F(9)]
    m, comps, _ = oracle.OracleGraph(g, omega).leiden(0, null_model=2, gamma_slices=gam)
    assert list(m) == list(range(g.n_supra))
    assert oracle.q_cpm_from_components(comps, 12, 3, gam, omega) == \
        D.q_all_singletons(g, gam, omega, cpm=True)


@pytest.mark.parametrize("nm", [0, 1, 2])
def test_identity_start_is_the_cold_start(nm):
    g = gen.dcsbm(80, 3, 4, 6, 0.3, 2.5, 0.05, seed=5)
    og = oracle.OracleGraph(g, F(1))
    gamma = F(1) if nm != 2 else F(1, 8)
    a = og.leiden(gamma, null_model=nm)
    b = og.leiden(gamma, null_model=nm, initial=np.arange(g.n_supra))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


@pytest.mark.parametrize("nm", [0, 1, 2])
def test_stable_start_returns_after_one_iteration_under_any_labelling(nm):
    g = gen.dcsbm(120, 3, 4, 8, 0.3, 2.5, 0.05, seed=6)
    og = oracle.OracleGraph(g, F(1, 2))
    gamma = F(1) if nm != 2 else F(1, 8)
    m, c, st = og.leiden(gamma, null_model=nm, max_iterations=0)
    rng = np.random.default_rng(nm)
    perm = rng.permutation(g.n_supra)
    for init in (m, perm[m]):   # the result, and the same partition under other labels
        m2, c2, st2 = og.leiden(gamma, null_model=nm, max_iterations=0, initial=init)
        assert np.array_equal(m2, m) and np.array_equal(c2, c)
        assert st2["iterations_run"] == 1


@pytest.mark.parametrize("seed", range(8))
def test_warm_start_never_lowers_q(seed):
    rng = random.Random(700 + seed)
    g = gen.erdos_renyi(6, 2, 0.5, seed=seed, weights_max=2)
    omega = F(1, 2)
    nm = [0, 2][seed % 2]
    gamma = F(1) if nm == 0 else F(1, 4)
    og = oracle.OracleGraph(g, omega)
    for _ in range(3):
        init = [rng.randrange(3) for _ in range(g.n_supra)]
        m, _, _ = og.leiden(gamma, null_model=nm, max_iterations=1, initial=init)
        assert _q(g, gamma, omega, m, nm == 2) >= _q(g, gamma, omega, init, nm == 2)


def test_variant_arguments_rejected():
    g = gen.erdos_renyi(4, 2, 0.5, seed=1)
    og = oracle.OracleGraph(g, 1)
    for kw in (dict(gamma_slices=[F(1), F(0)]),            # per-slice resolutions are positive
               dict(gamma_slices=[F(1), F(1)], null_model=1),
               dict(null_model=3),
               dict(initial=[0] * 7 + [8]),                  # labels in [0, N*T)
               dict(initial=[-1] + [0] * 7)):
        with pytest.raises(ValueError):
            og.leiden(F(1), **kw)


# --------------------------------------------------------------------------- optimum, invariants

NAMED = [
    ("two_triangles_cpm", lambda: gen.from_edge_lists(6, [[(0, 1), (1, 2), (0, 2), (3, 4), (4, 5),
                                                           (3, 5), (2, 3)]]), F(1, 2), F(1), 2, None),
    ("path5_T2_cpm", lambda: gen.from_edge_lists(5, [[(0, 1), (1, 2), (2, 3), (3, 4)],
                                                     [(0, 1), (1, 2), (3, 4), (2, 4)]]),
     F(1, 3), F(1, 2), 2, None),
    ("h2_per_slice", lambda: gen.from_edge_lists(2, [[(0, 1)], [(0, 1)]]), F(1), F(1), 0,
     [F(1, 2), F(2)]),
    ("two_triangles_T1_per_slice", lambda: gen.from_edge_lists(
        6, [[(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (2, 3)]]), F(1), F(1), 0, [F(3, 2)]),
]


@pytest.mark.parametrize("name,make,gamma,omega,nm,gs", NAMED, ids=[x[0] for x in NAMED])
def test_named_variant_cases_reach_brute_force_optimum(name, make, gamma, omega, nm, gs):
    g = make()
    gam = gs if gs is not None else gamma
    best, _ = D.brute_force_max(g, gam, omega, cpm=nm == 2)
    m, comps, _ = oracle.OracleGraph(g, omega).leiden(gamma, max_iterations=0, null_model=nm,
                                                      gamma_slices=gs)
    assert _q(g, gam, omega, m, nm == 2) == best


@pytest.mark.parametrize("seed", range(12))
def test_variant_tiny_random_below_optimum_connected_node_optimal(seed):
    rng = random.Random(800 + seed)
    n, t = rng.randint(2, 3), rng.randint(1, 3)
    g = gen.erdos_renyi(n, t, rng.uniform(0.4, 0.9), seed=seed, weights_max=rng.choice([1, 3]))
    omega = F(rng.randint(0, 3), rng.randint(1, 2))
    nm = [0, 2][seed % 2]
    gs = [F(rng.randint(1, 4), rng.randint(1, 4)) / (4 if nm == 2 else 1) for _ in range(t)]
    best, _ = D.brute_force_max(g, gs, omega, cpm=nm == 2)
    m, comps, _ = oracle.OracleGraph(g, omega).leiden(1, max_iterations=0, null_model=nm,
                                                      gamma_slices=gs)
    q = _q(g, gs, omega, m, nm == 2)
    assert q <= best
    if nm == 2:
        assert oracle.q_cpm_from_components(comps, n, t, gs, omega) == q
    else:
        assert oracle.q_from_components(comps, n, t, gs, omega) == q
    assert D.communities_connected(g, omega, m)
    assert D.improving_single_moves(g, gs, omega, m, cpm=nm == 2) == []
