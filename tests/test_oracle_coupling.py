"""Pins of the oracle's general coupling (Eq. 6's omega^(sr), Section 3.2; Table 1's absent
copies): omega^(sr) = omega * c_sr for an integer matrix c (ordinal, categorical, or varying
over time), optionally only between copies present in both slices (a copy is present when it
has an edge in its slice; under the CPM an absent copy carries node weight 0).

* Definitional tier: the supra-adjacency has the coupling blocks c_sr omega I (restricted to
  present copies); the three forms of the objective agree under general coupling, also with
  per-slice resolutions and the CPM; closed forms; a hand value of categorical coupling.
* The C oracle's CSR equals the dense supra-adjacency, its coupling total equals the sum of
  the coupling weights over omega, and its Q components give the definitional Q.
* The C oracle equals the literal schedule level by level on random tiny graphs under random
  coupling matrices and present-only copies, with planted mistakes caught.
* Reductions: the ordinal matrix is the default; present-only coupling on a graph whose copies
  all have edges is the default; categorical coupling at T = 2 is ordinal coupling.
* Named cases reach the brute-force optimum; random tiny graphs stay below it with connected
  communities and no improving single move.
"""
import os
import random
import subprocess
import sys
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from oracle import definitional as D
from oracle import schedule as S
from paper_2608_03695_amd import gen

import test_oracle_literal as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def random_matrix(rng, T, cmax=3):
    c = [[0] * T for _ in range(T)]
    for s in range(T):
        for r in range(s + 1, T):
            c[s][r] = c[r][s] = rng.randint(0, cmax)
    return c


def coupling_case(seed, max_nodes=6):
    g, omega, gamma, lv, it, sw, sd = L.random_case(seed, max_nodes)
    rng = random.Random(seed * 104729 + 3)
    T = g.n_slices
    kind = seed % 4
    cm = None if kind == 0 else random_matrix(rng, T)
    present_only = kind in (0, 2)
    if present_only and seed % 3 == 0:   # copies without edges, whose coupling is dropped
        g = _with_absent_copies(seed, n=max(3, min(max_nodes, 6)), t=T)
    kw = {}
    if seed % 5 == 1:
        kw["null_model"] = 2
        gamma = gamma / 4
    if seed % 7 == 2:
        kw["gamma_slices"] = [rng.choice([F(1, 3), F(1), F(3)]) for _ in range(T)]
        if kw.get("null_model") == 2:
            kw["gamma_slices"] = [x / 4 for x in kw["gamma_slices"]]
    if seed % 9 == 4 and kw.get("null_model") is None and "gamma_slices" not in kw:
        kw["null_model"] = 1
    return g, omega, gamma, lv, it, sw, sd, cm, present_only, kw


def coupling_differences(seed, max_nodes=6):
    g, omega, gamma, lv, it, sw, sd, cm, po, kw = coupling_case(seed, max_nodes)
    m1, st1, tr1 = S.leiden(g, gamma, omega, lv, it, sw, sd, coupling=cm, present_only=po, **kw)
    og = oracle.OracleGraph(g, omega, coupling=cm, present_only=po)
    oracle.trace_enable(True)
    try:
        m2, c2, st2 = og.leiden(gamma, lv, it, sw, sd, **kw)
        tr2 = oracle.trace_levels(g.n_supra)
    finally:
        oracle.trace_enable(False)
    st2 = {k: int(v) for k, v in st2.items()}
    diffs = [] if list(m2) == m1 else ["membership"]
    # the objective's value from the oracle's components against its definition
    cp = D.Coupling(omega, cm, po)
    nm = kw.get("null_model", 0)
    gam = kw.get("gamma_slices") or gamma
    n, T, ctot = g.n_nodes, g.n_slices, og.coupling_total()
    if nm == 1:
        qc = oracle.q_global_from_components(c2, n, T, gamma, omega, ctot)
        qd = D.q_global_pair_sum(g, gamma, cp, m2)
    elif nm == 2:
        qc = oracle.q_cpm_from_components(c2, n, T, gam, omega, ctot)
        qd = D.q_quadruple_sum(g, gam, cp, m2, cpm=True)
    else:
        qc = oracle.q_from_components(c2, n, T, gam, omega, ctot)
        qd = D.q_quadruple_sum(g, gam, cp, m2)
    if qc != qd:
        diffs.append("q")
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
            for T_, (_, ext, wc) in a["subs"].items():
                if rec["ext"][T_] != ext * b or bool(rec["wc"][T_]) != wc:
                    diffs.append("bookkeeping" + where)
    return diffs


def first_caught_coupling(seeds):
    for s in seeds:
        if coupling_differences(s):
            return s
    return None


def _with_absent_copies(seed, n=5, t=3):
    """A tiny graph in which some copies have no edge (absent)."""
    rng = random.Random(seed)
    edges = []
    for s in range(t):
        active = rng.sample(range(n), rng.randint(2, n - 1))
        es = set()
        for _ in range(rng.randint(1, 4)):
            a, b = rng.sample(active, 2)
            es.add((min(a, b), max(a, b)))
        edges.append(sorted(es))
    return gen.from_edge_lists(n, edges)


# --------------------------------------------------------------------------- definitional tier

def test_supra_adjacency_has_the_coupling_blocks():
    g = _with_absent_copies(1, n=4, t=3)
    cm = [[0, 2, 1], [2, 0, 3], [1, 3, 0]]
    n = 4
    pres = D.presence(g)
    for po in (False, True):
        A = D.supra_adjacency(g, D.Coupling(F(1, 2), cm, po))
        for s in range(3):
            for r in range(3):
                if s == r:
                    continue
                for i in range(n):
                    for j in range(n):
                        want = F(0)
                        if i == j and (not po or (pres[s][i] and pres[r][i])):
                            want = F(cm[s][r], 2)
                        assert A[s * n + i][r * n + j] == want


@pytest.mark.parametrize("seed", range(10))
def test_three_forms_agree_under_general_coupling(seed):
    rng = random.Random(1000 + seed)
    g = _with_absent_copies(seed, n=rng.randint(3, 4), t=rng.randint(2, 3))
    cp = D.Coupling(F(rng.randint(1, 3), rng.randint(1, 2)), random_matrix(rng, g.n_slices),
                    rng.random() < 0.5)
    gam = [F(rng.randint(1, 4), rng.randint(1, 3)) for _ in range(g.n_slices)]
    size = g.n_supra
    for cpm in (False, True):
        for _ in range(3):
            m = np.array([rng.randrange(size) for _ in range(size)])
            a = D.q_quadruple_sum(g, gam, cp, m, cpm=cpm)
            assert a == D.q_trace_form(g, gam, cp, m, cpm=cpm)
            assert a == D.q_component_form(g, gam, cp, m, cpm=cpm)
        assert D.q_quadruple_sum(g, gam, cp, np.arange(size), cpm=cpm) == \
            D.q_all_singletons(g, gam, cp, cpm=cpm)
        assert D.q_quadruple_sum(g, gam, cp, np.zeros(size, int), cpm=cpm) == \
            D.q_one_community(g, gam, cp, cpm=cpm)


def test_categorical_coupling_hand_value():
    """N = 1, T = 3, no edges, categorical coupling c_sr = 1 (s != r), omega = 1: the three
    copies form a triangle of coupling weight 1, 2mu = 6.  One community: the Eq. 6 null terms
    vanish (2m_s = 0), Q = 6/6 = 1.  Copies 0 and 1 together, 2 alone: Q = 2/6 = 1/3.  Under
    the CPM at gamma = 1/2 one community gives (6 - 3/2)/6 = 3/4."""
    g = gen.from_edge_lists(1, [[], [], []])
    cat = D.Coupling(1, [[0, 1, 1], [1, 0, 1], [1, 1, 0]])
    assert D.q_quadruple_sum(g, 1, cat, [0, 0, 0]) == 1
    assert D.q_quadruple_sum(g, 1, cat, [0, 0, 1]) == F(1, 3)
    assert D.q_quadruple_sum(g, F(1, 2), cat, [0, 0, 0], cpm=True) == F(3, 4)
    # ordinal coupling on the same copies: a path 0-1-2, 2mu = 4, one community Q = 1
    assert D.q_quadruple_sum(g, 1, 1, [0, 0, 0]) == 1
    assert D.two_mu(g, cat) == 6 and D.two_mu(g, 1) == 4


# --------------------------------------------------------------------------- C oracle

@pytest.mark.parametrize("seed", range(8))
def test_oracle_csr_total_and_components_equal_definition(seed):
    rng = random.Random(1100 + seed)
    g = _with_absent_copies(seed, n=rng.randint(3, 5), t=rng.randint(2, 4))
    T, n = g.n_slices, g.n_nodes
    omega = F(rng.randint(1, 3), rng.randint(1, 3))
    cm = random_matrix(rng, T)
    po = seed % 2 == 0
    cp = D.Coupling(omega, cm, po)
    og = oracle.OracleGraph(g, omega, coupling=cm, present_only=po)
    rp, col, w, raw, twom = og.csr()
    A = D.supra_adjacency(g, cp)
    dense = [[F(0)] * g.n_supra for _ in range(g.n_supra)]
    for v in range(g.n_supra):
        for e in range(rp[v], rp[v + 1]):
            dense[v][col[e]] = F(int(w[e]), omega.denominator)
    assert dense == A
    ctot = og.coupling_total()
    assert omega * ctot == D.two_mu(g, cp) - sum(int(x) for x in twom)
    gam = [F(rng.randint(1, 4), rng.randint(1, 3)) for _ in range(T)]
    for _ in range(4):
        m = np.array([rng.randrange(g.n_supra) for _ in range(g.n_supra)], dtype=np.int32)
        c0 = og.q_components(m)
        assert oracle.q_from_components(c0, n, T, gam, omega, ctot) == \
            D.q_quadruple_sum(g, gam, cp, m)
        c2 = og.q_components(m, null_model=2)
        assert oracle.q_cpm_from_components(c2, n, T, gam, omega, ctot) == \
            D.q_quadruple_sum(g, gam, cp, m, cpm=True)
        c1 = og.q_components(m, null_model=1)
        assert oracle.q_global_from_components(c1, n, T, gam[0], omega, ctot) == \
            D.q_global_pair_sum(g, gam[0], cp, m)


@pytest.mark.parametrize("chunk", range(6))
def test_c_oracle_equals_literal_schedule_under_general_coupling(chunk):
    for seed in range(chunk * 30, chunk * 30 + 30):
        assert coupling_differences(seed) == [], f"case {seed}"


def test_c_oracle_equals_literal_schedule_under_general_coupling_larger():
    for seed in range(30_000, 30_024):
        assert coupling_differences(seed, max_nodes=10) == [], f"case {seed}"


COUPLING_MUTATIONS = [
    ("present-only check dropped", "if (c && g->present_only &&", "if (c && 0 &&"),
    ("multiplier ignored in the weights",
     "L->w[k] = e[k].inter ? a * (int64_t)e[k].raw : b * (int64_t)e[k].raw;",
     "L->w[k] = e[k].inter ? a : b * (int64_t)e[k].raw;"),
    ("coupling pairs one way only", "for (int32_t r = s + 1; r < T; r++)",
     "for (int32_t r = s + 1; r < T && r == s + 1; r++)"),
    ("absent copies keep CPM weight", "return !G->present_only || G->present[v];", "return 1;"),
]


@pytest.mark.parametrize("what,old,new", COUPLING_MUTATIONS, ids=[m[0] for m in COUPLING_MUTATIONS])
def test_planted_coupling_mistake_is_caught(tmp_path, what, old, new):
    src = open(os.path.join(ROOT, "oracle", "mslm_oracle.c")).read()
    assert src.count(old) == 1, what
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-o", str(lib), str(path)])
    code = ("import sys; sys.path.insert(0, %r); sys.path.insert(0, %r); "
            "import test_oracle_coupling as t; print(t.first_caught_coupling(range(300)))"
            % (ROOT, os.path.join(ROOT, "tests")))
    env = dict(os.environ, MSLM_ORACLE_LIB=str(lib), OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=600)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() != "None", f"planted mistake not caught: {what}"


# --------------------------------------------------------------------------- reductions

def _same(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


@pytest.mark.parametrize("nm", [0, 1, 2])
def test_ordinal_matrix_is_the_default(nm):
    g = gen.dcsbm(80, 4, 4, 6, 0.3, 2.5, 0.05, weights_max=2, seed=3)
    ordinal = [[1 if abs(s - r) == 1 else 0 for r in range(4)] for s in range(4)]
    gamma = F(1) if nm != 2 else F(1, 8)
    a = oracle.OracleGraph(g, F(1, 2)).leiden(gamma, null_model=nm)
    b = oracle.OracleGraph(g, F(1, 2), coupling=ordinal).leiden(gamma, null_model=nm)
    assert _same(a, b)


def test_present_only_with_every_copy_present_is_the_default():
    g = gen.erdos_renyi(40, 3, 0.3, seed=4)
    assert all(all(row) for row in D.presence(g))
    for nm, gamma in ((0, F(1)), (2, F(1, 8))):
        a = oracle.OracleGraph(g, 1).leiden(gamma, null_model=nm)
        b = oracle.OracleGraph(g, 1, present_only=True).leiden(gamma, null_model=nm)
        assert _same(a, b)


def test_categorical_at_two_slices_is_ordinal():
    g = gen.dcsbm(70, 2, 4, 6, 0.3, 2.5, 0.05, seed=5)
    a = oracle.OracleGraph(g, F(2)).leiden(F(1))
    b = oracle.OracleGraph(g, F(2), coupling=[[0, 1], [1, 0]]).leiden(F(1))
    assert _same(a, b)


def test_invalid_couplings_rejected():
    g = gen.erdos_renyi(4, 3, 0.5, seed=1)
    for cm in ([[0, 1, 0], [2, 0, 1], [0, 1, 0]],      # not symmetric
               [[1, 1, 0], [1, 0, 1], [0, 1, 0]],      # diagonal
               [[0, -1, 0], [-1, 0, 1], [0, 1, 0]]):   # negative
        with pytest.raises(ValueError):
            oracle.OracleGraph(g, 1, coupling=cm)


# --------------------------------------------------------------------------- optimum, invariants

@pytest.mark.parametrize("seed", range(12))
def test_general_coupling_tiny_random_below_optimum_connected_node_optimal(seed):
    rng = random.Random(1200 + seed)
    g = _with_absent_copies(seed, n=3, t=3)
    omega = F(rng.randint(1, 3), rng.randint(1, 2))
    cm = random_matrix(rng, 3)
    po = seed % 2 == 0
    cp = D.Coupling(omega, cm, po)
    nm = [0, 2][(seed // 2) % 2]
    gamma = F(1) if nm == 0 else F(1, 4)
    best, _ = D.brute_force_max(g, gamma, cp, cpm=nm == 2)
    og = oracle.OracleGraph(g, omega, coupling=cm, present_only=po)
    m, comps, _ = og.leiden(gamma, max_iterations=0, null_model=nm)
    q = D.q_quadruple_sum(g, gamma, cp, m, cpm=nm == 2)
    assert q <= best
    assert D.communities_connected(g, cp, m)
    assert D.improving_single_moves(g, gamma, cp, m, cpm=nm == 2) == []


def test_named_categorical_case_reaches_brute_force_optimum():
    """Two triangles over three slices with categorical coupling: the optimum keeps each
    triangle together across the slices."""
    tri = [(0, 1), (1, 2), (0, 2)]
    g = gen.from_edge_lists(3, [tri, tri, [(0, 1)]])
    cat = [[0, 1, 1], [1, 0, 1], [1, 1, 0]]
    best, _ = D.brute_force_max(g, F(1), D.Coupling(F(1, 2), cat))
    m, comps, _ = oracle.OracleGraph(g, F(1, 2), coupling=cat).leiden(F(1), max_iterations=0)
    assert D.q_quadruple_sum(g, F(1), D.Coupling(F(1, 2), cat), m) == best
