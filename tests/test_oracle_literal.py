"""The C schedule oracle against the literal statement of the schedule (oracle/schedule.py).

The literal tier takes every local-moving and refinement decision on the exact change of Q_MS
(Eq. 6) of the level-0 partition the decision would produce, keeps aggregated units as sets of
level-0 supra-nodes and recomputes every refined sub-community's edge weight and
well-connectedness from scratch.  The C oracle instead decides on scaled integer gains over an
aggregated graph with slice profiles, Sigma tables and running counters.  Equality of the two
per level (colouring, labels after local moving, refinement) and at the end (membership and
every statistic) pins the C oracle's tie rule, strictness rule, empty-community rule and fresh
labels, its refinement eligibility rules and its bookkeeping.  The mutation cases show the
comparison has teeth: each plants one plausible mistake in a copy of the C oracle (on the
CPU) and expects the comparison to catch it.
"""
import os
import random
import subprocess
import sys
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from oracle import schedule as S
from paper_2608_03695_amd import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def random_case(seed, max_nodes=6):
    rng = random.Random(seed)
    n, t = rng.randint(2, max_nodes), rng.randint(1, 4)
    g = gen.erdos_renyi(n, t, rng.uniform(0.25, 0.8), seed=rng.randrange(1 << 30),
                        weights_max=rng.choice([1, 1, 3]))
    omega = rng.choice([F(0), F(1, 2), F(1), F(2), F(3, 2), F(1, 10)])
    gamma = rng.choice([F(1, 2), F(1), F(3, 2), F(2)])
    levels = rng.choice([32, 32, 1, 2, 3])
    iters = rng.choice([1, 2, 2, 0])
    sweeps = rng.choice([0, 0, 0, 1, 2])
    return g, omega, gamma, levels, iters, sweeps, rng.randrange(1 << 20)


def run_both(seed, max_nodes=6):
    g, omega, gamma, lv, it, sw, sd = random_case(seed, max_nodes)
    m1, st1, tr1 = S.leiden(g, gamma, omega, lv, it, sw, sd)
    og = oracle.OracleGraph(g, omega)
    oracle.trace_enable(True)
    try:
        m2, _, st2 = og.leiden(gamma, lv, it, sw, sd)
        tr2 = oracle.trace_levels(g.n_supra)
    finally:
        oracle.trace_enable(False)
    return (g, omega, gamma), (m1, st1, tr1), (m2, {k: int(v) for k, v in st2.items()}, tr2)


def differences(seed, max_nodes=6):
    _, (m1, st1, tr1), (m2, st2, tr2) = run_both(seed, max_nodes)
    diffs = []
    if list(m2) != m1:
        diffs.append("membership")
    diffs += [k for k in st1 if st1[k] != st2[k]]
    if len(tr1) != len(tr2):
        return diffs + ["levels"]
    for a, b in zip(tr1, tr2):
        where = f"@it{a['it']}/lvl{a['lvl']}"
        for k in ("colour", "p_in", "p_lm"):
            if a[k] != [int(x) for x in b[k]]:
                diffs.append(k + where)
        ra, rb = a.get("r"), b["r"]
        if (ra is None) != (rb is None) or (ra is not None and ra != [int(x) for x in rb]):
            diffs.append("r" + where)
    return diffs


def bookkeeping_errors(seed):
    """Founders whose C running edge weight or well-connectedness flag differs from the
    value recomputed from the definition (the C weights are scaled by the coupling
    denominator b)."""
    (g, omega, gamma), (_, _, tr1), (_, _, tr2) = run_both(seed)
    b = omega.denominator
    errs = []
    for a, rec in zip(tr1, tr2):
        if rec["r"] is None or "subs" not in a:
            continue
        for T, (_, ext, wc) in a["subs"].items():
            if rec["ext"][T] != ext * b or bool(rec["wc"][T]) != wc:
                errs.append((a["it"], a["lvl"], T))
    return errs


def first_caught(seeds):
    """The first case whose C run differs from the literal schedule in any way."""
    for s in seeds:
        if differences(s) or bookkeeping_errors(s):
            return s
    return None


@pytest.mark.parametrize("chunk", range(8))
def test_c_oracle_equals_literal_schedule(chunk):
    for seed in range(chunk * 30, chunk * 30 + 30):
        assert differences(seed) == [], f"case {seed}"


@pytest.mark.parametrize("chunk", range(2))
def test_c_oracle_equals_literal_schedule_larger(chunk):
    for seed in range(10_000 + chunk * 20, 10_000 + chunk * 20 + 20):
        assert differences(seed, max_nodes=12) == [], f"case {seed}"


def test_refinement_bookkeeping_equals_definition():
    """The C oracle's running edge weight of each refined sub-community to the rest of its
    community, and its well-connectedness flag, equal the values recomputed from the
    definition."""
    checked = 0
    for seed in range(200):
        assert bookkeeping_errors(seed) == [], f"case {seed}"
        _, (_, _, tr1), _ = run_both(seed)
        checked += sum(len(a.get("subs", {})) for a in tr1)
    assert checked > 500


def test_literal_score_is_eq6():
    from oracle import definitional as D
    rng = random.Random(7)
    for _ in range(30):
        g, omega, gamma, *_ = random_case(rng.randrange(1 << 30))
        G = S.SupraGraph(g, omega)
        sc = S.Score(G, gamma)
        for _ in range(3):
            memb = [rng.randrange(G.n) for _ in range(G.n)]
            assert sc.q(memb) == D.q_quadruple_sum(g, gamma, omega, np.array(memb))


def test_literal_hash_is_published_splitmix64():
    import json
    spec = json.load(open(os.path.join(ROOT, "tests", "golden", "splitmix64.json")))
    inc = int(spec["gamma_increment"], 16)
    state = 0
    for want in spec["seed0_outputs"]:
        state = (state + inc) % (1 << 64)
        assert S.splitmix64_mix(state) == int(want, 16)


# one plausible mistake per case: (what, text in mslm_oracle.c, replacement)
MUTATIONS = [
    ("ties to the highest label", "if (c > 0 || (c == 0 && best_empty))", "if (c >= 0)"),
    ("move on a tie with staying", "if (gval_cmp(&best, &gD) > 0) {", "if (gval_cmp(&best, &gD) >= 0) {"),
    ("fresh label off by a sweep", "(uint64_t)n * (1 + t) + (uint64_t)v", "(uint64_t)n * (2 + t) + (uint64_t)v"),
    ("no rule (a)", "if (prop[T] == NONE_LABEL) { elig[v] = 1; any = 1; continue; }",
     "if (prop[T] == NONE_LABEL) continue;"),
    ("rule (b) without the founder check", "if (prop[prop[T]] == NONE_LABEL) continue;", ""),
    ("rule (b) outranked by lower priority", "if (pri[u] > pri[v] || (pri[u] == pri[v] && u > v)) ok = 0;",
     "if (pri[u] < pri[v] || (pri[u] == pri[v] && u < v)) ok = 0;"),
    ("no co-joiner correction", "ext[T] += ext[v] - 2 * propw[v] - corr;", "ext[T] += ext[v] - 2 * propw[v];"),
    ("empty community wins ties", "if (c > 0 || (c == 0 && best_empty))", "if (c > 0)"),
    ("refinement candidates outside the community", "int64_t nc = gather(g, v, R, P, P[v], buf);",
     "int64_t nc = gather(g, v, R, NULL, 0, buf);"),
    ("strict well-connectedness", "return gval_sign(&g) >= 0;", "return gval_sign(&g) > 0;"),
]


@pytest.mark.parametrize("what,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_oracle_mistake_is_caught(tmp_path, what, old, new):
    src = open(os.path.join(ROOT, "oracle", "mslm_oracle.c")).read()
    assert src.count(old) == 1, what
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-o", str(lib), str(path)])
    code = ("import sys; sys.path.insert(0, %r); sys.path.insert(0, %r); "
            "import test_oracle_literal as t; print(t.first_caught(range(600)))"
            % (ROOT, os.path.join(ROOT, "tests")))
    env = dict(os.environ, MSLM_ORACLE_LIB=str(lib), OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=600)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() != "None", f"planted mistake not caught: {what}"
