"""C-ABI checks that need no GPU: the library loads, exports every declared symbol,
rejects malformed input on the host before touching the device, and its host-side exact
reduction of Q agrees with rational arithmetic."""
import os
import random
import re
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from paper_2608_03695_amd import gen, mslm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "mslm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mslm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = mslm.load()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(mslm.EXPORTED)


@pytest.mark.parametrize("bad,code", [
    (lambda: gen.from_edge_lists(3, [[(0, 3)]]), mslm.MSLM_EINVAL),
    (lambda: gen.from_edge_lists(3, [[(-1, 2)]]), mslm.MSLM_EINVAL),
    (lambda: gen.from_edge_lists(3, [[(1, 1)]]), mslm.MSLM_EINVAL),
    (lambda: gen.from_edge_lists(3, [[(0, 1, 0)]], weighted=True), mslm.MSLM_EINVAL),
    (lambda: gen.from_edge_lists(3, [[(0, 1, -4)]], weighted=True), mslm.MSLM_EINVAL),
    (lambda: gen.from_edge_lists(2, [[]] * 65), mslm.MSLM_EUNSUPPORTED),
])
def test_create_rejects_bad_graphs_on_host(bad, code):
    with pytest.raises(mslm.MslmError) as ei:
        mslm.Graph(bad(), 1)
    assert ei.value.status == code


@pytest.mark.parametrize("omega,code", [(F(-1), mslm.MSLM_EINVAL), (F(1, 2 ** 31), mslm.MSLM_EOVERFLOW)])
def test_create_rejects_bad_coupling(omega, code):
    g = gen.from_edge_lists(3, [[(0, 1)]])
    with pytest.raises(mslm.MslmError) as ei:
        mslm.Graph(g, omega)
    assert ei.value.status == code


def test_null_arguments_rejected():
    lib = mslm.load()
    import ctypes as C
    assert lib.mslm_create(None, None, C.byref(C.c_void_p())) == mslm.MSLM_EINVAL
    p, _ = mslm.params()
    assert lib.mslm_leiden(None, C.byref(p), None, None) == mslm.MSLM_EINVAL
    lib.mslm_destroy(None)   # NULL-safe
    assert b"NULL" in lib.mslm_last_error() or lib.mslm_last_error()


@pytest.mark.parametrize("seed", range(20))
def test_exact_q_reduction_matches_rationals(seed):
    rng = random.Random(seed)
    T = rng.randint(1, 64)
    N = rng.randint(1, 10 ** 6)
    comps = np.zeros(3 * T + 1, np.int64)
    for s in range(T):
        tm = rng.choice([0, rng.randint(1, 2 ** 31 - 1)])
        comps[2 * T + s] = tm
        comps[s] = rng.randint(0, tm) if tm else 0
        comps[T + s] = rng.randint(0, tm * tm) if tm else 0
    comps[3 * T] = 2 * rng.randint(0, N * (T - 1))
    gamma = F(rng.randint(0, 2 ** 31 - 1), rng.randint(1, 2 ** 31 - 1))
    omega = F(rng.randint(0, 2 ** 31 - 1), rng.randint(1, 2 ** 31 - 1))
    want = oracle.q_from_components(comps, N, T, gamma, omega)
    assert mslm.q_exact(comps, T, N, gamma, omega) == want


def test_exact_q_of_the_hand_example():
    comps = np.array([2, 2, 4, 4, 2, 2, 4], dtype=np.int64)   # one community, H2
    assert mslm.q_exact(comps, 2, 2, 1, 1) == F(1, 2)


def test_footprint_grows_with_the_graph():
    small = mslm.footprint_bytes(gen.erdos_renyi(100, 2, 0.05, seed=1))
    large = mslm.footprint_bytes(gen.erdos_renyi(400, 4, 0.05, seed=1))
    assert 0 < small < large


@pytest.mark.parametrize("seed", range(20))
def test_exact_global_q_reduction_matches_rationals(seed):
    """The library's reduction of the global null model's components (SS' in the first SS
    slot) against the oracle's rational formula, inside the documented head-room:
    2mu' < 2^31 and max(p, q) * 2mu'^2 < 2^62."""
    rng = random.Random(500 + seed)
    T = rng.randint(1, 64)
    N = rng.randint(1, 10 ** 4)
    omega = F(rng.randint(0, 50), rng.randint(1, 50))
    a, b = omega.numerator, omega.denominator
    budget = (2 ** 31 - 1 - 2 * a * N * (T - 1)) // b
    if budget < T:
        omega, a, b = F(0), 0, 1
        budget = 2 ** 31 - 1
    comps = np.zeros(3 * T + 1, np.int64)
    for s in range(T):
        tm = rng.choice([0, rng.randint(1, max(1, budget // T))])
        comps[2 * T + s] = tm
        comps[s] = rng.randint(0, tm) if tm else 0
    comps[3 * T] = 2 * rng.randint(0, N * (T - 1))
    two_mu = b * int(comps[2 * T:3 * T].sum()) + 2 * a * N * (T - 1)
    assert two_mu < 2 ** 31
    comps[T] = rng.randint(0, two_mu * two_mu)
    lim = (2 ** 62 - 1) // max(1, two_mu * two_mu)
    gamma = F(rng.randint(0, min(lim, 2 ** 31 - 1)), rng.randint(1, min(lim, 2 ** 31 - 1)))
    want = oracle.q_global_from_components(comps, N, T, gamma, omega)
    assert mslm.q_exact_global(comps, T, N, gamma, omega) == want


def test_exact_global_q_of_the_hand_example():
    """N=2, T=2, edge 0-1 in both slices, omega = gamma = 1.  One community: W' = 4 + I = 8
    (I = 4 ordered coupled pairs), 2mu' = 8, SS' = 8^2, Q_G = 0.  By node ({0,2},{1,3}): no
    intra weight inside, I = 4, SS' = 2 * 4^2, Q_G = (8*4 - 32)/64 = 0.  Singletons:
    SS' = 4 * 2^2, Q_G = -16/64."""
    assert mslm.q_exact_global(np.array([2, 2, 64, 0, 2, 2, 4]), 2, 2, 1, 1) == 0
    assert mslm.q_exact_global(np.array([0, 0, 32, 0, 2, 2, 4]), 2, 2, 1, 1) == 0
    assert mslm.q_exact_global(np.array([0, 0, 16, 0, 2, 2, 0]), 2, 2, 1, 1) == F(-1, 4)


@pytest.mark.parametrize("seed", range(20))
def test_exact_q_reduction_of_the_variants_matches_rationals(seed):
    """The library's reduction with a resolution per slice, for Eq. 6 and for the multislice
    CPM (SS_s = squared community sizes), against the oracle's rational formulas."""
    rng = random.Random(900 + seed)
    T = rng.randint(1, 64)
    N = rng.randint(1, 10 ** 6)
    comps = np.zeros(3 * T + 1, np.int64)
    for s in range(T):
        tm = rng.choice([0, rng.randint(1, 2 ** 31 - 1)])
        comps[2 * T + s] = tm
        comps[s] = rng.randint(0, tm) if tm else 0
        comps[T + s] = rng.randint(0, tm * tm) if tm else 0
    comps[3 * T] = 2 * rng.randint(0, N * (T - 1))
    gs = [F(rng.randint(1, 2 ** 31 - 1), rng.randint(1, 2 ** 31 - 1)) for _ in range(T)]
    omega = F(rng.randint(0, 2 ** 31 - 1), rng.randint(1, 2 ** 31 - 1))
    assert mslm.q_exact_variant(comps, T, N, 1, omega, mslm.MSLM_NULL_MULTISLICE, gs) == \
        oracle.q_from_components(comps, N, T, gs, omega)
    assert mslm.q_exact_variant(comps, T, N, 1, omega, mslm.MSLM_NULL_CPM, gs) == \
        oracle.q_cpm_from_components(comps, N, T, gs, omega)
    # one resolution: the same as mslm_q_exact
    assert mslm.q_exact_variant(comps, T, N, gs[0], omega) == mslm.q_exact(comps, T, N, gs[0], omega)


def test_exact_q_variant_refuses_bad_arguments():
    comps = np.zeros(7, np.int64)
    with pytest.raises(mslm.MslmError) as e:
        mslm.q_exact_variant(comps, 2, 2, 1, 1, mslm.MSLM_NULL_GLOBAL, [F(1), F(2)])
    assert e.value.status == mslm.MSLM_EINVAL
    with pytest.raises(mslm.MslmError) as e:
        mslm.q_exact_variant(comps, 2, 2, 1, 1, 7)
    assert e.value.status == mslm.MSLM_EINVAL
