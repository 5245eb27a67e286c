"""GPU parity of the Bethe-Hessian pathway (Section 3.1) against the oracle's (oracle/spectral.py):

* the operator H(r) x against the oracle's sparse H(r) @ x, to float64 rounding;
* the k-means entry on seeded synthetic points: labels, centroids and iteration counts bit for
  bit (both sides take every decision in float64 on the same values, and the centroid sums are
  exact);
* the k smallest eigenpairs against scipy's symmetric eigensolver: eigenvalues to 1e-8 of the
  spectral scale, residuals, the same invariant subspace (principal angles), H(1) = Laplacian;
* the whole pathway's labels against the oracle's (up to relabelling) on planted graphs.
"""
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import spectral as SP
from paper_2608_03695_amd import gen

pytestmark = pytest.mark.gpu


def _mslm():
    from paper_2608_03695_amd import mslm
    return mslm


GRAPHS = [
    ("planted_static", lambda: gen.planted_partition(800, 1, 4, 0.06, 0.003, 0.0, seed=5), F(0), None, False),
    ("planted_T4_strong", lambda: gen.planted_partition(600, 4, 4, 0.06, 0.003, 0.0, seed=5), F(3), None, False),
    ("dcsbm_weighted", lambda: gen.dcsbm(2000, 4, 8, 6, 0.2, 2.5, 0.02, weights_max=4, seed=8), F(1), None, False),
    ("categorical_absent", lambda: gen.with_absences(gen.dcsbm(1500, 4, 10, 5, 0.2, 2.5, 0.02, seed=9), 0.2, seed=1),
     F(1, 2), [[0, 1, 1, 1], [1, 0, 1, 1], [1, 1, 0, 1], [1, 1, 1, 0]], True),
]
IDS = [g[0] for g in GRAPHS]


def _handle(tg, omega, cm, po):
    return _mslm().Graph(tg, omega, coupling=cm, present_only=po)


def _oracle_H(tg, omega, cm, po, r):
    A = SP.adjacency(tg, omega, cm, po)
    rr = SP.default_r(A) if r is None else r
    return SP.bethe_hessian(A, rr), rr


@pytest.mark.parametrize("name,make,omega,cm,po", GRAPHS, ids=IDS)
def test_operator_matches_oracle(name, make, omega, cm, po):
    tg = make()
    g = _handle(tg, omega, cm, po)
    rng = np.random.default_rng(7)
    for r in (1.0, 2.75):
        H, _ = _oracle_H(tg, omega, cm, po, r)
        x = rng.standard_normal(tg.n_supra)
        y = g.bh_apply(x, r)
        want = H @ x
        scale = abs(H).max() * np.abs(x).max() * 64
        assert np.max(np.abs(y - want)) <= 1e-14 * scale, name
    g.close()


@pytest.mark.parametrize("n,dim,k,seed", [(5000, 3, 4, 1), (20000, 8, 8, 2), (3000, 16, 12, 3),
                                          (40000, 5, 6, 4)])
def test_kmeans_entry_bit_exact(n, dim, k, seed):
    mslm = _mslm()
    rng = np.random.default_rng(seed)
    centres = rng.normal(scale=3.0, size=(k, dim))
    P = centres[rng.integers(0, k, n)] + rng.normal(size=(n, dim))
    lab, cen, it = mslm.kmeans(P, k, max_iterations=200)
    olab, ocen, oit = SP.kmeans(P, k, max_iter=200)
    assert np.array_equal(lab, olab)
    assert np.array_equal(cen.view(np.int64), ocen.view(np.int64))   # bitwise
    assert it == oit


@pytest.mark.parametrize("name,make,omega,cm,po", GRAPHS, ids=IDS)
def test_eigenpairs_match_oracle(name, make, omega, cm, po):
    tg = make()
    k = 6
    g = _handle(tg, omega, cm, po)
    ev, Y, _, res = g.bethe_hessian(k, lanczos_steps=160, labels=False)
    g.close()
    H, r = _oracle_H(tg, omega, cm, po, None)
    assert res["r"] == pytest.approx(r, rel=1e-12)
    w, V = SP.smallest_eigenpairs(H, k + 1)
    scale = abs(H).sum(axis=1).max()   # a bound of the spectral radius
    assert np.max(np.abs(ev - w[:k])) <= 1e-8 * scale, (ev, w)
    assert res["residual_max"] <= 1e-7 * scale
    # the same invariant subspace where the k-th eigenvalue is separated from the next
    if w[k] - w[k - 1] > 1e-6 * scale:
        s = np.linalg.svd(Y.T @ V[:, :k], compute_uv=False)
        assert s.min() > 1 - 1e-6
    assert np.allclose(Y.T @ Y, np.eye(k), atol=1e-8)
    assert res["tridiagonal_steps"] > 0
    assert 0 <= res["second_passes"] <= res["lanczos_steps"]


def test_full_krylov_space_takes_second_passes():
    """Lanczos run to (nearly) the whole space: late vectors lose most of their norm to the
    projection, so the second Gram-Schmidt pass is taken, and the eigenpairs still equal a
    dense eigensolver's."""
    tg = gen.planted_partition(40, 2, 2, 0.3, 0.05, 0.0, seed=3)
    n = tg.n_supra
    g = _handle(tg, F(1), None, False)
    ev, Y, _, res = g.bethe_hessian(6, lanczos_steps=n, labels=False)
    g.close()
    H, _ = _oracle_H(tg, F(1), None, False, None)
    w = np.linalg.eigvalsh(H.toarray())
    scale = abs(H).sum(axis=1).max()
    assert res["second_passes"] > 0
    assert np.max(np.abs(ev - w[:6])) <= 1e-10 * scale, (ev, w[:6])
    assert res["residual_max"] <= 1e-9 * scale
    assert np.allclose(Y.T @ Y, np.eye(6), atol=1e-10)


def test_r_one_is_the_laplacian():
    tg = gen.planted_partition(500, 3, 4, 0.08, 0.004, 0.0, seed=2)
    g = _handle(tg, F(1), None, False)
    ev, Y, _, res = g.bethe_hessian(3, r=1.0, lanczos_steps=120, labels=False)
    g.close()
    assert res["r"] == 1.0
    assert abs(ev[0]) < 1e-9 * 100          # the Laplacian's zero eigenvalue (connected graph)
    L = SP.bethe_hessian(SP.adjacency(tg, F(1)), 1.0)
    w, _ = SP.smallest_eigenpairs(L, 3)
    assert np.max(np.abs(ev - w)) < 1e-8 * 100


@pytest.mark.parametrize("T,omega", [(1, F(0)), (4, F(3))])
def test_pathway_labels_match_oracle(T, omega):
    from sklearn.metrics import normalized_mutual_info_score as nmi
    tg = gen.planted_partition(600, T, 4, 0.06, 0.003, 0.0, seed=5)
    g = _handle(tg, omega, None, False)
    ev, Y, lab, res = g.bethe_hessian(4, lanczos_steps=120)
    g.close()
    olab, ow, _, _ = SP.spectral_communities(tg, omega, 4)
    assert nmi(lab, olab) > 0.99
    assert nmi(lab, tg.planted.ravel()) > 0.95


def test_invalid_spectral_arguments():
    mslm = _mslm()
    tg = gen.planted_partition(100, 2, 2, 0.1, 0.01, 0.0, seed=1)
    g = _handle(tg, F(1), None, False)
    for kw in (dict(k=0), dict(k=33), dict(k=4, lanczos_steps=3), dict(k=2, r=-1.0)):
        with pytest.raises(mslm.MslmError) as e:
            g.bethe_hessian(**kw)
        assert e.value.status == mslm.MSLM_EINVAL, kw
    with pytest.raises(mslm.MslmError):
        mslm.kmeans(np.zeros((3, 2)), 4)
    g.close()


@pytest.mark.parametrize("T,N,omega", [(1, 200, F(0)), (2, 100, F(1, 100))])
def test_path_laplacian_closed_form(T, N, omega):
    """H(1) = D - A of a path of N nodes has the eigenvalues 2 - 2 cos(pi k / N), k = 0..N-1;
    two copies of the path coupled node to node with weight omega add the coupling Laplacian's
    eigenvalues {0, 2 omega}.  With the Krylov space run to the whole space, the smallest eight
    must equal these closed forms (a pin of the operator, the Lanczos recurrence and the
    tridiagonal eigensolver that does not go through another eigensolver)."""
    path = [(i, i + 1) for i in range(N - 1)]
    tg = gen.from_edge_lists(N, [path] * T)
    g = _handle(tg, omega, None, False)
    n = N * T
    ev, _, _, res = g.bethe_hessian(8, r=1.0, lanczos_steps=n, labels=False)
    g.close()
    lam = 2.0 - 2.0 * np.cos(np.pi * np.arange(N) / N)
    want = np.sort(np.concatenate([lam + 2.0 * float(omega) * c for c in range(T)]))[:8]
    assert res["lanczos_steps"] <= n
    assert np.max(np.abs(ev - want)) < 1e-10, (ev, want)
