"""Pins of the oracle's Bethe-Hessian pathway (Section 3.1, after Eq. 4):

* H(1) is the graph Laplacian D - A; H(r) is symmetric; its supra-adjacency is Eq. 3's.
* Ihara-Bass: every real eigenvalue lambda (|lambda| != 1) of the non-backtracking matrix B of
  an unweighted graph makes H(lambda) singular, the relation that maps B's informative
  eigenvalues to H's negative ones.
* The default r of a d-regular graph is sqrt(d - 1) (the degree-corrected sqrt(c)).
* The sparse eigensolver step equals a dense eigendecomposition (a second library routine).
* k-means: a hand example, the maximin start, and Lloyd's fixed point (every point with its
  nearest centroid, ties to the lowest; every centroid the mean of its points).
* Planted recovery on a static SBM and on a strongly coupled temporal one (a sanity bar; the
  paper prints no number for it: **parity unpinned** for recovery quality).
"""
import numpy as np
import pytest
from fractions import Fraction as F

from oracle import definitional as D
from oracle import spectral as SP
from paper_2608_03695_amd import gen


def _nmi(a, b):
    from sklearn.metrics import normalized_mutual_info_score
    return normalized_mutual_info_score(a, b)


@pytest.mark.parametrize("seed", range(4))
def test_h_at_one_is_the_laplacian_and_adjacency_is_eq3(seed):
    g = gen.erdos_renyi(6, 3, 0.5, seed=seed, weights_max=3)
    omega = F(3, 2)
    A = SP.adjacency(g, omega).toarray()
    dense = np.array([[float(x) for x in row] for row in D.supra_adjacency(g, omega)])
    assert np.array_equal(A, dense)
    H1 = SP.bethe_hessian(SP.adjacency(g, omega), 1.0).toarray()
    assert np.array_equal(H1, np.diag(A.sum(axis=1)) - A)
    Hr = SP.bethe_hessian(SP.adjacency(g, omega), 2.5).toarray()
    assert np.array_equal(Hr, Hr.T)
    assert np.allclose(Hr, (2.5 ** 2 - 1) * np.eye(len(A)) - 2.5 * A + np.diag(A.sum(axis=1)))


def _nonbacktracking(edges, n):
    directed = [(u, v) for u, v in edges] + [(v, u) for u, v in edges]
    idx = {e: i for i, e in enumerate(directed)}
    B = np.zeros((len(directed), len(directed)))
    for (u, v), i in idx.items():
        for (x, w), j in idx.items():
            if x == v and w != u:
                B[i, j] = 1.0
    return B


@pytest.mark.parametrize("seed", range(4))
def test_ihara_bass_real_eigenvalues_of_b_make_h_singular(seed):
    rng = np.random.default_rng(seed)
    g = gen.erdos_renyi(7, 2, 0.5, seed=seed)          # unweighted, coupling weight 1
    A = SP.adjacency(g, 1).toarray()
    n = len(A)
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if A[u, v]]
    lam = np.linalg.eigvals(_nonbacktracking(edges, n))
    real = [x.real for x in lam if abs(x.imag) < 1e-9 and abs(abs(x.real) - 1) > 1e-3]
    assert real, "no real eigenvalue away from +-1"
    for x in real:
        H = (x * x - 1) * np.eye(n) - x * A + np.diag(A.sum(axis=1))
        smin = np.linalg.svd(H, compute_uv=False)[-1]
        assert smin < 1e-7 * max(1.0, x * x), (x, smin)
    # and a value that is no eigenvalue of B leaves H regular
    y = max(abs(v) for v in lam) + 0.5 + rng.random()
    H = (y * y - 1) * np.eye(n) - y * A + np.diag(A.sum(axis=1))
    assert np.linalg.svd(H, compute_uv=False)[-1] > 1e-6


def test_present_only_adjacency_equals_the_definitional_one():
    g = gen.with_absences(gen.erdos_renyi(5, 3, 0.6, seed=2), 0.3, seed=4)
    cm = [[0, 2, 1], [2, 0, 1], [1, 1, 0]]
    A = SP.adjacency(g, F(1, 2), cm, True).toarray()
    dense = np.array([[float(x) for x in row]
                      for row in D.supra_adjacency(g, D.Coupling(F(1, 2), cm, True))])
    assert np.array_equal(A, dense)


def test_default_r_of_a_regular_graph():
    # a ring of 12 nodes in every slice, T = 1: 2-regular, r = sqrt(1) -> 1; a 4-regular
    # circulant: r = sqrt(3)
    ring = [(i, (i + 1) % 12) for i in range(12)]
    circ = ring + [(i, (i + 2) % 12) for i in range(12)]
    g = gen.from_edge_lists(12, [circ])
    assert SP.default_r(SP.adjacency(g, 0)) == pytest.approx(np.sqrt(3.0), rel=1e-15)
    g2 = gen.from_edge_lists(12, [ring])
    assert SP.default_r(SP.adjacency(g2, 0)) == 1.0


@pytest.mark.parametrize("k", [2, 5])
def test_sparse_eigensolver_equals_dense(k):
    g = gen.planted_partition(150, 3, 4, 0.1, 0.01, 0.1, seed=3)
    A = SP.adjacency(g, F(1, 2))
    H = SP.bethe_hessian(A, SP.default_r(A))
    w, V = SP.smallest_eigenpairs(H, k)
    wd, Vd = np.linalg.eigh(H.toarray())
    assert np.allclose(w, wd[:k], rtol=0, atol=1e-9 * abs(wd).max())
    # the same subspace: singular values of V^T Vd are all 1
    s = np.linalg.svd(V.T @ Vd[:, :k], compute_uv=False)
    assert s.min() > 1 - 1e-8


def test_kmeans_hand_example():
    P = np.array([[0.0, 0.0], [0.0, 1.0], [10.0, 10.0], [10.0, 11.0], [0.5, 0.5]])
    labels, C, it = SP.kmeans(P, 2)
    assert list(labels) == [0, 0, 1, 1, 0]
    assert np.allclose(C[0], [0.5 / 3, 1.5 / 3], atol=1e-12) and np.allclose(C[1], [10, 10.5])
    # maximin start: point 0, then the point farthest from it (index 3)
    labels1, C1, _ = SP.kmeans(P, 2, max_iter=1)
    assert list(labels1) == [0, 0, 1, 1, 0]


@pytest.mark.parametrize("seed", range(4))
def test_kmeans_reaches_lloyds_fixed_point(seed):
    rng = np.random.default_rng(seed)
    P = rng.normal(size=(400, 3)) + np.repeat(rng.normal(scale=4, size=(4, 3)), 100, axis=0)
    labels, C, it = SP.kmeans(P, 4, max_iter=200)
    assert it < 200
    d = np.stack([SP._sqdist(P, C[c]) for c in range(4)], axis=1)
    assert np.array_equal(labels, np.argmin(d, axis=1))        # nearest, ties to the lowest
    for c in range(4):
        m = P[labels == c].mean(axis=0)
        assert np.allclose(C[c], m, rtol=0, atol=2.0 ** -38)


@pytest.mark.parametrize("T,omega", [(1, 0), (4, 3)])
def test_planted_sbm_is_recovered(T, omega):
    """A static SBM, and a temporal one whose communities persist under strong coupling (with
    weak coupling each slice's communities give their own informative eigenvectors, so k
    eigenvectors do not separate k communities)."""
    g = gen.planted_partition(600, T, 4, 0.06, 0.003, 0.0, seed=5)
    labels, w, V, r = SP.spectral_communities(g, omega, 4)
    assert w[0] < 0 and r > 1
    assert _nmi(labels, g.planted.ravel()) > 0.95
