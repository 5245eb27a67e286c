"""The Bethe-Hessian spectral pathway, plainly (test infrastructure only).

This file belongs to the oracle: only tests, the smoke check and the benchmark's CPU baseline
may use it.  It shares no code with the HIP path.  Section 3.1 (the paragraphs after Eq. 4):

* The supra-graph of Eq. 3 with adjacency A (intra weights on the diagonal blocks, coupling
  omega^(sr) between the copies of a node) and degree matrix D = diag(A 1).
* The Bethe-Hessian H(r) = (r^2 - 1) I - r A + D (Saade et al.), symmetric; its informative
  (most negative) eigenvectors embed the supra-nodes.  r defaults to sqrt(<d^2>/<d> - 1), the
  degree-corrected form of r ~ sqrt(c) for an average degree c (the paper's refinement for
  degree heterogeneity).
* The k eigenvectors of the k algebraically smallest eigenvalues, by scipy's symmetric sparse
  eigensolver (ARPACK) in float64: a library routine used as one step.
* k-means on the rows of that embedding (n points in R^k), deterministic: maximin (farthest
  point) initialisation starting from point 0, then Lloyd iterations until no assignment
  changes or the iteration cap.  Distances are sums over the coordinates in index order of
  squared differences, each product and sum rounded separately (no fused multiply-add); ties
  go to the lowest centroid (assignment) and the lowest point index (initialisation).  Centroid
  sums are exact: every coordinate is first rounded to a fixed-point integer (scale 2^40) and
  the integer sums are converted once, so their value does not depend on summation order.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

FIX_SHIFT = 40


def supra_coo(g, omega, coupling=None, present_only=False):
    """Entries (row, col, weight) of the supra-adjacency as float64 arrays: both directions of
    every intra edge (repeated pairs summed), and omega * c_sr between (i,s) and (i,r)
    (c: T x T integers, ordinal when None; with present_only only between copies that have an
    edge in their slices)."""
    n, T = g.n_nodes, g.n_slices
    rows, cols, vals = [], [], []
    present = np.zeros((T, n), bool)
    for s in range(T):
        u, x, w = g.slice_edges(s)
        ww = np.ones(u.size) if w is None else w.astype(np.float64)
        rows += [s * n + u, s * n + x]
        cols += [s * n + x, s * n + u]
        vals += [ww, ww]
        present[s, u] = True
        present[s, x] = True
    om = float(Fraction(omega))
    if om != 0.0:
        for s in range(T):
            for r in range(T):
                c = (1 if abs(s - r) == 1 else 0) if coupling is None else int(coupling[s][r])
                if s != r and c:
                    i = np.arange(n)
                    if present_only:
                        i = i[present[s] & present[r]]
                    rows.append(s * n + i)
                    cols.append(r * n + i)
                    vals.append(np.full(i.size, om * c))
    if not rows:
        z = np.zeros(0, np.int64)
        return z, z, np.zeros(0)
    return (np.concatenate(rows).astype(np.int64), np.concatenate(cols).astype(np.int64),
            np.concatenate(vals))


def adjacency(g, omega, coupling=None, present_only=False):
    import scipy.sparse as sp
    r, c, v = supra_coo(g, omega, coupling, present_only)
    N = g.n_supra
    return sp.csr_matrix((v, (r, c)), shape=(N, N))   # duplicates are summed


def default_r(A):
    """sqrt(<d^2>/<d> - 1) of the weighted degrees d (1 when that is not above 1)."""
    d = np.asarray(A.sum(axis=1)).ravel()
    s1 = d.sum()
    if s1 <= 0:
        return 1.0
    x = float((d * d).sum() / s1 - 1.0)
    return float(np.sqrt(x)) if x > 1.0 else 1.0


def bethe_hessian(A, r):
    """H(r) = (r^2 - 1) I - r A + D as a sparse matrix."""
    import scipy.sparse as sp
    d = np.asarray(A.sum(axis=1)).ravel()
    N = A.shape[0]
    return ((r * r - 1.0) * sp.identity(N, format="csr") - r * A + sp.diags(d)).tocsr()


def smallest_eigenpairs(H, k):
    """The k algebraically smallest eigenvalues (ascending) and their eigenvectors (columns)."""
    import scipy.sparse.linalg as sla
    N = H.shape[0]
    if N <= max(2 * k + 1, 64):
        w, V = np.linalg.eigh(H.toarray())
        return w[:k], V[:, :k]
    w, V = sla.eigsh(H, k=k, which="SA", tol=1e-12, ncv=min(N, max(4 * k, k + 40)))
    order = np.argsort(w)
    return w[order], V[:, order]


# --------------------------------------------------------------------------- k-means

def _sqdist(P, c):
    """sum_j (P[:, j] - c[j])^2 in index order, each operation rounded on its own."""
    d = np.zeros(P.shape[0])
    for j in range(P.shape[1]):
        t = P[:, j] - c[j]
        d = d + t * t
    return d


def to_fixed(P):
    return np.rint(np.ldexp(P, FIX_SHIFT)).astype(np.int64)


def kmeans(P, k, max_iter=100):
    """Deterministic k-means of the rows of P (n x dim, float64): returns (labels int32,
    centroids k x dim, iterations run).  k <= n."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    n, dim = P.shape
    Q = to_fixed(P)                      # exact per-coordinate integers
    C = np.zeros((k, dim))
    C[0] = P[0]
    near = _sqdist(P, C[0])
    for c in range(1, k):
        i = int(np.argmax(near))          # first index of the largest distance
        C[c] = P[i]
        near = np.minimum(near, _sqdist(P, C[c]))
    labels = np.full(n, -1, np.int32)
    it = 0
    for it in range(1, max_iter + 1):
        best = np.full(n, np.inf)
        lab = np.zeros(n, np.int32)
        for c in range(k):
            d = _sqdist(P, C[c])
            better = d < best                # strict: ties stay with the lower centroid
            best[better] = d[better]
            lab[better] = c
        changed = not np.array_equal(lab, labels)
        labels = lab
        for c in range(k):
            mask = labels == c
            cnt = int(mask.sum())
            if cnt == 0:
                continue                     # an empty cluster keeps its centroid
            sums = [int(v) for v in Q[mask].astype(object).sum(axis=0)]   # exact
            C[c] = np.array([np.ldexp(float(s) / cnt, -FIX_SHIFT) for s in sums])
        if not changed:
            break
    return labels, C, it


def spectral_communities(g, omega, k, r=None, coupling=None, max_iter=100):
    """The pathway end to end: (labels, eigenvalues, embedding, r)."""
    A = adjacency(g, omega, coupling)
    rr = default_r(A) if r is None else float(r)
    H = bethe_hessian(A, rr)
    w, V = smallest_eigenpairs(H, k)
    labels, _, _ = kmeans(V, k, max_iter)
    return labels, w, V, rr
