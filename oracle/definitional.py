"""Definitional multislice modularity in exact rational arithmetic (test infrastructure).

This file belongs to the oracle: only tests, the smoke check and the benchmark's CPU
baseline may use it.  Everything is written straight from the paper's definitions with
``fractions.Fraction`` and plain loops, for tiny inputs only.

* Supra-adjacency of Eq. 3 (Section 3.1): diagonal blocks A^(t), off-diagonal
  coupling omega*I between consecutive snapshots (ordinal coupling).
* Multislice modularity Q_MS of Eq. 6 (Section 3.2), evaluated three independent ways:
  the literal quadruple sum over (i, j, s, r); the trace form Tr(C^T M C) / 2mu of the
  supra-modularity matrix (Section 3.2, the paragraph after Eq. 6); and a per-slice
  component form (intra weight inside communities, sum of squared community degrees,
  coupled copies kept together).
* Static Newman modularity (Eq. 5, undirected, so d_out = d_in = k) for T = 1.
* Closed forms for the all-singleton and one-community partitions.
* Brute-force maximum over all set partitions of the supra-nodes (n <= 10).
* The variants Eq. 6 admits: a resolution gamma^(s) per slice (every function taking gamma
  accepts one value or a sequence of T), and the multislice CPM (cpm=True): the null term
  gamma^(s) k_i^s k_j^s / 2m^s replaced by gamma^(s) n_i n_j with node weight n = 1 per
  supra-node, under the same normalisation 1/2mu.

Readings where the paper is silent (all listed with the design notes):
* 2mu is the total weight of the supra-graph of Eq. 3: sum_s 2m_s + 2*omega*N*(T-1) for the
  ordinal coupling, sum_s 2m_s + sum of omega^(sr) over ordered coupled copy pairs in general.
* omega^(sr) = omega when |s - r| = 1 and 0 otherwise (ordinal coupling), omega^(ss) = 0.
  Every function taking omega also takes a Coupling: omega^(sr) = omega * c_sr for an integer
  matrix c, optionally only between copies present in both slices (a copy is present when it
  has an edge in its slice; under the CPM an absent copy then has node weight 0).
* A snapshot without edges (2m_s = 0) contributes no null-model term.
* Supra-node (i, s) has index s*N + i (slice-major).
"""
from __future__ import annotations

from fractions import Fraction
from itertools import product
from math import lcm

import numpy as np


# --------------------------------------------------------------------------- inputs

def slice_matrices(g):
    """Dense symmetric A^(s) (python ints) per slice; repeated pairs add their weights."""
    n, t = g.n_nodes, g.n_slices
    mats = []
    for s in range(t):
        a = [[0] * n for _ in range(n)]
        u, x, w = g.slice_edges(s)
        for e in range(u.size):
            i, j = int(u[e]), int(x[e])
            ww = 1 if w is None else int(w[e])
            a[i][j] += ww
            a[j][i] += ww
        mats.append(a)
    return mats


def coupling(s, r, omega):
    """Ordinal coupling omega^(sr)."""
    return Fraction(omega) if abs(s - r) == 1 else Fraction(0)


class Coupling:
    """omega^(sr) = omega * c_sr between the copies (i, s) and (i, r) (Eq. 6); c is a T x T
    integer matrix (None: the ordinal coupling, c_sr = 1 for |s - r| = 1); present_only: only
    between copies that have an edge in their slices."""

    def __init__(self, omega, matrix=None, present_only=False):
        self.omega = Fraction(omega)
        self.matrix = None if matrix is None else [[int(x) for x in row] for row in matrix]
        self.present_only = bool(present_only)

    def c(self, s, r):
        if s == r:
            return 0
        if self.matrix is None:
            return 1 if abs(s - r) == 1 else 0
        return self.matrix[s][r]


def as_coupling(omega):
    return omega if isinstance(omega, Coupling) else Coupling(omega)


def presence(g):
    """present[s][i]: the copy (i, s) has an edge in slice s."""
    out = [[False] * g.n_nodes for _ in range(g.n_slices)]
    for s in range(g.n_slices):
        u, x, _ = g.slice_edges(s)
        for e in range(u.size):
            out[s][int(u[e])] = out[s][int(x[e])] = True
    return out


def omega_sr(g, omega, i, s, r, pres=None):
    """The coupling weight between (i, s) and (i, r)."""
    cp = as_coupling(omega)
    c = cp.c(s, r)
    if not c:
        return Fraction(0)
    if cp.present_only:
        pres = pres or presence(g)
        if not (pres[s][i] and pres[r][i]):
            return Fraction(0)
    return cp.omega * c


def node_weights(g, omega):
    """CPM node weight per copy: 1, or 0 for an absent copy when only present copies are
    coupled (they are then not supra-nodes)."""
    cp = as_coupling(omega)
    if not cp.present_only:
        return [[1] * g.n_nodes for _ in range(g.n_slices)]
    return [[1 if x else 0 for x in row] for row in presence(g)]


def supra_adjacency(g, omega):
    """Dense A^supra of Eq. 3 as a list of lists of Fractions (order N*T, slice-major)."""
    n, t = g.n_nodes, g.n_slices
    mats = slice_matrices(g)
    size = n * t
    A = [[Fraction(0)] * size for _ in range(size)]
    for s in range(t):
        for i in range(n):
            for j in range(n):
                A[s * n + i][s * n + j] = Fraction(mats[s][i][j])
    pres = presence(g)
    for s in range(t):
        for r in range(t):
            if s != r:
                for i in range(n):
                    c = omega_sr(g, omega, i, s, r, pres)
                    if c:
                        A[s * n + i][r * n + i] = c
    return A


def degrees(mats):
    return [[sum(row) for row in a] for a in mats]


def two_mu(g, omega):
    mats = slice_matrices(g)
    tot = sum(sum(sum(row) for row in a) for a in mats)
    pres = presence(g)
    return Fraction(tot) + sum((omega_sr(g, omega, i, s, r, pres) for s in range(g.n_slices)
                                for r in range(g.n_slices) for i in range(g.n_nodes)),
                               Fraction(0))


def gammas(gamma, t):
    """gamma^(s), s = 0..t-1, from one resolution or a sequence of t."""
    if isinstance(gamma, (list, tuple, np.ndarray)):
        assert len(gamma) == t
        return [Fraction(x) for x in gamma]
    return [Fraction(gamma)] * t


def null_term(gam, k, twom, s, i, j, cpm, nw=None):
    """The null-model term of the pair (i, j) in slice s: gamma^(s) k_i k_j / 2m_s (zero in a
    slice without edges), or gamma^(s) n_i n_j under the multislice CPM (node weights nw,
    1 by default)."""
    if cpm:
        return gam[s] * (nw[s][i] * nw[s][j] if nw else 1)
    if not twom[s]:
        return Fraction(0)
    return gam[s] * k[s][i] * k[s][j] / Fraction(twom[s])


def _over_two_mu(num, g, omega):
    """num / 2mu; an empty supra-graph (2mu = 0) has Q = 0 by convention."""
    tm = two_mu(g, omega)
    return num / tm if tm else Fraction(0)


# --------------------------------------------------------------------------- Eq. 6, three ways

def q_quadruple_sum(g, gamma, omega, membership, cpm=False):
    """Eq. 6 literally: (1/2mu) sum_{ijsr} [(A_ij^s - gamma^(s) k_i^s k_j^s / 2m^s) delta_sr
    + delta_ij omega^sr] delta(c_i^s, c_j^r)  (cpm: gamma^(s) n_i n_j, n = 1)."""
    n, t = g.n_nodes, g.n_slices
    gam = gammas(gamma, t)
    mats = slice_matrices(g)
    k = degrees(mats)
    twom = [sum(ks) for ks in k]
    nw = node_weights(g, omega)
    pres = presence(g)
    c = np.asarray(membership).reshape(t, n)
    total = Fraction(0)
    for i, j, s, r in product(range(n), range(n), range(t), range(t)):
        if c[s][i] != c[r][j]:
            continue
        term = Fraction(0)
        if s == r:
            term += mats[s][i][j]
            term -= null_term(gam, k, twom, s, i, j, cpm, nw)
        if i == j:
            term += omega_sr(g, omega, i, s, r, pres)
        total += term
    return _over_two_mu(total, g, omega) 


def modularity_matrix(g, gamma, omega, cpm=False):
    """Supra-modularity matrix: per-slice A - gamma^(s) k k^T / 2m blocks (cpm: A - gamma^(s)
    J), omega couplings off-block."""
    n, t = g.n_nodes, g.n_slices
    gam = gammas(gamma, t)
    mats = slice_matrices(g)
    k = degrees(mats)
    twom = [sum(ks) for ks in k]
    nw = node_weights(g, omega)
    pres = presence(g)
    size = n * t
    M = [[Fraction(0)] * size for _ in range(size)]
    for s in range(t):
        for i in range(n):
            for j in range(n):
                M[s * n + i][s * n + j] = Fraction(mats[s][i][j]) - null_term(gam, k, twom, s, i,
                                                                               j, cpm, nw)
    for s in range(t):
        for r in range(t):
            if s != r:
                for i in range(n):
                    M[s * n + i][r * n + i] += omega_sr(g, omega, i, s, r, pres)
    return M


def q_trace_form(g, gamma, omega, membership, cpm=False):
    """Tr(C^T M C) / 2mu with C the one-hot community assignment matrix."""
    M = modularity_matrix(g, gamma, omega, cpm)
    labels = sorted(set(int(x) for x in np.asarray(membership).ravel()))
    col = {lab: a for a, lab in enumerate(labels)}
    size = len(M)
    C = [[0] * len(labels) for _ in range(size)]
    for u, lab in enumerate(np.asarray(membership).ravel()):
        C[u][col[int(lab)]] = 1
    # (C^T M C)_{aa}
    tr = Fraction(0)
    for a in range(len(labels)):
        mc = [sum((M[u][v] for v in range(size) if C[v][a]), Fraction(0)) for u in range(size)]
        tr += sum((mc[u] for u in range(size) if C[u][a]), Fraction(0))
    return _over_two_mu(tr, g, omega) 


def q_component_form(g, gamma, omega, membership, cpm=False):
    """Per-slice form: (sum_s [W_s - gamma^(s) SS_s / 2m_s] + omega I) / 2mu, where W_s is the
    intra weight inside communities (both directions), SS_s the sum over communities of
    the squared slice-s community degree (cpm: of the squared slice-s community size, and no
    2m_s), and omega I the coupling weight of the ordered copy pairs (i, s), (i, r) that share
    a community.  Works on edge lists (no dense matrix)."""
    n, t = g.n_nodes, g.n_slices
    gam = gammas(gamma, t)
    nw = node_weights(g, omega)
    pres = presence(g)
    c = np.asarray(membership).reshape(t, n)
    num = Fraction(0)
    for s in range(t):
        u, x, w = g.slice_edges(s)
        kdeg = [0] * n
        W = 0
        for e in range(u.size):
            ww = 1 if w is None else int(w[e])
            a, b = int(u[e]), int(x[e])
            kdeg[a] += ww
            kdeg[b] += ww
            if c[s][a] == c[s][b]:
                W += 2 * ww
        tm = sum(kdeg)
        sig = {}
        for i in range(n):
            sig[int(c[s][i])] = sig.get(int(c[s][i]), 0) + (nw[s][i] if cpm else kdeg[i])
        SS = sum(v * v for v in sig.values())
        num += W
        if cpm:
            num -= gam[s] * SS
        elif tm:
            num -= gam[s] * SS / Fraction(tm)
    for s in range(t):
        for r in range(t):
            for i in range(n):
                if c[s][i] == c[r][i]:
                    num += omega_sr(g, omega, i, s, r, pres)
    return _over_two_mu(num, g, omega)


def q_newman_static(g, gamma, membership):
    """Textbook undirected modularity for one snapshot: sum_c [L_c/m - gamma (d_c/2m)^2]."""
    assert g.n_slices == 1
    u, x, w = g.slice_edges(0)
    m = Fraction(0)
    inside, vol = {}, {}
    c = np.asarray(membership).ravel()
    for e in range(u.size):
        ww = 1 if w is None else int(w[e])
        a, b = int(u[e]), int(x[e])
        m += ww
        vol[int(c[a])] = vol.get(int(c[a]), 0) + ww
        vol[int(c[b])] = vol.get(int(c[b]), 0) + ww
        if c[a] == c[b]:
            inside[int(c[a])] = inside.get(int(c[a]), 0) + ww
    if m == 0:
        return Fraction(0)
    gamma = Fraction(gamma)
    return sum((Fraction(inside.get(cl, 0)) / m - gamma * (Fraction(vol.get(cl, 0)) / (2 * m)) ** 2
                for cl in set(int(v) for v in c)), Fraction(0))


# --------------------------------------------------------------------------- global null model
# Eq. 5 (undirected, so d_out = d_in) applied to the supra-adjacency of Eq. 3 as one graph:
# kappa_u = sum_v A_uv (intra degree plus coupling weight), 2mu = sum_u kappa_u, and
#   Q_G = (1/2mu) sum_{uv} [A_uv - gamma kappa_u kappa_v / 2mu] delta(c_u, c_v).
# The paper's GPU path optimised this on the supra-graph as a stand-in for Eq. 6.

def supra_degrees(g, omega):
    A = supra_adjacency(g, omega)
    return [sum(row, Fraction(0)) for row in A]


def global_modularity_matrix(g, gamma, omega):
    A = supra_adjacency(g, omega)
    kap = [sum(row, Fraction(0)) for row in A]
    tm = sum(kap, Fraction(0))
    gamma = Fraction(gamma)
    size = len(A)
    if tm == 0:
        return A
    return [[A[u][v] - gamma * kap[u] * kap[v] / tm for v in range(size)] for u in range(size)]


def q_global_pair_sum(g, gamma, omega, membership):
    """Q_G by the literal double sum over supra-node pairs."""
    A = supra_adjacency(g, omega)
    kap = [sum(row, Fraction(0)) for row in A]
    tm = sum(kap, Fraction(0))
    if tm == 0:
        return Fraction(0)
    gamma = Fraction(gamma)
    c = np.asarray(membership).ravel()
    total = Fraction(0)
    for u in range(len(A)):
        for v in range(len(A)):
            if c[u] == c[v]:
                total += A[u][v] - gamma * kap[u] * kap[v] / tm
    return total / tm


def q_global_trace_form(g, gamma, omega, membership):
    """Tr(C^T B C) / 2mu with B the global modularity matrix of the supra-graph."""
    B = global_modularity_matrix(g, gamma, omega)
    tm = sum(supra_degrees(g, omega), Fraction(0))
    if tm == 0:
        return Fraction(0)
    c = np.asarray(membership).ravel()
    groups = {}
    for u, lab in enumerate(c):
        groups.setdefault(int(lab), []).append(u)
    tr = sum((B[u][v] for mem in groups.values() for u in mem for v in mem), Fraction(0))
    return tr / tm


def q_global_all_singletons(g, gamma, omega):
    """Every supra-node alone: -gamma sum_u kappa_u^2 / (2mu)^2."""
    kap = supra_degrees(g, omega)
    tm = sum(kap, Fraction(0))
    return -Fraction(gamma) * sum(x * x for x in kap) / (tm * tm) if tm else Fraction(0)


def q_global_one_community(g, gamma, omega):
    """All supra-nodes together: 1 - gamma (0 for an empty supra-graph)."""
    tm = sum(supra_degrees(g, omega), Fraction(0))
    return 1 - Fraction(gamma) if tm else Fraction(0)


def brute_force_max_global(g, gamma, omega):
    """Maximum of Q_G over every set partition of at most 10 supra-nodes."""
    best, mems = _brute_force(global_modularity_matrix(g, gamma, omega))
    return _over_two_mu(best, g, omega), mems


# --------------------------------------------------------------------------- closed forms

def q_all_singletons(g, gamma, omega, cpm=False):
    """Every supra-node alone: only the diagonal null terms survive (cpm: -gamma^(s) per
    supra-node)."""
    mats = slice_matrices(g)
    k = degrees(mats)
    gam = gammas(gamma, g.n_slices)
    nw = node_weights(g, omega)
    num = Fraction(0)
    for s in range(g.n_slices):
        tm = sum(k[s])
        if cpm:
            num -= gam[s] * sum(nw[s])
        elif tm:
            num -= gam[s] * sum(x * x for x in k[s]) / Fraction(tm)
    return _over_two_mu(num, g, omega)


def q_one_community(g, gamma, omega, cpm=False):
    """All supra-nodes together: [sum_s (1 - gamma^(s)) 2m_s + 2 omega N (T-1)] / 2mu
    (cpm: sum_s (2m_s - gamma^(s) N^2) in place of the first sum)."""
    mats = slice_matrices(g)
    gam = gammas(gamma, g.n_slices)
    nw = node_weights(g, omega)
    num = two_mu(g, omega)
    for s, a in enumerate(mats):
        tm = sum(sum(row) for row in a)
        num -= gam[s] * sum(nw[s]) ** 2 if cpm else gam[s] * tm
    return _over_two_mu(num, g, omega)


# --------------------------------------------------------------------------- brute force

def brute_force_max(g, gamma, omega, cpm=False):
    """Maximum Q over every set partition of the N*T supra-nodes (restricted growth strings).

    Returns (Q*, list of optimal memberships).  Sizes up to 10 supra-nodes (Bell(10) = 115975).
    """
    best, mems = _brute_force(modularity_matrix(g, gamma, omega, cpm))
    return _over_two_mu(best, g, omega), mems


def _brute_force(M):
    """Maximum over all set partitions of the sum of M_uv over pairs in one block, and every
    membership reaching it (restricted growth strings)."""
    size = len(M)
    assert size <= 10, "brute force is for tiny graphs only"
    L = 1
    for row in M:
        for v in row:
            L = lcm(L, v.denominator)
    Mi = [[int(v * L) for v in row] for row in M]
    best = [None, []]
    assign = [0] * size
    blocks: list[list[int]] = []

    def rec(u, acc):
        if u == size:
            if best[0] is None or acc > best[0]:
                best[0], best[1] = acc, [assign.copy()]
            elif acc == best[0]:
                best[1].append(assign.copy())
            return
        for b in range(len(blocks) + 1):
            if b == len(blocks):
                blocks.append([])
            add = Mi[u][u] + 2 * sum(Mi[u][v] for v in blocks[b])
            blocks[b].append(u)
            assign[u] = b
            rec(u + 1, acc + add)
            blocks[b].pop()
            if not blocks[b]:
                blocks.pop()

    rec(0, 0)
    return Fraction(best[0], L), best[1]


# --------------------------------------------------------------------------- invariant helpers

def supra_edges(g, omega):
    """Undirected supra-edges (u, v, weight) of Eq. 3 with duplicates merged (omega > 0 adds
    the coupling edges)."""
    n, t = g.n_nodes, g.n_slices
    acc = {}
    for s in range(t):
        u, x, w = g.slice_edges(s)
        for e in range(u.size):
            a, b = s * n + int(u[e]), s * n + int(x[e])
            key = (min(a, b), max(a, b))
            acc[key] = acc.get(key, 0) + (1 if w is None else int(w[e]))
    out = [(a, b, Fraction(ww)) for (a, b), ww in acc.items()]
    pres = presence(g)
    for s in range(t):
        for r in range(s + 1, t):
            for i in range(n):
                c = omega_sr(g, omega, i, s, r, pres)
                if c:
                    out.append((s * n + i, r * n + i, c))
    return out


def communities_connected(g, omega, membership):
    """True when every community induces a connected subgraph of the supra-graph."""
    size = g.n_supra
    c = np.asarray(membership).ravel()
    adj = [[] for _ in range(size)]
    for a, b, _ in supra_edges(g, omega):
        if c[a] == c[b]:
            adj[a].append(b)
            adj[b].append(a)
    seen = [False] * size
    comps_per_label = {}
    for v in range(size):
        if seen[v]:
            continue
        comps_per_label[int(c[v])] = comps_per_label.get(int(c[v]), 0) + 1
        stack = [v]
        seen[v] = True
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if not seen[y]:
                    seen[y] = True
                    stack.append(y)
    return all(k == 1 for k in comps_per_label.values())


def improving_single_moves(g, gamma, omega, membership, cpm=False):
    """All (supra-node, target) pairs whose move raises Q strictly (targets: communities of
    neighbours, and a fresh empty community).  Evaluated by recomputing Q exactly."""
    c = np.asarray(membership).ravel().copy()
    base = q_component_form(g, gamma, omega, c, cpm)
    nbr = [set() for _ in range(g.n_supra)]
    for a, b, _ in supra_edges(g, omega):
        nbr[a].add(b)
        nbr[b].add(a)
    fresh = int(c.max()) + 1
    found = []
    for v in range(g.n_supra):
        targets = {int(c[x]) for x in nbr[v]} | {fresh}
        targets.discard(int(c[v]))
        for tgt in sorted(targets):
            old = c[v]
            c[v] = tgt
            if q_component_form(g, gamma, omega, c, cpm) > base:
                found.append((v, tgt))
            c[v] = old
    return found
