"""Seeded synthetic snapshot temporal networks (inputs only).

This module draws random temporal graphs and nothing else: it holds none of the
clustering arithmetic, so both the oracle and the HIP path take their inputs from
here.  The paper's datasets (Table 1) are not available; the stand-ins follow the
structure of its synthetic SBM rows (Section 4, Table 1): planted communities,
node persistence with churn between consecutive snapshots, and edges resampled in
every snapshot.

Layout of a graph (the boundary's input format): ``T`` snapshots over the same
``N`` node ids; slice ``s`` owns edges ``[offsets[s], offsets[s+1])`` of the
``src``/``dst``/``weight`` arrays, each undirected edge listed once, no self-loops,
``weight`` int32 >= 1 or ``None`` for unit weights.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from fractions import Fraction
from typing import Optional

import numpy as np


@dataclass
class TemporalGraph:
    n_nodes: int
    n_slices: int
    offsets: np.ndarray            # int64[T+1]
    src: np.ndarray                # int32[E]
    dst: np.ndarray                # int32[E]
    weight: Optional[np.ndarray]   # int32[E] or None (unit weights)
    planted: Optional[np.ndarray] = None   # int32[T, N] generating labels, if any
    name: str = ""

    @property
    def n_edges(self) -> int:
        return int(self.offsets[-1])

    @property
    def n_supra(self) -> int:
        return self.n_nodes * self.n_slices

    def slice_edges(self, s: int):
        a, b = int(self.offsets[s]), int(self.offsets[s + 1])
        w = None if self.weight is None else self.weight[a:b]
        return self.src[a:b], self.dst[a:b], w


@dataclass(frozen=True)
class SolveSpec:
    """One clustering request: resolution gamma and coupling omega as exact fractions."""
    gamma: Fraction = Fraction(1)
    omega: Fraction = Fraction(1)
    max_levels: int = 32
    max_iterations: int = 2
    seed: int = 0


def _assemble(n, t, per_slice, planted=None, name="", weighted=False):
    offs = np.zeros(t + 1, dtype=np.int64)
    srcs, dsts, ws = [], [], []
    for s, (u, x, w) in enumerate(per_slice):
        offs[s + 1] = offs[s] + u.size
        srcs.append(u.astype(np.int32))
        dsts.append(x.astype(np.int32))
        if weighted:
            ws.append(w.astype(np.int32))
    src = np.concatenate(srcs) if srcs else np.zeros(0, np.int32)
    dst = np.concatenate(dsts) if dsts else np.zeros(0, np.int32)
    weight = (np.concatenate(ws) if ws else np.zeros(0, np.int32)) if weighted else None
    return TemporalGraph(n, t, offs, src, dst, weight, planted, name)


def _dedup_pairs(u, x, n):
    """Drop self-pairs and repeated unordered pairs, keeping first occurrences in order."""
    keep = u != x
    u, x = u[keep], x[keep]
    lo = np.minimum(u, x).astype(np.int64)
    hi = np.maximum(u, x).astype(np.int64)
    _, first = np.unique(lo * n + hi, return_index=True)
    first.sort()
    return u[first], x[first]


# --------------------------------------------------------------------------- planted partition

def planted_partition(n=1000, t=4, k=10, p_in=0.05, p_out=0.002, churn=0.10, seed=0,
                      name="planted"):
    """Planted partition with exact Bernoulli edges over all node pairs, per snapshot.

    Community of node i in snapshot 0 is i // (n/k).  Between consecutive snapshots a
    ``churn`` fraction of nodes, drawn without replacement, moves to a uniformly chosen
    other community.  Unit weights.
    """
    rng = np.random.default_rng(seed)
    z = (np.arange(n) * k // n).astype(np.int64)
    iu, ju = np.triu_indices(n, 1)
    per_slice, planted = [], []
    for s in range(t):
        if s > 0:
            z = z.copy()
            movers = rng.choice(n, size=int(round(churn * n)), replace=False)
            z[movers] = (z[movers] + rng.integers(1, k, size=movers.size)) % k
        planted.append(z.astype(np.int32))
        prob = np.where(z[iu] == z[ju], p_in, p_out)
        keep = rng.random(iu.size) < prob
        per_slice.append((iu[keep], ju[keep], None))
    return _assemble(n, t, per_slice, np.stack(planted), name)


# --------------------------------------------------------------------------- degree-corrected SBM

def _powerlaw_propensity(n, alpha, mean, rng):
    """Continuous power law x^-alpha on [kmin, kmax], kmax = floor(sqrt(n*mean)), mean fixed."""
    kmax = float(math.floor(math.sqrt(n * mean)))
    a, b = 1.0 - alpha, 2.0 - alpha

    def mean_of(kmin):
        return ((kmax ** b - kmin ** b) / b) / ((kmax ** a - kmin ** a) / a)

    lo, hi = 1e-6, mean
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mean_of(mid) < mean:
            lo = mid
        else:
            hi = mid
    kmin = 0.5 * (lo + hi)
    u = rng.random(n)
    return (kmin ** a + u * (kmax ** a - kmin ** a)) ** (1.0 / a)


def _community_sizes(n, k, rng, exponent=1.5, min_size=10):
    """k sizes from a power law with the given exponent, scaled to sum to n, each >= min_size."""
    if n < k * min_size:
        min_size = max(1, n // k)
    a = 1.0 - exponent
    xmax = float(max(k, 2))
    u = rng.random(k)
    raw = (1.0 + u * (xmax ** a - 1.0)) ** (1.0 / a)
    spare = n - k * min_size
    sizes = min_size + np.floor(spare * raw / raw.sum()).astype(np.int64)
    rem = n - int(sizes.sum())
    order = np.argsort(-raw, kind="stable")
    sizes[order[:rem]] += 1
    return sizes


def _sample_in_block(theta, labels, comm_of_u, rng, k):
    """x ~ theta restricted to community comm_of_u[j] (vectorised inverse-CDF draws)."""
    order = np.argsort(labels, kind="stable")
    cum = np.cumsum(theta[order])
    counts = np.bincount(labels, minlength=k)
    end = np.cumsum(counts)
    start = end - counts
    before = np.where(start > 0, cum[np.maximum(start - 1, 0)], 0.0)
    total = cum[np.maximum(end - 1, 0)] - before
    r = before[comm_of_u] + rng.random(comm_of_u.size) * total[comm_of_u]
    idx = np.searchsorted(cum, r, side="right")
    idx = np.clip(idx, start[comm_of_u], np.maximum(end[comm_of_u] - 1, start[comm_of_u]))
    return order[idx]


def _dcsbm_slice(s, seed, cdf, theta, labels, k, m, mu, weights_max):
    """Edges of snapshot s, drawn from the snapshot's own generator (seed, s + 1)."""
    n = cdf.size
    rng = np.random.default_rng([seed, s + 1])
    u = np.searchsorted(cdf, rng.random(m), side="right").clip(0, n - 1)
    inside = rng.random(m) >= mu
    x = np.empty(m, dtype=np.int64)
    x[inside] = _sample_in_block(theta, labels, labels[u[inside]], rng, k)
    out_idx = np.nonzero(~inside)[0]
    xo = np.searchsorted(cdf, rng.random(out_idx.size), side="right").clip(0, n - 1)
    bad = labels[xo] == labels[u[out_idx]]
    tries = 0
    while bad.any() and tries < 1000:
        xo[bad] = np.searchsorted(cdf, rng.random(int(bad.sum())), side="right").clip(0, n - 1)
        bad = labels[xo] == labels[u[out_idx]]
        tries += 1
    x[out_idx] = xo
    uu, xx = _dedup_pairs(u, x, n)
    w = rng.integers(1, weights_max + 1, size=uu.size) if weights_max > 1 else None
    return uu.astype(np.int32), xx.astype(np.int32), None if w is None else w.astype(np.int32)


def _pool(workers):
    import concurrent.futures as cf
    import multiprocessing as mp
    # fresh interpreters: the parent may already hold a GPU context
    return cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"))


def dcsbm(n, t, mean_degree, k, mu, alpha, churn, weights_max=1, seed=0, name="dcsbm",
          workers=1):
    """Degree-corrected SBM snapshots with power-law propensities and community churn.

    Propensity theta_i is fixed across snapshots.  Per snapshot, round(n*mean/2) endpoint
    pairs are drawn: u ~ theta; with probability 1-mu, x ~ theta inside u's community,
    else x ~ theta outside it (rejection).  Self-pairs and repeated pairs are dropped.
    Between snapshots floor(churn*n) nodes move to another community chosen with
    probability proportional to its size.  Weights are uniform integers in
    1..weights_max (``None`` when weights_max == 1).  The propensities and the community
    chain come from generator ``seed``; snapshot s draws its edges from generator
    (seed, s + 1), so snapshots can be drawn in ``workers`` processes with identical output.
    """
    rng = np.random.default_rng(seed)
    theta = _powerlaw_propensity(n, alpha, mean_degree, rng)
    sizes = _community_sizes(n, k, rng)
    labels = np.repeat(np.arange(k), sizes)[rng.permutation(n)].astype(np.int64)
    cdf = np.cumsum(theta)
    cdf /= cdf[-1]
    m = int(round(n * mean_degree / 2))
    planted = []
    for s in range(t):
        if s > 0:
            labels = labels.copy()
            movers = rng.choice(n, size=int(math.floor(churn * n)), replace=False)
            cnt = np.bincount(labels, minlength=k).astype(np.float64)
            pcum = np.cumsum(cnt / cnt.sum())
            new = np.searchsorted(pcum, rng.random(movers.size), side="right").clip(0, k - 1)
            clash = new == labels[movers]
            while clash.any():
                new[clash] = np.searchsorted(pcum, rng.random(int(clash.sum())),
                                             side="right").clip(0, k - 1)
                clash = new == labels[movers]
            labels[movers] = new
        planted.append(labels)
    args = [(s, seed, cdf, theta, planted[s], k, m, mu, weights_max) for s in range(t)]
    if workers > 1 and t > 1:
        with _pool(min(workers, t)) as ex:
            per_slice = list(ex.map(_dcsbm_slice, *zip(*args)))
    else:
        per_slice = [_dcsbm_slice(*a) for a in args]
    planted = np.stack([p.astype(np.int32) for p in planted])
    return _assemble(n, t, per_slice, planted, name, weighted=weights_max > 1)


# --------------------------------------------------------------------------- small random graphs

def erdos_renyi(n, t, p, seed=0, weights_max=1, name="er"):
    """Independent G(n, p) snapshots; used for small parity and invariant cases."""
    rng = np.random.default_rng(seed)
    per_slice = []
    iu, ju = np.triu_indices(n, 1)
    for _ in range(t):
        keep = rng.random(iu.size) < p
        u, x = iu[keep], ju[keep]
        flip = rng.random(u.size) < 0.5          # orientation carries no meaning
        u2, x2 = np.where(flip, x, u), np.where(flip, u, x)
        w = rng.integers(1, weights_max + 1, size=u.size) if weights_max > 1 else None
        per_slice.append((u2, x2, w))
    return _assemble(n, t, per_slice, None, name, weighted=weights_max > 1)


def with_absences(g, frac, seed=0):
    """g with every edge of a node dropped in the snapshots where it is absent: each node is
    absent from each snapshot with probability frac (the data of the paper's Table 1, whose
    nodes appear in only some snapshots)."""
    rng = np.random.default_rng(seed)
    absent = rng.random((g.n_slices, g.n_nodes)) < frac
    src, dst, w, off = [], [], [], [0]
    for s in range(g.n_slices):
        u, x, ww = g.slice_edges(s)
        keep = ~(absent[s][u] | absent[s][x])
        src.append(u[keep])
        dst.append(x[keep])
        if ww is not None:
            w.append(ww[keep])
        off.append(off[-1] + int(keep.sum()))
    return TemporalGraph(g.n_nodes, g.n_slices, np.array(off, np.int64),
                         np.concatenate(src).astype(np.int32), np.concatenate(dst).astype(np.int32),
                         None if g.weight is None else np.concatenate(w).astype(np.int32),
                         g.planted, g.name + "_absent")


def from_edge_lists(n, slices, weighted=False, name="custom"):
    """Build a graph from a list of per-slice [(u, x[, w]), ...] edge lists."""
    per = []
    for edges in slices:
        if len(edges) == 0:
            per.append((np.zeros(0, np.int64), np.zeros(0, np.int64),
                        np.zeros(0, np.int64) if weighted else None))
            continue
        arr = np.asarray(edges, dtype=np.int64)
        per.append((arr[:, 0], arr[:, 1], arr[:, 2] if weighted else None))
    return _assemble(n, len(slices), per, None, name, weighted=weighted)


# --------------------------------------------------------------------------- the named workloads

def config1():
    """Planted partition: T=4 x N=1000, 10 equal communities, p_in=.05, p_out=.002, 10% churn."""
    return planted_partition(1000, 4, 10, 0.05, 0.002, 0.10, seed=0, name="cfg1_planted_T4_N1k")


def config2(workers=1):
    """DC-SBM: T=16 x N=100k, exponent 2.5, mean degree 16, 100 communities, mu=.3, w in 1..8."""
    return dcsbm(100_000, 16, 16, 100, 0.3, 2.5, 0.05, weights_max=8, seed=2,
                 name="cfg2_dcsbm_T16_N100k", workers=workers)


def config3(workers=1):
    """DC-SBM: T=64 x N=1M, exponent 2.1, mean degree 10, 1000 communities, mu=.4, unit."""
    return dcsbm(1_000_000, 64, 10, 1000, 0.4, 2.1, 0.02, weights_max=1, seed=3,
                 name="cfg3_dcsbm_T64_N1M", workers=workers)


CONFIG_SOLVE = {
    1: SolveSpec(Fraction(1), Fraction(1)),
    2: SolveSpec(Fraction(1), Fraction(1)),
    3: SolveSpec(Fraction(1), Fraction(1, 2)),
}

# The SBM rows of the paper's Table 1 (the snapshot graphs of its Fig. 2b doubling study):
# nodes N, snapshots T and mean degree per snapshot, with 10 communities: the base (50k nodes,
# 5 snapshots, 1.25M edges), then N, the edges and T doubled in turn.
SWEEP_SHAPES = {
    "sbm": (50_000, 5, 10),
    "sbm_n": (100_000, 5, 10),
    "sbm_e": (50_000, 5, 20),
    "sbm_t": (50_000, 10, 10),
}
SWEEP_SOLVE = SolveSpec(Fraction(1), Fraction(1))


def sweep_graph(name, workers=1):
    """A DC-SBM of one of the SWEEP_SHAPES (exponent 2.5, mu 0.3, churn 0.05, unit weights)."""
    n, t, mean = SWEEP_SHAPES[name]
    return dcsbm(n, t, mean, 10, 0.3, 2.5, 0.05, seed=11, name=f"{name}_dcsbm_N{n}_T{t}_d{mean}",
                 workers=workers)


# The two long sequences of the paper's Table 1, as synthetic stand-ins of the same shape: N
# nodes, T snapshots, about E/T edges per snapshot (drawn before repeated pairs are dropped), drawn with the DC-SBM rule over all N nodes
# (so each snapshot holds only the nodes its edges touch, as in the data, whose nodes appear in
# few snapshots): Patent (the headline speed-up: N 12 214, T 891, 41 916 edges, 41 529 present
# node copies) and School (the longest sequence: N 327, T 7 375, 188 508 edges, 309 006 copies).
# Entries: N, T, edges per snapshot, communities, mu, propensity exponent, churn.
LONG_SHAPES = {
    "patent": (12_214, 891, 52, 60, 0.2, 2.1, 0.01),
    "school": (327, 7_375, 28, 10, 0.3, 2.5, 0.01),
}
LONG_SOLVE = SolveSpec(Fraction(1), Fraction(1))
LONG_WINDOW = (64, 8)   # snapshots per window, overlapping snapshots


def long_graph(name, workers=1):
    """A DC-SBM sequence of one of the LONG_SHAPES (unit weights)."""
    n, t, e, k, mu, alpha, churn = LONG_SHAPES[name]
    return dcsbm(n, t, 2.0 * e / n, k, mu, alpha, churn, seed=13,
                 name=f"long_{name}_N{n}_T{t}", workers=workers)


GAMMA_GRID = (Fraction(1, 2), Fraction(1), Fraction(2))
OMEGA_GRID = (Fraction(1, 10), Fraction(1), Fraction(10))


def batch_graph_shape(g):
    """Shape of graph g of the 512-graph batch: N log-uniform in 200..50k, T in 2..32, ..."""
    rng = np.random.default_rng(1000 + g)
    n = int(round(math.exp(rng.uniform(math.log(200), math.log(50_000)))))
    t = int(rng.integers(2, 33))
    kbar = float(rng.uniform(4, 24))
    mu = float(rng.uniform(0.1, 0.5))
    return n, t, kbar, mu


def batch_graph(g, scale=1.0):
    """Graph g of the batched workload (unit weights, exponent 2.5, K=max(2,round(sqrt N)))."""
    n, t, kbar, mu = batch_graph_shape(g)
    n = max(20, int(round(n * scale)))
    k = max(2, int(round(math.sqrt(n))))
    return dcsbm(n, t, kbar, k, mu, 2.5, 0.05, weights_max=1, seed=1000 + g,
                 name=f"cfg4_g{g}")


def batch_solves(n_graphs=512):
    """The (graph, gamma, omega) grid of the batched workload: 9 solves per graph."""
    out = []
    for g in range(n_graphs):
        for gam in GAMMA_GRID:
            for om in OMEGA_GRID:
                out.append((g, SolveSpec(gam, om, 32, 2, 0)))
    return out


def serve_trace(n_requests=1000, rate_per_s=100.0, n_graphs=512, large_frac=0.05, seed=5):
    """Poisson arrivals; each request picks a batched-workload graph (95%) or one of eight
    config-2-sized graphs (5%), and a (gamma, omega) pair from the grid."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for r in range(n_requests):
        large = rng.random() < large_frac
        gid = int(rng.integers(0, 8)) if large else int(rng.integers(0, n_graphs))
        gam = GAMMA_GRID[int(rng.integers(0, 3))]
        om = OMEGA_GRID[int(rng.integers(0, 3))]
        reqs.append(dict(t=float(arrivals[r]), large=bool(large), graph=gid,
                         spec=SolveSpec(gam, om, 32, 2, 0)))
    return reqs


def large_serve_graph(i, workers=1):
    """One of the eight config-2-sized graphs of the served mix (seeds 9000..9007)."""
    return dcsbm(100_000, 16, 16, 100, 0.3, 2.5, 0.05, weights_max=8, seed=9000 + i,
                 name=f"cfg5_large{i}", workers=workers)


def batch_graphs(indices, scale=1.0, workers=1):
    """Several graphs of the batched workload, drawn in ``workers`` processes."""
    indices = list(indices)
    if workers > 1 and len(indices) > 1:
        with _pool(workers) as ex:
            return list(ex.map(batch_graph, indices, [scale] * len(indices)))
    return [batch_graph(g, scale) for g in indices]
