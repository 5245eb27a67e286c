"""The deterministic multislice Leiden schedule, taken step by step (test infrastructure only).

This file belongs to the oracle: only tests, the smoke check and the benchmark's CPU baseline
may use it.  It is a second, independent statement of the schedule that ``mslm_oracle.c``
runs at scale, written for tiny inputs and for being read against the paper:

* Every decision is taken on the exact change of Q_MS (Eq. 6, Section 3.2) of the partition
  of the level-0 supra-graph (Eq. 3, Section 3.1) that the decision would produce.  Units of
  aggregated levels are kept as sets of level-0 supra-nodes, so no aggregated graph, slice
  profile, scaled integer gain, Sigma table or running edge-weight counter enters a decision.
* Exact integers throughout: Q_MS * 2mu * L for a common multiple L of every denominator.

The schedule (Leiden with local moving, refinement and aggregation, Section 3.2, made
deterministic; the readings are the ones listed in the design notes):

* Objectives: Q_MS of Eq. 6 with a resolution gamma^(s) per slice (one gamma for all slices
  by default); the global modularity of the supra-graph (Eq. 5); the multislice CPM, whose
  null term is gamma^(s) n_i n_j with node weight n = 1 per supra-node (no 2m_s).
* Iterations start from the canonical form of the previous partition (singletons, or the
  given start partition, first); an
  iteration whose output equals its start is stable and ends the solve; max_iterations <= 0
  means until stable, at most 32.
* Per level: first-fit colouring of the units in decreasing hash priority; colour-batched
  synchronous local moving; stop when every community is one unit or the level cap is
  reached; refinement; stop when no two units merged; aggregation by refined sub-communities.
* Local moving: every unit of a colour batch is decided against the state at the batch's
  start; its candidates are the communities of its neighbouring units plus an empty community
  that ranks above every label; the best candidate has the largest change of Q, ties going to
  the lowest label; the unit moves only when that change is strictly positive; a unit that
  moves to the empty community in sweep t takes the label n*(1+t)+u (n units at the level).
  Sweeps end at the first sweep without a move or after max_sweeps (32 by default).
* Refinement (greedy Leiden refinement): sub-communities start as single units; a set X is
  well connected in its community K when the edge weight between X and K minus X is at least
  sum_s gamma^(s) Sigma_{X,s} (Sigma_{K,s} - Sigma_{X,s}) / 2m_s.  In each round every single
  unit that is well connected and still active proposes the well-connected sub-community of
  its own community, adjacent to it, whose joining raises Q of the refined partition the most
  (strictly positive, ties to the lowest label); an active unit without a proposal drops out
  for the rest of the refinement.  A proposer joins its target when the target's founder does
  not propose, or when the proposer outranks (phase-1 hash priority) every proposing neighbour
  of its community and the founder's own target is itself a proposing unit.  Rounds end at the
  first round without a merge (at most 256).
* After the levels: communities split into their connected components on the level-0
  supra-graph; labels in order of first appearance in v = s*N + i.
"""
from __future__ import annotations

from fractions import Fraction
from math import lcm

MASK64 = (1 << 64) - 1
MAX_ITER_CAP = 32
DEFAULT_SWEEPS = 32
MAX_REFINE_ROUNDS = 256


# --------------------------------------------------------------------------- priorities

def splitmix64_mix(z: int) -> int:
    """The SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def hash_priority(seed: int, it: int, lvl: int, phase: int, u: int) -> int:
    """H(seed, it, level, phase, u): the unit id in the low 32 bits, the phase, level and
    iteration above it, mixed with the mixed seed."""
    key = u | (phase << 32) | (lvl << 40) | (it << 48)
    return splitmix64_mix(key ^ splitmix64_mix(seed))


# --------------------------------------------------------------------------- the supra-graph

class SupraGraph:
    """Level-0 supra-graph of Eq. 3; supra-node v = s*N + i.  Coupling omega^(sr) = omega *
    c_sr between (i, s) and (i, r): c ordinal (1 for |s - r| = 1) unless a T x T integer matrix
    is given; present_only: only between copies that have an edge in their slices."""

    def __init__(self, g, omega, coupling=None, present_only=False):
        self.N, self.T = g.n_nodes, g.n_slices
        self.n = self.N * self.T
        self.omega = Fraction(omega)
        self.present_only = bool(present_only)
        nbr = [dict() for _ in range(self.n)]          # v -> {x: weight (Fraction)}
        intra = [dict() for _ in range(self.n)]        # raw intra weights only
        for s in range(self.T):
            u, x, w = g.slice_edges(s)
            for e in range(len(u)):
                a, b = s * self.N + int(u[e]), s * self.N + int(x[e])
                ww = 1 if w is None else int(w[e])
                intra[a][b] = intra[a].get(b, 0) + ww
                intra[b][a] = intra[b].get(a, 0) + ww
        for v in range(self.n):
            for x, ww in intra[v].items():
                nbr[v][x] = Fraction(ww)
        self.present = [bool(intra[v]) for v in range(self.n)]

        def c_of(s, r):
            if coupling is None:
                return 1 if abs(s - r) == 1 else 0
            return int(coupling[s][r]) if s != r else 0

        mult = {}                                          # (v, x) -> c_sr of a coupled pair
        for s in range(self.T):
            for r in range(self.T):
                c = c_of(s, r)
                if not c:
                    continue
                for i in range(self.N):
                    a, b = s * self.N + i, r * self.N + i
                    if self.present_only and not (self.present[a] and self.present[b]):
                        continue
                    mult[(a, b)] = c
        self.mult = mult
        if self.omega != 0:
            for (a, b), c in mult.items():
                nbr[a][b] = self.omega * c
        self.nbr = nbr
        self.intra = intra
        self.slice = [v // self.N for v in range(self.n)]
        self.k = [sum(intra[v].values()) for v in range(self.n)]     # intra degree k_{i,s}
        self.two_m = [sum(self.k[s * self.N:(s + 1) * self.N]) for s in range(self.T)]
        # directed entries for the integer score
        self.intra_entries = [(v, x, ww) for v in range(self.n) for x, ww in intra[v].items()]
        self.inter_entries = [(v, x, mult[(v, x)]) for v in range(self.n) for x in nbr[v]
                              if x not in intra[v]]


class GlobalScore:
    """The global modularity Q_G of the supra-graph (Eq. 5 over all supra-nodes) as an exact
    integer multiple: with kappa'_u = b * (intra degree) + a * (coupling count) (omega = a/b),
    2mu' = sum kappa', W' = b * (intra weight inside communities) + a * (coupling entries
    inside communities), SS' = sum over communities of (sum kappa')^2:
        q * 2mu' * W' - p * SS' = q * 2mu'^2 * Q_G            (gamma = p/q)."""

    def __init__(self, G: SupraGraph, gamma):
        self.G = G
        gamma = Fraction(gamma)
        self.p, self.q = gamma.numerator, gamma.denominator
        a, b = G.omega.numerator, G.omega.denominator
        self.a, self.b = a, b
        self.kap = [b * G.k[v] + a * sum(c for (u, x, c) in G.inter_entries if u == v)
                    for v in range(G.n)]
        self.two_mu = sum(self.kap)

    def __call__(self, lab) -> int:
        G = self.G
        W = 0
        for v, x, ww in G.intra_entries:
            if lab[v] == lab[x]:
                W += self.b * ww
        for v, x, c in G.inter_entries:
            if lab[v] == lab[x]:
                W += self.a * c
        sig = {}
        for v in range(G.n):
            sig[lab[v]] = sig.get(lab[v], 0) + self.kap[v]
        return self.q * self.two_mu * W - self.p * sum(x * x for x in sig.values())

    def q(self, lab) -> Fraction:
        return Fraction(self(lab), self.q * self.two_mu ** 2) if self.two_mu else Fraction(0)


def per_slice(gamma, T):
    """gamma^(s) for s = 0..T-1 from one resolution or a sequence of T."""
    if isinstance(gamma, (list, tuple)):
        assert len(gamma) == T
        return [Fraction(x) for x in gamma]
    return [Fraction(gamma)] * T


def null_weight(G, v, cpm):
    """The weight a supra-node carries into its slice's null term: its intra degree k_{i,s}
    (Eq. 6), or 1 under the multislice CPM (0 for an absent copy when only present copies
    are coupled: it is then not a supra-node)."""
    if cpm:
        return 0 if (G.present_only and not G.present[v]) else 1
    return G.k[v]


class Score:
    """L * 2mu * Q_MS(partition) as an exact integer, for one (graph, per-slice gamma):
        2mu Q = sum_s [ W_s - gamma^(s) SS_s / 2m_s ] + omega I        (Eq. 6)
    W_s: intra weight (both directions) inside communities, SS_s: sum over communities of the
    squared slice-s degree, I: directed coupling entries inside communities.  Under the
    multislice CPM SS_s sums squared supra-node counts and there is no 2m_s.  L clears every
    denominator, so comparisons of changes of Q are comparisons of integers."""

    def __init__(self, G: SupraGraph, gamma, cpm=False):
        self.G = G
        self.cpm = cpm
        gam = per_slice(gamma, G.T)
        coef = [gam[s] if cpm else (gam[s] / G.two_m[s] if G.two_m[s] > 0 else Fraction(0))
                for s in range(G.T)]
        L = lcm(G.omega.denominator, *[c.denominator for c in coef])
        self.L = L
        self.c_null = [L * c for c in coef]
        assert all(c.denominator == 1 for c in self.c_null)
        self.c_null = [int(c) for c in self.c_null]
        c_int = L * G.omega
        assert c_int.denominator == 1
        self.c_inter = int(c_int)

    def __call__(self, lab) -> int:
        G = self.G
        total = 0
        for v, x, ww in G.intra_entries:
            if lab[v] == lab[x]:
                total += self.L * ww
        for v, x, c in G.inter_entries:
            if lab[v] == lab[x]:
                total += self.c_inter * c
        sig = {}
        for v in range(G.n):
            x = null_weight(G, v, self.cpm)
            if x:
                key = (lab[v], G.slice[v])
                sig[key] = sig.get(key, 0) + x
        for (c, s), x in sig.items():
            total -= self.c_null[s] * x * x
        return total

    def q(self, lab) -> Fraction:
        G = self.G
        two_mu = sum(G.two_m) + G.omega * sum(G.mult.values())
        return Fraction(self(lab), self.L) / two_mu if two_mu else Fraction(0)


# --------------------------------------------------------------------------- helpers

def canonical(labels):
    """Dense rank of each element's community by the smallest element holding its label."""
    first = {}
    for u, c in enumerate(labels):
        if c not in first:
            first[c] = len(first)
    return [first[c] for c in labels]


def unit_adjacency(G: SupraGraph, unit_of, n_units):
    """Neighbouring units: units joined by at least one level-0 entry (self-loops dropped)."""
    adj = [set() for _ in range(n_units)]
    for v in range(G.n):
        for x in G.nbr[v]:
            a, b = unit_of[v], unit_of[x]
            if a != b:
                adj[a].add(b)
    return [sorted(s) for s in adj]


def first_fit_colouring(adj, seed, it, lvl):
    """colour(u) = smallest colour not taken by a neighbour of higher priority
    (hash, id); computed in decreasing priority order."""
    n = len(adj)
    pri = {u: (hash_priority(seed, it, lvl, 0, u), u) for u in range(n)}
    colour = [-1] * n
    for u in sorted(range(n), key=lambda x: pri[x], reverse=True):
        taken = {colour[x] for x in adj[u] if pri[x] > pri[u]}
        c = 0
        while c in taken:
            c += 1
        colour[u] = c
    return colour


def flatten(units, unit_labels, n0):
    lab = [None] * n0
    for u, members in enumerate(units):
        for v in members:
            lab[v] = unit_labels[u]
    return lab


# --------------------------------------------------------------------------- local moving

def local_move(G, score, units, adj, colour, labels, max_sweeps, stats):
    """Colour-batched synchronous moves on exact changes of Q; returns the sweeps run."""
    n = len(units)
    ncol = max(colour) + 1 if n else 0
    sweeps = 0
    for t in range(max_sweeps):
        sweeps += 1
        moved = 0
        for c in range(ncol):
            batch = [u for u in range(n) if colour[u] == c]
            base_lab = flatten(units, labels, G.n)
            base = score(base_lab)
            decision = {}
            for u in batch:
                D = labels[u]

                def change(target):
                    lab = list(base_lab)
                    for v in units[u]:
                        lab[v] = target
                    return score(lab) - base
                cands = sorted({labels[x] for x in adj[u]} - {D})
                # the empty community: a label no unit holds, ranking above every label
                best_gain, best_label = change(("empty",)), None
                for C in cands:
                    gC = change(C)
                    if gC > best_gain or (gC == best_gain and best_label is None):
                        best_gain, best_label = gC, C
                if best_gain > 0:
                    decision[u] = n * (1 + t) + u if best_label is None else best_label
            for u, lab in decision.items():
                labels[u] = lab
            moved += len(decision)
        stats["sweeps"] += 1
        stats["moves"] += moved
        if moved == 0:
            break
        if t == max_sweeps - 1:
            stats["sweep_cap_hits"] += 1
    return sweeps


# --------------------------------------------------------------------------- refinement

def well_connected(G, gamma, X, K, null_model=0):
    """ext(X) >= sum_s gamma^(s) Sigma_{X,s} (Sigma_{K,s} - Sigma_{X,s}) / 2m_s, where ext(X) is
    the weight of the supra-edges between X and K minus X (X, K sets of level-0 supra-nodes);
    for the global null model ext(X) >= gamma * kappa_X (kappa_K - kappa_X) / 2mu; for the
    multislice CPM the Sigmas count supra-nodes and there is no 2m_s."""
    if null_model == 1:
        return external_weight(G, X, K) >= null_between_global(G, gamma, X, K)
    return external_weight(G, X, K) >= null_between(G, gamma, X, K, cpm=null_model == 2)


def null_between_global(G, gamma, X, K):
    kap = [G.k[v] + sum((w for x, w in G.nbr[v].items() if x not in G.intra[v]), Fraction(0))
           for v in range(G.n)]
    tm = sum(kap, Fraction(0))
    if tm == 0:
        return Fraction(0)
    kx = sum((kap[v] for v in X), Fraction(0))
    kk = sum((kap[v] for v in K), Fraction(0))
    return Fraction(gamma) * kx * (kk - kx) / tm


def external_weight(G, X, K):
    return sum((w for v in X for x, w in G.nbr[v].items() if x in K and x not in X), Fraction(0))


def null_between(G, gamma, X, K, cpm=False):
    gam = per_slice(gamma, G.T)
    sx, sk = [0] * G.T, [0] * G.T
    for v in X:
        sx[G.slice[v]] += null_weight(G, v, cpm)
    for v in K:
        sk[G.slice[v]] += null_weight(G, v, cpm)
    tot = Fraction(0)
    for s in range(G.T):
        if cpm:
            tot += gam[s] * sx[s] * (sk[s] - sx[s])
        elif G.two_m[s]:
            tot += gam[s] * Fraction(sx[s] * (sk[s] - sx[s]), G.two_m[s])
    return tot


def refine(G, score, gamma, units, adj, labels, seed, it, lvl, stats, null_model=0):
    """Greedy round-synchronous refinement inside the communities `labels`; returns R (the
    founder unit of each unit's sub-community)."""
    n = len(units)
    R = list(range(n))
    single = [True] * n
    comm_members = {}
    for u in range(n):
        comm_members.setdefault(labels[u], set()).update(units[u])

    def members(T):
        return {v for u in range(n) if R[u] == T for v in units[u]}

    def wc(T):
        return well_connected(G, gamma, members(T), comm_members[labels[T]], null_model)

    active = [wc(u) for u in range(n)]
    pri = [(hash_priority(seed, it, lvl, 1, u), u) for u in range(n)]
    for _ in range(MAX_REFINE_ROUNDS):
        base_lab = flatten(units, R, G.n)
        base = score(base_lab)
        wc_now = {T: wc(T) for T in set(R)}
        prop = {}
        for u in range(n):
            if not active[u]:
                continue
            best = None
            for T in sorted({R[x] for x in adj[u] if labels[x] == labels[u]} - {R[u]}):
                if not wc_now[T]:
                    continue
                lab = list(base_lab)
                for v in units[u]:
                    lab[v] = T
                gain = score(lab) - base
                if gain > 0 and (best is None or gain > best[0]):
                    best = (gain, T)
            if best is not None:
                prop[u] = best[1]
            else:
                active[u] = False
        eligible = []
        for u, T in prop.items():
            if T not in prop:                       # the target's founder stays where it is
                eligible.append(u)
            elif prop[T] in prop and all(pri[x] < pri[u] for x in adj[u]
                                         if labels[x] == labels[u] and x in prop):
                eligible.append(u)
        stats["refine_rounds"] += 1
        if not eligible:
            break
        for u in eligible:
            T = prop[u]
            R[u] = T
            single[u] = single[T] = False
            active[u] = active[T] = False
        stats["merges"] += len(eligible)
    return R


# --------------------------------------------------------------------------- driver

def split_components(G, flat):
    """Connected components of the supra-graph restricted to entries inside one community,
    numbered by their smallest supra-node."""
    out = [-1] * G.n
    c = 0
    for v in range(G.n):
        if out[v] >= 0:
            continue
        out[v] = c
        stack = [v]
        while stack:
            x = stack.pop()
            for y in G.nbr[x]:
                if out[y] < 0 and flat[y] == flat[x]:
                    out[y] = c
                    stack.append(y)
        c += 1
    return out


def leiden(g, gamma=1, omega=1, max_levels=32, max_iterations=2, max_sweeps=0, seed=0,
           null_model=0, gamma_slices=None, initial=None, coupling=None, present_only=False):
    """Run the schedule; returns (membership, stats, trace).  trace holds one record per
    level: colour, labels at the level's start (p_in), after local moving (p_lm), R, and the
    refined sub-communities (founder -> level-0 members) with their well-connectedness.
    null_model 0 optimises Q_MS of Eq. 6; 1 the global modularity of the supra-graph; 2 the
    multislice CPM.  gamma_slices: T per-slice resolutions in place of gamma; initial: the
    first iteration's start partition."""
    G = SupraGraph(g, omega, coupling, present_only)
    if gamma_slices is not None:
        assert null_model != 1
        gamma = [Fraction(x) for x in gamma_slices]
    else:
        gamma = Fraction(gamma)
    score = GlobalScore(G, gamma) if null_model == 1 else Score(G, gamma, cpm=null_model == 2)
    if max_sweeps <= 0:
        max_sweeps = DEFAULT_SWEEPS
    iters = max_iterations if max_iterations > 0 else MAX_ITER_CAP
    iters = min(iters, MAX_ITER_CAP)
    stats = dict(sweeps=0, moves=0, sweep_cap_hits=0, refine_rounds=0, merges=0, splits=0,
                 levels_run=0, iterations_run=0, n_communities=0, colours_first=0)
    trace = []
    prev = list(range(G.n)) if initial is None else canonical([int(x) for x in initial])
    for it in range(iters):
        units = [[v] for v in range(G.n)]
        labels = canonical(prev)
        lvl = 0
        while lvl < max_levels:
            n = len(units)
            unit_of = [0] * G.n
            for u, mem in enumerate(units):
                for v in mem:
                    unit_of[v] = u
            adj = unit_adjacency(G, unit_of, n)
            colour = first_fit_colouring(adj, seed, it, lvl)
            if it == 0 and lvl == 0:
                stats["colours_first"] = max(colour) + 1 if n else 0
            rec = dict(it=it, lvl=lvl, n=n, colour=list(colour), p_in=list(labels),
                       units=[list(m) for m in units])
            trace.append(rec)
            rec["sweeps"] = local_move(G, score, units, adj, colour, labels, max_sweeps, stats)
            rec["p_lm"] = list(labels)
            if len(set(labels)) == n or lvl == max_levels - 1:
                break
            R = refine(G, score, gamma, units, adj, labels, seed, it, lvl, stats, null_model)
            rec["r"] = list(R)
            # refined sub-communities: founder -> (level-0 members, weight to the rest of the
            # community, well connected)
            comm0 = {}
            for u in range(n):
                comm0.setdefault(labels[u], set()).update(units[u])
            subs = {}
            for u in range(n):
                subs.setdefault(R[u], set()).update(units[u])
            rec["subs"] = {T: (sorted(mem), external_weight(G, mem, comm0[labels[T]]),
                               well_connected(G, gamma, mem, comm0[labels[T]], null_model))
                           for T, mem in subs.items()}
            if len(set(R)) == n:
                break
            # aggregation: one unit per refined sub-community, ordered by its smallest unit;
            # each starts in the community of its members
            founders = sorted(set(R), key=lambda T: min(u for u in range(n) if R[u] == T))
            new_units = [sorted(v for u in range(n) if R[u] == T for v in units[u])
                         for T in founders]
            new_labels = canonical([labels[T] for T in founders])
            units, labels = new_units, new_labels
            lvl += 1
        stats["levels_run"] = max(stats["levels_run"], lvl + 1)
        flat = flatten(units, labels, G.n)
        new = split_components(G, flat)
        ncomp = max(new) + 1 if G.n else 0
        stats["splits"] += ncomp - len(set(flat))
        stats["iterations_run"] = it + 1
        stats["n_communities"] = ncomp
        stable = new == prev
        prev = new
        if stable:
            break
    return prev, stats, trace
