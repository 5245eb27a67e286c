// Hand-written HIP kernels of the multislice Leiden path (gfx950, wave64, no MFMA: every
// step is a scan, a gather or a hash update, bounded by HBM bandwidth).
//
// Units are supra-nodes at level 0 and super-nodes at later levels.  Several independent
// solves can share one launch as a disjoint union: each unit knows its solve (coefficients,
// priority seed, local id offset) and its slices are global slice ids, so nothing here
// ever compares quantities of two different solves.
#pragma once
#include <type_traits>
#include <math.h>

#include "device.hpp"

namespace mslm {

typedef __int128 i128;

// Barrier for one workgroup that also makes global writes of every wave visible to the
// others: release before the barrier, and drop possibly stale vector-L1 lines after it
// (Sigma-table atomics are performed in L2).
__device__ inline void block_sync_global() {
  __threadfence();
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// ------------------------------------------------------------------ per-solve constants
struct SolveDev {
  const int64_t *p, *q, *pb, *a, *b;   // gamma = p/q, omega = a/b (reduced), pb = p*b
  const uint64_t *seedmix;             // mix64(seed)
  const int64_t *uoff;                 // first unit of the solve at the current level
  const int32_t *sfirst;               // first global slice of the solve
  const int64_t *S;                    // per global slice: 2m_s, or 1 for an empty slice
  int64_t *fallbacks;                  // exact-comparison counter per solve
  uint32_t *redo;                      // per solve: a sweep met a near-tie it could not settle
  // during local-moving sweeps: solves that take no part in the sweep (stopped, or not being
  // taken again); their units are not decided (their moves would not be applied); else nullptr
  const uint8_t *frozen;
  // a sweep replayed from a HIP graph reads the base of its fresh labels here (its launches
  // were captured once); nullptr: the base passed to the kernel
  const uint32_t *fresh;
};

__device__ inline uint32_t fresh_of(const SolveDev &sd, uint32_t fresh_base) {
  return sd.fresh ? *sd.fresh : fresh_base;
}

// ------------------------------------------------------------------ level views
// Level 0: the supra-CSR of Eq. 3 with raw weights; an entry whose column lies outside the
// unit's slice is a coupling entry of raw weight c_sr and scaled weight a * c_sr (absent when
// a == 0).
struct View0 {
  static constexpr bool kLevel0 = true;
  const int64_t *rp;
  const int32_t *col;
  const int32_t *w;        // raw weight per entry (intra w, coupling c_sr), or nullptr: all 1
  // degree in the null model of the unit's solve: the intra degree k_i^s (Eq. 6), or the
  // scaled supra-degree b*k_i^s + a*(coupling entries of the unit) (the global null model)
  const int32_t *k;
  const int32_t *uslice;   // global slice of each unit
  const int64_t *sstart;   // [slices + 1] first unit of each global slice
  const int32_t *usolve;   // solve of each unit
  // Sigma slice of each global slice (nullptr: the slice itself); a solve under the global
  // null model maps all its slices to one Sigma slice
  const int32_t *pmap;
  const int32_t *rev;      // per entry (u, x): offset of (x, u) within x's row
  int64_t N1 = 0;          // one solve: nodes per slice (slice and solve follow from the id)
  double invN1 = 0.0;      // 1 / N1
  struct Row {
    int64_t lo, hi, slo, shi, a, b;
  };
  // slice of unit v: v / N1 for one solve (a double estimate corrected by one step either
  // way, exact for every v < 2^32), else the stored slice
  __device__ int slice_of(int64_t v) const {
    if (N1 == 0) return uslice[v];
    int64_t q = (int64_t)((double)v * invN1);
    if (q * N1 > v) q--;
    else if ((q + 1) * N1 <= v) q++;
    return (int)q;
  }
  __device__ int solve_of(int64_t v) const { return N1 ? 0 : usolve[v]; }
  __device__ Row row(int64_t v, const SolveDev &sd) const {
    const int gs = slice_of(v);
    const int j = solve_of(v);
    const int64_t slo = N1 ? (int64_t)gs * N1 : sstart[gs];
    const int64_t shi = N1 ? slo + N1 : sstart[gs + 1];
    return Row{rp[v], rp[v + 1], slo, shi, sd.a[j], sd.b[j]};
  }
  __device__ int64_t wt(const Row &r, int64_t e, int32_t x) const {
    return (x >= r.slo && x < r.shi ? r.b : r.a) * (w ? (int64_t)w[e] : 1);
  }
  // neighbour of entry e and its scaled weight
  __device__ int64_t nbr(const Row &r, int64_t e, int64_t &ww) const {
    const int32_t x = col[e];
    ww = wt(r, e, x);
    return x;
  }
  __device__ int64_t orig(int64_t v) const { return v; }
  __device__ uint32_t lab_at(const uint32_t *comm, int64_t, int64_t x) const { return comm[x]; }
  __device__ int plen(int64_t v) const { return k[v] > 0 ? 1 : 0; }
  __device__ void pent(int64_t v, int, int &gs, int64_t &kk) const {
    gs = slice_of(v);
    if (pmap) gs = pmap[gs];
    kk = k[v];
  }
  __device__ int64_t degree(int64_t v) const { return rp[v + 1] - rp[v]; }
};

// Level 0 in colour-batch order, for the local-moving sweeps: the level's units are stored in
// the order of their colour batches (colour, degree bin, id), so a batch is one contiguous
// range of positions whose rows, degrees, slices and labels are read in sequence; only the
// neighbours' labels and the Sigma probes stay random.  Entries hold neighbour positions,
// with bit 31 set on the coupling entries (scaled weight a); labels and priorities keep the
// unit ids (orig), so every decision is the one the id-ordered level makes.
struct ViewP {
  static constexpr bool kLevel0 = true;
  const int64_t *rp;       // [n+1] rows by position
  const int32_t *col;      // neighbour position | coupling << 31
  const int32_t *w;        // raw intra weight per entry, or nullptr for unit weights
  const int32_t *k;        // null-model degree by position (View0::k)
  const int32_t *slice;    // Sigma slice by position
  const int32_t *solve;    // solve by position, or nullptr (one solve)
  const int32_t *uid;      // unit id by position
  // per entry, the neighbour's current label (kept up to date by the moves: a moved unit
  // writes its new label into the entries that point at it, found through prev), so the
  // decisions read labels in entry order instead of gathering them; nullptr: gather
  uint32_t *elab;
  const int32_t *prev;     // per entry (i, x): index of the entry (x, i)
  int64_t nnz;             // entries (host use)
  struct Row {
    int64_t lo, hi, a, b;
  };
  __device__ int solve_of(int64_t i) const { return solve ? solve[i] : 0; }
  __device__ Row row(int64_t i, const SolveDev &sd) const {
    const int j = solve_of(i);
    return Row{rp[i], rp[i + 1], sd.a[j], sd.b[j]};
  }
  __device__ int64_t nbr(const Row &r, int64_t e, int64_t &ww) const {
    const int32_t raw = col[e];
    ww = (raw < 0 ? r.a : r.b) * (w ? (int64_t)w[e] : 1);
    return raw & 0x7fffffff;
  }
  __device__ int64_t orig(int64_t i) const { return uid[i]; }
  __device__ uint32_t lab_at(const uint32_t *comm, int64_t e, int64_t x) const {
    return elab ? elab[e] : comm[x];
  }
  __device__ int plen(int64_t i) const { return k[i] > 0 ? 1 : 0; }
  __device__ void pent(int64_t i, int, int &gs, int64_t &kk) const {
    gs = slice[i];
    kk = k[i];
  }
  __device__ int64_t degree(int64_t i) const { return rp[i + 1] - rp[i]; }
};

// Aggregated levels: scaled int64 weights, per-unit slice profiles (global slice, degree).
struct ViewK {
  static constexpr bool kLevel0 = false;
  const int64_t *rp;
  const int32_t *col;
  const int64_t *w;
  const int64_t *pp;
  const int32_t *ps;
  const int32_t *pk;
  const int32_t *usolve;
  struct Row {
    int64_t lo, hi;
  };
  __device__ Row row(int64_t v, const SolveDev &) const { return Row{rp[v], rp[v + 1]}; }
  __device__ int64_t wt(const Row &, int64_t e, int32_t) const { return w[e]; }
  __device__ int64_t nbr(const Row &, int64_t e, int64_t &ww) const {
    ww = w[e];
    return col[e];
  }
  __device__ int64_t orig(int64_t v) const { return v; }
  __device__ uint32_t lab_at(const uint32_t *comm, int64_t, int64_t x) const { return comm[x]; }
  __device__ int solve_of(int64_t v) const { return usolve[v]; }
  __device__ int plen(int64_t v) const { return (int)(pp[v + 1] - pp[v]); }
  __device__ void pent(int64_t v, int j, int &gs, int64_t &kk) const {
    gs = ps[pp[v] + j];
    kk = pk[pp[v] + j];
  }
  __device__ int64_t degree(int64_t v) const { return rp[v + 1] - rp[v]; }
};

// ------------------------------------------------------------------ gains
// Targets: a community label, the empty community (label kNone, gain 0), or "stay" (the
// unit's own community without itself).  The value compared for unit v and target X is
//     q*W_X - p*b * sum_s k_{v,s} * y_{X,s} / S_s
// (W_X the scaled edge weight from v to X, y_{X,s} the slice-s degree of X), which orders
// targets exactly as the change of Q in Eq. 6 does (a positive multiple of it).
enum { kTarget = 0, kEmpty = 1, kStay = 2 };

struct UnitCtx {
  int64_t v;
  int j;
  uint32_t D;
  int m;          // profile length
  int gs0;        // first profile slice
  int64_t k0;     // first profile degree
  int64_t p, q, pb, S0;
};

template <class V>
__device__ inline UnitCtx unit_ctx(const V &g, const SolveDev &sd, int64_t v, uint32_t D) {
  UnitCtx u;
  u.v = v;
  u.j = g.solve_of(v);
  u.D = D;
  u.m = g.plen(v);
  u.gs0 = 0;
  u.k0 = 0;
  if (u.m > 0) g.pent(v, 0, u.gs0, u.k0);
  u.p = sd.p[u.j];
  u.q = sd.q[u.j];
  u.pb = sd.pb[u.j];
  u.S0 = u.m > 0 ? sd.S[u.gs0] : 1;
  return u;
}

__device__ inline int64_t target_y(const SliceTable &tab, int gs, int64_t k, uint32_t lab, int kind) {
  if (kind == kEmpty) return 0;
  int64_t y = tab_get(tab, gs, lab);
  return kind == kStay ? y - k : y;
}

// Level 0: one slice per unit; exact in int64 under the checked head-room precondition.
struct Score0 {
  int64_t g;
  uint32_t lab;
};

struct Policy0 {
  typedef Score0 Score;
  template <class V>
  __device__ static Score make(const V &, const UnitCtx &u, const SolveDev &, const SliceTable &tab,
                               uint32_t lab, int64_t W, int kind) {
    Score s;
    s.lab = kind == kEmpty ? kNone : lab;
    if (u.m == 0) {
      s.g = u.q * W;
    } else {
      int64_t y = target_y(tab, u.gs0, u.k0, lab, kind);
      s.g = u.q * u.S0 * W - u.pb * (u.k0 * y);
    }
    return s;
  }
  template <class V>
  __device__ static int cmp(const V &, const UnitCtx &, const SolveDev &, const SliceTable &,
                            const Score &a, const Score &b) {
    return a.g < b.g ? -1 : (a.g > b.g ? 1 : 0);
  }
  // the null term is never negative, so q*S*W bounds a target's value from above; a target
  // whose bound is strictly below the best value so far can neither win nor tie
  __device__ static bool prunable(const UnitCtx &u, int64_t W, const Score &best) {
    int64_t ub = u.m == 0 ? u.q * W : u.q * u.S0 * W;
    return ub < best.g;
  }
  __device__ static Score shfl(const Score &s, int m) {
    Score o;
    o.g = shfl_xor64(s.g, m);
    o.lab = shfl_xor32(s.lab, m);
    return o;
  }
  // the score of staying when the Sigma of the unit's own community is already known
  __device__ static Score stay_from(const UnitCtx &u, uint32_t D, int64_t W, int64_t yD) {
    Score s;
    s.lab = D;
    s.g = u.m == 0 ? u.q * W : u.q * u.S0 * W - u.pb * (u.k0 * (yD - u.k0));
    return s;
  }
};

// Aggregated levels: int128 when the unit lies in one slice, otherwise a double estimate
// with a rigorous error bound and an exact big-integer evaluation when the estimates of
// two targets are too close to order.
struct ScoreK {
  i128 ex;
  double ap, er;
  int64_t W;
  uint32_t lab;
  int kind;   // kTarget / kEmpty / kStay; +4 when the value has no null term (it is q*W)
};

template <class V>
__device__ __noinline__ int exact_big(const V &g, const UnitCtx &u, const SolveDev &sd,
                                      const SliceTable &tab, uint32_t la, int ka, int64_t Wa,
                                      uint32_t lb, int kb, int64_t Wb) {
  atomicAdd(reinterpret_cast<unsigned long long *>(sd.fallbacks + u.j), 1ull);
  ExactAcc acc;
  acc.init();
  for (int jj = 0; jj < u.m; jj++) {
    int gs;
    int64_t k;
    g.pent(u.v, jj, gs, k);
    int64_t ya = target_y(tab, gs, k, la, ka);
    int64_t yb = target_y(tab, gs, k, lb, kb);
    acc.term(k * (ya - yb), sd.S[gs]);
  }
  return acc.sign(u.q, Wa - Wb, u.pb);
}

// Exact order of two targets whose estimates cannot be told apart.  Equal per-slice terms
// (the usual case: both targets hold the same Sigma in every slice of the unit) are settled
// here, inline; only a genuine near-tie calls the out-of-line big-integer evaluation (a call
// spills the caller's registers, so it must stay off the common path).
template <class V>
__device__ inline int exact_cmp(const V &g, const UnitCtx &u, const SolveDev &sd,
                                const SliceTable &tab, uint32_t la, int ka, int64_t Wa,
                                uint32_t lb, int kb, int64_t Wb) {
  bool same = true;
  for (int jj = 0; jj < u.m && same; jj++) {
    int gs;
    int64_t k;
    g.pent(u.v, jj, gs, k);
    same = target_y(tab, gs, k, la, ka) == target_y(tab, gs, k, lb, kb);
  }
  if (same) return Wa > Wb ? 1 : (Wa < Wb ? -1 : 0);
  return exact_big(g, u, sd, tab, la, ka, Wa, lb, kb, Wb);
}

// The same order for the sweeps that run without the big-integer path (it needs per-lane
// scratch memory, which slows every launch of a kernel that contains it): equal per-slice
// terms are settled here as well; a genuine near-tie raises its solve's redo flag and gets a
// provisional answer, and the host takes that solve's sweep again with the exact kernels.
template <class V>
__device__ inline int exact_cmp_flag(const V &g, const UnitCtx &u, const SolveDev &sd,
                                     const SliceTable &tab, uint32_t la, int ka, int64_t Wa,
                                     uint32_t lb, int kb, int64_t Wb) {
  bool same = true;
  for (int jj = 0; jj < u.m && same; jj++) {
    int gs;
    int64_t k;
    g.pent(u.v, jj, gs, k);
    same = target_y(tab, gs, k, la, ka) == target_y(tab, gs, k, lb, kb);
  }
  if (!same) atomicOr(sd.redo + u.j, 1u);
  return Wa > Wb ? 1 : (Wa < Wb ? -1 : 0);
}

// Exact: near-ties go to the big-integer evaluation; otherwise they raise the redo flag.
template <bool Exact>
struct PolicyKT {
  typedef ScoreK Score;
  template <class V>
  __device__ static Score make(const V &g, const UnitCtx &u, const SolveDev &sd,
                               const SliceTable &tab, uint32_t lab, int64_t W, int kind) {
    Score s;
    s.lab = kind == kEmpty ? kNone : lab;
    s.kind = kind;
    s.W = W;
    s.ex = 0;
    s.ap = 0;
    s.er = 0;
    if (u.m <= 1) {
      i128 val = (i128)u.q * W;
      if (u.m == 1) {
        int64_t y = target_y(tab, u.gs0, u.k0, lab, kind);
        val = val * u.S0 - (i128)u.pb * (i128)(u.k0 * y);
      }
      s.ex = val;
    } else if (kind == kEmpty) {
      // every null term of the empty community is 0: the value is q*W, no slice to visit
      finish(u, W, 0.0, 0.0, s);
    } else {
      double acc = 0.0, mag = 0.0;
      for (int jj = 0; jj < u.m; jj++) {
        int gs;
        int64_t k;
        g.pent(u.v, jj, gs, k);
        int64_t y = target_y(tab, gs, k, lab, kind);
        double t = (double)(k * y) / (double)sd.S[gs];
        acc += t;
        mag += fabs(t);
      }
      finish(u, W, acc, mag, s);
    }
    return s;
  }
  // estimate and error bound from the summed null terms (any summation order)
  __device__ static void finish(const UnitCtx &u, int64_t W, double acc, double mag, Score &s) {
    double qw = (double)u.q * (double)W;
    s.ap = qw - (double)u.pb * acc;
    s.er = (double)(u.m + 8) * 0x1p-50 * (fabs(qw) + (double)u.pb * mag);
    if (mag == 0.0 || u.pb == 0) s.kind |= 4;
  }
  template <class V>
  __device__ static int cmp(const V &g, const UnitCtx &u, const SolveDev &sd, const SliceTable &tab,
                            const Score &a, const Score &b) {
    if (u.m <= 1) return a.ex < b.ex ? -1 : (a.ex > b.ex ? 1 : 0);
    if (a.lab == b.lab && a.kind == b.kind && a.W == b.W) return 0;   // the same target
    if ((a.kind & 4) && (b.kind & 4)) return a.W < b.W ? -1 : (a.W > b.W ? 1 : 0);   // both q*W
    double d = a.ap - b.ap;
    if (fabs(d) > 2.0 * (a.er + b.er)) return d > 0 ? 1 : -1;
    if constexpr (Exact)
      return exact_cmp(g, u, sd, tab, a.lab, a.kind & 3, a.W, b.lab, b.kind & 3, b.W);
    else
      return exact_cmp_flag(g, u, sd, tab, a.lab, a.kind & 3, a.W, b.lab, b.kind & 3, b.W);
  }
  __device__ static bool prunable(const UnitCtx &u, int64_t W, const Score &best) {
    if (u.m <= 1) {
      i128 ub = (i128)u.q * W * (u.m ? u.S0 : 1);
      return ub < best.ex;
    }
    // q*W rounded up versus a rigorous lower bound of the best value
    double ub = (double)u.q * (double)W * (1.0 + 0x1p-48);
    return ub < best.ap - best.er;
  }
  __device__ static Score shfl(const Score &s, int m) {
    Score o;
    uint64_t lo = (uint64_t)s.ex, hi = (uint64_t)(s.ex >> 64);
    lo = (uint64_t)shfl_xor64((int64_t)lo, m);
    hi = (uint64_t)shfl_xor64((int64_t)hi, m);
    o.ex = (i128)(((unsigned __int128)hi << 64) | lo);
    o.ap = __shfl_xor(s.ap, m, 64);
    o.er = __shfl_xor(s.er, m, 64);
    o.W = shfl_xor64(s.W, m);
    o.lab = shfl_xor32(s.lab, m);
    o.kind = __shfl_xor(s.kind, m, 64);
    return o;
  }
};
using PolicyK = PolicyKT<true>;
using PolicyKF = PolicyKT<false>;
// policies of units spanning several slices (cooperative evaluation applies to them)
template <class P>
struct IsMulti : std::false_type {};
template <bool E>
struct IsMulti<PolicyKT<E>> : std::true_type {};

// Aggregated levels, units in at most one slice: the same int128 value as PolicyK's
// single-slice case without the multi-slice machinery (far fewer registers).
struct Score1 {
  i128 ex;
  uint32_t lab;
};
struct PolicyK1 {
  typedef Score1 Score;
  template <class V>
  __device__ static Score make(const V &, const UnitCtx &u, const SolveDev &,
                               const SliceTable &tab, uint32_t lab, int64_t W, int kind) {
    Score s;
    s.lab = kind == kEmpty ? kNone : lab;
    i128 val = (i128)u.q * W;
    if (u.m == 1) {
      int64_t y = target_y(tab, u.gs0, u.k0, lab, kind);
      val = val * u.S0 - (i128)u.pb * (i128)(u.k0 * y);
    }
    s.ex = val;
    return s;
  }
  template <class V>
  __device__ static int cmp(const V &, const UnitCtx &, const SolveDev &, const SliceTable &,
                            const Score &a, const Score &b) {
    return a.ex < b.ex ? -1 : (a.ex > b.ex ? 1 : 0);
  }
  __device__ static bool prunable(const UnitCtx &u, int64_t W, const Score &best) {
    i128 ub = (i128)u.q * W * (u.m ? u.S0 : 1);
    return ub < best.ex;
  }
  __device__ static Score shfl(const Score &s, int m) {
    Score o;
    uint64_t lo = (uint64_t)s.ex, hi = (uint64_t)(s.ex >> 64);
    lo = (uint64_t)shfl_xor64((int64_t)lo, m);
    hi = (uint64_t)shfl_xor64((int64_t)hi, m);
    o.ex = (i128)(((unsigned __int128)hi << 64) | lo);
    o.lab = shfl_xor32(s.lab, m);
    return o;
  }
};

template <class P, class V>
__device__ inline bool better(const V &g, const UnitCtx &u, const SolveDev &sd, const SliceTable &tab,
                              const typename P::Score &a, const typename P::Score &b) {
  int c = P::cmp(g, u, sd, tab, a, b);
  return c > 0 || (c == 0 && a.lab < b.lab);
}

template <class P, class V>
__device__ inline typename P::Score wave_best(const V &g, const UnitCtx &u, const SolveDev &sd,
                                              const SliceTable &tab, typename P::Score s) {
  for (int m = 32; m >= 1; m >>= 1) {
    typename P::Score o = P::shfl(s, m);
    if (better<P>(g, u, sd, tab, o, s)) s = o;
  }
  return s;
}

// ------------------------------------------------------------------ accumulation tables
// LDS accumulation table with the list of its occupied slots (L holds at most the number of
// distinct keys: the unit's degree bound for its bin, and never more than the table size).
struct LdsTab {
  uint32_t *K;
  int64_t *V;
  int lg;
  uint16_t *L;
  int *n;
  __device__ int size() const { return 1 << lg; }
  __device__ void add(uint32_t lab, int64_t w) const { lds_add_listed(K, V, lg, lab, w, L, n); }
  __device__ int64_t get(uint32_t lab) const { return lds_get(K, V, lg, lab); }
  __device__ int count() const { return *(volatile int *)n; }
  __device__ int slot(int i) const { return L[i]; }
  __device__ void reset(int rank) const {
    if (rank == 0) *n = 0;
  }
};
struct GTab {
  uint32_t *K;
  int64_t *V;
  int lg;
  __device__ int size() const { return 1 << lg; }
  __device__ void add(uint32_t lab, int64_t w) const {
    gtab_add(K, V, (1u << lg) - 1, 32 - lg, lab, w);
  }
  __device__ int64_t get(uint32_t lab) const {
    return gtab_get(K, V, (1u << lg) - 1, 32 - lg, lab);
  }
  __device__ int count() const { return 1 << lg; }
  __device__ int slot(int i) const { return i; }
  __device__ void reset(int) const {}
};

// Group = the threads cooperating on one unit: one wave, or a whole block.
struct WaveGrp {
  __device__ int rank() const { return threadIdx.x & 63; }
  __device__ int size() const { return 64; }
  __device__ void sync() const { wave_sync(); }
};
struct BlockGrp {
  __device__ int rank() const { return threadIdx.x; }
  __device__ int size() const { return blockDim.x; }
  __device__ void sync() const { __syncthreads(); }
};
// A block whose accumulation table lives in global memory: its barriers must also make the
// plain stores and atomics of every wave visible to the others.
struct BlockGrpG {
  __device__ int rank() const { return threadIdx.x; }
  __device__ int size() const { return blockDim.x; }
  __device__ void sync() const { block_sync_global(); }
};

// Reduce a score over the group; every thread gets the result.
template <class P, class V>
__device__ inline typename P::Score group_best(WaveGrp, const V &g, const UnitCtx &u,
                                               const SolveDev &sd, const SliceTable &tab,
                                               typename P::Score s, typename P::Score *) {
  return wave_best<P>(g, u, sd, tab, s);
}
template <class P, class V>
__device__ inline typename P::Score group_best(BlockGrp grp, const V &g, const UnitCtx &u,
                                               const SolveDev &sd, const SliceTable &tab,
                                               typename P::Score s, typename P::Score *red) {
  s = wave_best<P>(g, u, sd, tab, s);
  int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) red[wv] = s;
  grp.sync();
  typename P::Score b = red[0];
  for (int i = 1; i < nw; i++)
    if (better<P>(g, u, sd, tab, red[i], b)) b = red[i];
  grp.sync();
  return b;
}

template <class P, class V>
__device__ inline typename P::Score group_best(BlockGrpG, const V &g, const UnitCtx &u,
                                               const SolveDev &sd, const SliceTable &tab,
                                               typename P::Score s, typename P::Score *red) {
  return group_best<P>(BlockGrp(), g, u, sd, tab, s, red);   // LDS only
}

// heaviest entry of the accumulation table over the group (ties to the lower label), skipping
// one excluded label; kNone when there is none
template <class Grp, class Tab>
__device__ inline void group_heaviest(Grp grp, const Tab &tab, uint32_t skip, const uint8_t *ok,
                                      int64_t &W, uint32_t &lab, int64_t *sred, uint32_t *lred) {
  const int r = grp.rank(), gsz = grp.size();
  W = -1;
  lab = kNone;
  const int nc = tab.count();
  for (int i = r; i < nc; i += gsz) {
    const int h = tab.slot(i);
    uint32_t key = tab.K[h];
    if (key == 0 || key - 1 == skip) continue;
    if (ok && !ok[key - 1]) continue;
    int64_t w = tab.V[h];
    if (w > W || (w == W && key - 1 < lab)) {
      W = w;
      lab = key - 1;
    }
  }
  for (int m = 32; m >= 1; m >>= 1) {
    int64_t w2 = shfl_xor64(W, m);
    uint32_t l2 = shfl_xor32(lab, m);
    if (w2 > W || (w2 == W && l2 < lab)) {
      W = w2;
      lab = l2;
    }
  }
  if (gsz > 64) {
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
      sred[wv] = W;
      lred[wv] = lab;
    }
    grp.sync();
    for (int i = 0; i < nw; i++)
      if (sred[i] > W || (sred[i] == W && lred[i] < lab)) {
        W = sred[i];
        lab = lred[i];
      }
    grp.sync();
  }
}

// ------------------------------------------------------------------ cooperative evaluation
// Units spanning many slices: the lanes of an aligned subgroup of mp = 2^ceil(log2 m) lanes
// hold one profile slice each (slice, degree, S and that slice's Sigma sub-table, loaded
// once per unit), so one candidate costs one independent lookup per lane and a butterfly
// sum instead of m dependent lookups in one lane.
constexpr int kCoopMinM = 4;
__host__ __device__ inline int coop_width(int m) {
  int mp = 4;
  while (mp < m) mp <<= 1;
  return mp;
}

struct CoopLane {
  int mp;          // subgroup width
  int j;           // this lane's slice index within the profile (valid when j < m)
  bool valid;
  int64_t k;       // unit degree in that slice
  double S;        // slice denominator
  const uint64_t *sub;
  uint32_t mask;
  int shift;
};

template <class V>
__device__ inline CoopLane coop_lane(const V &g, const UnitCtx &u, const SolveDev &sd,
                                     const SliceTable &tab, int rank) {
  CoopLane c;
  c.mp = coop_width(u.m);
  c.j = rank & (c.mp - 1);
  c.valid = c.j < u.m;
  c.k = 0;
  c.S = 1.0;
  c.sub = tab.slots;
  c.mask = 0;
  c.shift = 32;
  if (c.valid) {
    int gs;
    g.pent(u.v, c.j, gs, c.k);
    c.S = (double)sd.S[gs];
    c.shift = tab.shift[gs];
    c.mask = 0xffffffffu >> c.shift;
    c.sub = tab.slots + tab.base[gs];
  }
  return c;
}

// This lane's slice Sigma of U targets (the raw table value, 0 when absent or when the lane
// holds no slice); the U first probes are issued together so that their latencies overlap.
template <int U>
__device__ inline void coop_lookup(const CoopLane &c, const uint32_t *lab, const bool *ok,
                                   int64_t *y) {
  uint64_t e[U];
  uint32_t h[U];
  for (int k = 0; k < U; k++) {
    const bool on = c.valid && ok[k];
    h[k] = on ? fib_hash(lab[k], c.shift) : 0u;
    e[k] = on ? c.sub[h[k]] : 0ull;
  }
  for (int k = 0; k < U; k++) {
    int64_t yy = 0;
    if (c.valid && ok[k]) {
      const uint32_t key = lab[k] + 1;
      for (;;) {
        const uint32_t kk = (uint32_t)e[k];
        if (kk == key) {
          yy = (int32_t)(e[k] >> 32);
          break;
        }
        if (kk == 0) break;
        h[k] = (h[k] + 1) & c.mask;
        e[k] = c.sub[h[k]];
      }
    }
    y[k] = yy;
  }
}

// Score of one target from this lane's Sigma y of it, identical on every lane of the subgroup.
__device__ inline ScoreK coop_score(const UnitCtx &u, const CoopLane &c, uint32_t lab, int64_t W,
                                    int64_t y, int kind) {
  ScoreK s;
  s.lab = kind == kEmpty ? kNone : lab;
  s.kind = kind;
  s.W = W;
  s.ex = 0;
  double t = 0.0;
  if (c.valid && kind != kEmpty) {
    if (kind == kStay) y -= c.k;
    t = (double)(c.k * y) / c.S;
  }
  double acc = t, mag = fabs(t);
  for (int o = 1; o < c.mp; o <<= 1) {
    acc += __shfl_xor(acc, o, 64);
    mag += __shfl_xor(mag, o, 64);
  }
  s.ap = 0;
  s.er = 0;
  PolicyK::finish(u, W, acc, mag, s);
  return s;
}

__device__ inline ScoreK coop_make(const UnitCtx &u, const CoopLane &c, uint32_t lab, int64_t W,
                                   int kind) {
  const bool ok = kind != kEmpty;
  int64_t y = 0;
  coop_lookup<1>(c, &lab, &ok, &y);
  return coop_score(u, c, lab, W, y, kind);
}

// Candidates evaluated per subgroup turn (their Sigma lookups in flight together).
constexpr int kCoopBatch = 4;

// ------------------------------------------------------------------ local moving
// One unit: accumulate neighbour-community weights in the table, evaluate every candidate
// community (strictly better gain wins, ties to the lower label, the empty community has
// gain 0 and label +inf), and decide a move only when it beats staying strictly.
// Profiling counters of the decision kernels (filled only when profiling is requested):
// [0] units decided, [1] entries scanned, [2] candidate communities evaluated.
struct LmCounters {
  unsigned long long *c;
};

// Candidates of one unit shared by B blocks (latency mode, units spanning several slices with
// many candidates): each block builds the unit's whole table, evaluates the heaviest candidate
// (it seeds pruning) and the candidates whose label hashes to its part, and publishes its
// best; the block that finishes last reduces the B bests in the same total order (value, then
// label) and decides.  The result is the one a single block reaches.
struct CandSplit {
  int part = 0, B = 1;
  uint16_t *L2 = nullptr;   // LDS list of this block's candidate slots
  int *n2 = nullptr;
  ScoreK *parts = nullptr;  // [B] published bests of this unit
  uint32_t *done = nullptr; // blocks of this unit finished (the last one resets it to 0)
  int *last = nullptr;      // LDS: this block reduces
  __device__ bool mine(uint32_t lab) const {
    return (int)(((uint64_t)(lab * 2654435769u) * (uint32_t)B) >> 32) == part;
  }
};

// This block's list of its own candidates (B > 1), else the table itself.
template <class Grp, class Tab>
__device__ inline Tab split_view(Grp grp, const Tab &tab, const CandSplit &cs) {
  Tab ctab = tab;
  if constexpr (std::is_same<Tab, LdsTab>::value) {
    if (cs.B > 1) {
      const int r = grp.rank(), gsz = grp.size();
      if (r == 0) *cs.n2 = 0;
      grp.sync();
      const int nc = tab.count();
      for (int i = r; i < nc; i += gsz) {
        const int h = tab.slot(i);
        const uint32_t key = tab.K[h];
        if (key != 0 && cs.mine(key - 1)) cs.L2[atomicAdd(cs.n2, 1)] = (uint16_t)h;
      }
      grp.sync();
      ctab.L = cs.L2;
      ctab.n = cs.n2;
    }
  }
  return ctab;
}

// Publish this block's best; true in the block that finishes last, whose `best` is then the
// best over all B blocks.
template <class P, class V, class Grp>
__device__ inline bool split_reduce(Grp grp, const V &g, const UnitCtx &u, const SolveDev &sd,
                                    const SliceTable &sig, const CandSplit &cs,
                                    typename P::Score &best) {
  if constexpr (std::is_same<typename P::Score, ScoreK>::value) {
    if (grp.rank() == 0) {
      cs.parts[cs.part] = best;
      __threadfence();
      const uint32_t old = atomicAdd(cs.done, 1u);
      *cs.last = old == (uint32_t)(cs.B - 1);
    }
    grp.sync();
    const bool last = *cs.last != 0;
    grp.sync();
    if (!last) return false;
    __threadfence();
    for (int i = 0; i < cs.B; i++) {
      const ScoreK o = cs.parts[i];
      if (better<P>(g, u, sd, sig, o, best)) best = o;
    }
    if (grp.rank() == 0) *cs.done = 0;
    return true;
  } else {
    return true;
  }
}

template <class P, class Grp, class Tab, class V>
__device__ inline uint32_t lm_unit_coop(Grp grp, Tab tab, const V &g, const SolveDev &sd,
                                        const UnitCtx &u, const SliceTable &sig,
                                        uint32_t fresh_base, typename P::Score *red,
                                        LmCounters pc, typename P::Score best, int64_t hW,
                                        uint32_t hL, const CandSplit &cs) {
  const int r = grp.rank(), gsz = grp.size();
  const CoopLane c = coop_lane(g, u, sd, sig, r);
  const Tab ctab = split_view(grp, tab, cs);
  const int sub = r / c.mp, nsub = gsz / c.mp;
  int ncand = 0;
  if (hL != kNone) {
    ScoreK s = coop_make(u, c, hL, hW, kTarget);
    if (better<P>(g, u, sd, sig, s, best)) best = s;
    ncand = r == 0 && cs.part == 0;
  }
  // subgroups take table slots kCoopBatch at a time; every lane runs the same turns
  const int nc = ctab.count();
  for (int i0 = 0; i0 < nc; i0 += nsub * kCoopBatch) {
    uint32_t lab[kCoopBatch];
    int64_t W[kCoopBatch], y[kCoopBatch];
    bool ok[kCoopBatch];
    for (int k = 0; k < kCoopBatch; k++) {
      const int i = i0 + k * nsub + sub;
      const int h = i < nc ? ctab.slot(i) : 0;
      const uint32_t key = i < nc ? tab.K[h] : 0u;
      lab[k] = key - 1;
      ok[k] = key != 0 && key - 1 != u.D && key - 1 != hL;
      W[k] = ok[k] ? tab.V[h] : 0;
      ok[k] = ok[k] && !P::prunable(u, W[k], best);
    }
    coop_lookup<kCoopBatch>(c, lab, ok, y);
    for (int k = 0; k < kCoopBatch; k++) {
      if (!ok[k]) continue;
      ncand += c.j == 0;
      ScoreK s = coop_score(u, c, lab[k], W[k], y[k], kTarget);
      if (better<P>(g, u, sd, sig, s, best)) best = s;
    }
  }
  if (pc.c) {
    if (ncand) atomicAdd(pc.c + 2, (unsigned long long)ncand);
    if (r == 0 && cs.part == 0) {
      atomicAdd(pc.c + 0, 1ull);
      atomicAdd(pc.c + 1, (unsigned long long)g.degree(u.v));
    }
  }
  best = group_best<P>(grp, g, u, sd, sig, best, red);
  if (cs.B > 1 && !split_reduce<P>(grp, g, u, sd, sig, cs, best)) return kNone;
  const int64_t wD = tab.get(u.D);
  const ScoreK stay = coop_make(u, c, u.D, wD, kStay);
  uint32_t out = kNone;
  if (P::cmp(g, u, sd, sig, best, stay) > 0)
    out = best.lab == kNone ? fresh_of(sd, fresh_base) + (uint32_t)g.orig(u.v) : best.lab;
  grp.sync();
  return out;
}

template <class P, class V, class Grp, class Tab>
__device__ inline uint32_t lm_unit(Grp grp, Tab tab, const V &g, const SolveDev &sd, int64_t v,
                                   const uint32_t *comm, const SliceTable &sig, uint32_t fresh_base,
                                   typename P::Score *red, LmCounters pc, int64_t *sredW = nullptr,
                                   uint32_t *sredL = nullptr, const CandSplit &cs = CandSplit()) {
  const int r = grp.rank(), gsz = grp.size();
  if (sd.frozen && sd.frozen[g.solve_of(v)]) {   // its solve is out of this sweep
    if (cs.B > 1 && r == 0) *cs.last = 0;
    return kNone;
  }
  for (int i = r; i < tab.size(); i += gsz) {
    tab.K[i] = 0;
    tab.V[i] = 0;
  }
  tab.reset(r);
  grp.sync();
  const uint32_t D = comm[v];
  typename V::Row row = g.row(v, sd);
  // kGather entries per lane at a time: their column and label loads go out together
  constexpr int kGather = 4;
  for (int64_t e0 = row.lo + r; e0 < row.hi; e0 += (int64_t)kGather * gsz) {
    int64_t w[kGather];
    uint32_t lab[kGather];
#pragma unroll
    for (int t = 0; t < kGather; t++) {
      const int64_t e = e0 + (int64_t)t * gsz;
      w[t] = 0;
      int64_t x = 0;
      if (e < row.hi) x = g.nbr(row, e, w[t]);
      lab[t] = w[t] != 0 ? g.lab_at(comm, e, x) : kNone;
    }
#pragma unroll
    for (int t = 0; t < kGather; t++)
      if (lab[t] != kNone) tab.add(lab[t], w[t]);
  }
  grp.sync();
  UnitCtx u = unit_ctx(g, sd, v, D);
  typename P::Score best = P::make(g, u, sd, sig, kNone, 0, kEmpty);
  // the heaviest candidate first: its value is a strong bound for pruning the others
  int64_t hW;
  uint32_t hL;
  group_heaviest(grp, tab, D, (const uint8_t *)nullptr, hW, hL, sredW, sredL);
  if constexpr (!V::kLevel0 && IsMulti<P>::value) {
    if (u.m >= kCoopMinM)
      return lm_unit_coop<P>(grp, tab, g, sd, u, sig, fresh_base, red, pc, best, hW, hL, cs);
  }
  int ncand = 0;
  if (hL != kNone) {
    typename P::Score s = P::make(g, u, sd, sig, hL, hW, kTarget);
    if (better<P>(g, u, sd, sig, s, best)) best = s;
    ncand = r == 0 && cs.part == 0;
  }
  const Tab ctab = split_view(grp, tab, cs);
  const int nc = ctab.count();
  for (int i = r; i < nc; i += gsz) {
    const int h = ctab.slot(i);
    uint32_t key = tab.K[h];
    if (key == 0 || key - 1 == D || key - 1 == hL) continue;
    if (P::prunable(u, tab.V[h], best)) continue;
    ncand++;
    typename P::Score s = P::make(g, u, sd, sig, key - 1, tab.V[h], kTarget);
    if (better<P>(g, u, sd, sig, s, best)) best = s;
  }
  if (pc.c) {
    if (ncand) atomicAdd(pc.c + 2, (unsigned long long)ncand);
    if (r == 0 && cs.part == 0) {
      atomicAdd(pc.c + 0, 1ull);
      atomicAdd(pc.c + 1, (unsigned long long)(row.hi - row.lo));
    }
  }
  best = group_best<P>(grp, g, u, sd, sig, best, red);
  if (cs.B > 1 && !split_reduce<P>(grp, g, u, sd, sig, cs, best)) {
    grp.sync();
    return kNone;
  }
  int64_t wD = tab.get(D);
  typename P::Score stay = P::make(g, u, sd, sig, D, wD, kStay);
  uint32_t out = kNone;
  if (P::cmp(g, u, sd, sig, best, stay) > 0)
    out = best.lab == kNone ? fresh_of(sd, fresh_base) + (uint32_t)g.orig(v) : best.lab;
  grp.sync();
  return out;
}

constexpr int kWaveLg = 9;        // 512-slot LDS table per wave: units of degree <= 256
constexpr int kBlockLg = 13;      // 8192-slot LDS table per block: degree <= 4096
constexpr int kSmallBlockLg = 11; // 2048-slot LDS table per 256-thread block: degree <= 1024
constexpr int kWaveMaxDeg = 256;
constexpr int kSmallBlockMaxDeg = 1024;
constexpr int kBlockMaxDeg = 4096;

// Degree bins of the decision kernels: 0..3 lane groups of 4/8/16/32 lanes per unit (one
// adjacency entry per lane, equal labels merged in an LDS table), 4 a wave with an LDS
// table, 5 a block with an LDS table, 6 a block with a global-memory table.
constexpr int kNumBins = 8;
constexpr int kBinWaveLast = 4;          // bins 0..4 fit a wave's table
constexpr int kBinGtab = kNumBins - 1;   // global-memory tables
// Colour batches are bucketed by (colour, slot): slots 0..7 are the degree bins; at aggregated
// levels units in at most one slice use slots 8..15 and the lean single-slice decision.
constexpr int kBatchShift = 4;
constexpr int kBatchSlots = 1 << kBatchShift;
__host__ __device__ inline uint32_t degree_bin(int64_t d) {
  return d <= 4 ? 0u : d <= 8 ? 1u : d <= 16 ? 2u : d <= 32 ? 3u
       : d <= kWaveMaxDeg ? 4u : d <= kSmallBlockMaxDeg ? 5u : d <= kBlockMaxDeg ? 6u : 7u;
}
// Bin of a unit of degree d in m slices: by degree; a unit in kCoopMinM or more slices is
// evaluated cooperatively by a wave, or by a block when its (candidate x slice) work exceeds
// 64 turns of a wave.  A bin never receives a degree above its table's capacity
// (bin_fits checks that on the host before the first solve).
__host__ __device__ inline uint32_t bin_of(int64_t d, int m) {
  if (m < kCoopMinM) return degree_bin(d);
  const int64_t work = d * coop_width(m);
  if (d > kBlockMaxDeg) return 7u;
  if (d <= kWaveMaxDeg && work <= 64 * 64) return 4u;
  if (d <= kSmallBlockMaxDeg && work <= 256 * 64) return 5u;
  return 6u;
}
__host__ __device__ inline bool bin_fits(int64_t d, uint32_t bin) {
  const int64_t cap[kNumBins] = {4, 8, 16, 32, kWaveMaxDeg, kSmallBlockMaxDeg, kBlockMaxDeg,
                                 INT64_MAX};
  return bin < (uint32_t)kNumBins && d <= cap[bin];
}
__device__ inline uint32_t unit_bin(const View0 &g, int64_t v) { return degree_bin(g.degree(v)); }
__device__ inline uint32_t unit_bin(const ViewK &g, int64_t v) {
  return bin_of(g.degree(v), g.plen(v));
}
__device__ inline uint32_t batch_slot(const View0 &g, int64_t v) { return unit_bin(g, v); }
__device__ inline uint32_t batch_slot(const ViewK &g, int64_t v) {
  return unit_bin(g, v) + (g.plen(v) <= 1 ? (uint32_t)kNumBins : 0u);
}

// Units of degree <= G: G lanes per unit, one adjacency entry per lane; the group merges
// equal community labels in a 2G-slot LDS table per group (the lane that claims a label's slot
// leads it), every leader evaluates its community, and the group reduces to the best.  lk/lv:
// the block's LDS, 128 slots per wave.
template <class P, class V, int G>
__device__ inline void lm_group_block(const V &g, const SolveDev &sd, const int32_t *units,
                                      int64_t count, const uint32_t *comm, const SliceTable &sig,
                                      uint32_t *target, uint32_t fresh_base, LmCounters pc,
                                      int64_t blk, uint32_t *lk, int64_t *lv) {
  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);
  const int gbase = lane & ~(G - 1);
  const int64_t idx = (blk * blockDim.x + threadIdx.x) / G;
  if (idx >= count) return;   // whole groups leave together; shuffles stay inside a group
  const int64_t v = units[idx];
  if (sd.frozen && sd.frozen[g.solve_of(v)]) return;   // its solve is out of this sweep
  const uint32_t D = comm[v];
  typename V::Row row = g.row(v, sd);
  UnitCtx u = unit_ctx(g, sd, v, D);
  // level 0: the lookup of the own community's Sigma goes out with the neighbour gathers
  int64_t yD = 0;
  if constexpr (std::is_same<P, Policy0>::value)
    if (gl == 0 && u.m > 0) yD = tab_get(sig, u.gs0, D);
  const int64_t e = row.lo + gl;
  uint32_t c = kNone;
  int64_t w = 0;
  if (e < row.hi) {
    const int64_t x = g.nbr(row, e, w);
    if (w != 0) c = g.lab_at(comm, e, x);
  }
  int64_t wsum = 0, wD = 0;
  bool leader = false;
  {
    constexpr int kSlots = 2 * G;
    uint32_t *sk = lk + (threadIdx.x >> 6) * 128 + (gbase / G) * kSlots;
    unsigned long long *sv =
        reinterpret_cast<unsigned long long *>(lv) + (threadIdx.x >> 6) * 128 + (gbase / G) * kSlots;
    sk[gl] = 0u;
    sk[gl + G] = 0u;
    sv[gl] = 0ull;
    sv[gl + G] = 0ull;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the clears land before the claims
    int h = -1;
    if (c != kNone) {
      const uint32_t key = c + 1;
      uint32_t hh = (c * 2654435769u) >> (32 - __builtin_ctz(kSlots));
      for (;;) {
        const uint32_t prev = atomicCAS(sk + hh, 0u, key);
        if (prev == 0u || prev == key) {
          leader = prev == 0u;
          break;
        }
        hh = (hh + 1) & (kSlots - 1);
      }
      h = (int)hh;
      atomicAdd(sv + hh, (unsigned long long)w);
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);
    if (leader) wsum = (int64_t)sv[h];
    if (gl == 0) {   // the own community's weight
      const uint32_t key = D + 1;
      uint32_t hh = (D * 2654435769u) >> (32 - __builtin_ctz(kSlots));
      for (int probes = 0; probes < kSlots; probes++) {
        const uint32_t k = sk[hh];
        if (k == key) {
          wD = (int64_t)sv[hh];
          break;
        }
        if (k == 0u) break;
        hh = (hh + 1) & (kSlots - 1);
      }
    }
  }
  typename P::Score best = P::make(g, u, sd, sig, kNone, 0, kEmpty);
  const bool cand = leader && c != D;
  if (cand) {
    typename P::Score s = P::make(g, u, sd, sig, c, wsum, kTarget);
    if (better<P>(g, u, sd, sig, s, best)) best = s;
  }
  for (int m = G / 2; m >= 1; m >>= 1) {
    typename P::Score o = P::shfl(best, m);
    if (better<P>(g, u, sd, sig, o, best)) best = o;
  }
  if (pc.c) {
    unsigned long long nc = __popcll(__ballot(cand) & (((G == 64) ? ~0ull : ((1ull << G) - 1)) << gbase));
    if (gl == 0) {
      atomicAdd(pc.c + 0, 1ull);
      atomicAdd(pc.c + 1, (unsigned long long)(row.hi - row.lo));
      if (nc) atomicAdd(pc.c + 2, nc);
    }
  }
  if (gl == 0) {
    typename P::Score stay;
    if constexpr (std::is_same<P, Policy0>::value) stay = Policy0::stay_from(u, D, wD, yD);
    else stay = P::make(g, u, sd, sig, D, wD, kStay);
    uint32_t out = kNone;
    if (P::cmp(g, u, sd, sig, best, stay) > 0)
      out = best.lab == kNone ? fresh_of(sd, fresh_base) + (uint32_t)g.orig(v) : best.lab;
    target[idx] = out;
  }
}

// One slice's Sigma sub-table, resolved once per unit (the probes of the unit's own community
// and of its candidates all go to it).
struct SubTab {
  const uint64_t *sub;
  int sh;
  __device__ void open(const SliceTable &t, int s) {
    sh = t.shift[s];
    sub = t.slots + t.base[s];
  }
  // first probe: its slot and entry (issued for several units before any is resolved)
  __device__ uint64_t first(uint32_t label, uint32_t &h) const {
    h = fib_hash(label, sh);
    return sub[h];
  }
  // the value of `label` from its first probe, continuing the linear probe when needed
  __device__ int64_t resolve(uint32_t label, uint32_t h, uint64_t e) const {
    const uint32_t key = label + 1, mask = 0xffffffffu >> sh;
    for (;;) {
      const uint32_t k = (uint32_t)e;
      if (k == key) return (int32_t)(e >> 32);
      if (k == 0) return 0;
      h = (h + 1) & mask;
      e = sub[h];
    }
  }
};

// Level 0 in colour-batch order, units of degree <= G, Policy0.  Each group of G lanes decides
// U units in lockstep (their dependent loads in flight together; one unit measured fastest, at
// 8 waves per SIMD); a batch segment is a range of positions, so a unit's position is computed,
// not loaded.  Equal neighbour labels are merged in a small LDS table per group (a claim, an
// add, a read) rather than by G rounds of shuffles.  Entry weights travel as 32-bit raw values
// (coupling entries flagged in bit 31) and are scaled once per candidate:
// W = b * (raw intra weight) + a * (coupling entries).  Every decision equals
// lm_group_block's with Policy0: the same candidates and values (the best under the same total
// order).
template <int G, int U, bool kOne, bool kCopy>
__device__ inline void lm0_lockstep(const ViewP &g, const SolveDev &sd, int64_t first,
                                    int64_t count, const uint32_t *comm, const SliceTable &sig,
                                    uint32_t *target, uint32_t fresh_base, LmCounters pc,
                                    int64_t blk, uint32_t *lm0_keys,
                                    unsigned long long *lm0_vals) {
  constexpr int kGroups = 256 / G;
  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);
  const int gbase = lane & ~(G - 1);
  const int64_t base = blk * (int64_t)(kGroups * U) + threadIdx.x / G;
  if (base >= count) return;   // whole groups leave together
  int64_t pos[U];
  bool live[U];
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int64_t i = base + (int64_t)u * kGroups;
    live[u] = i < count;
    pos[u] = first + (live[u] ? i : 0);
  }
  // unit headers
  uint32_t D[U];
  int64_t lo[U], hi[U];
  int32_t kv[U], gs[U], js[U];
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int64_t v = pos[u];
    D[u] = comm[v];
    lo[u] = g.rp[v];
    hi[u] = live[u] ? g.rp[v + 1] : lo[u];
    kv[u] = g.k[v];
    gs[u] = g.slice[v];
    js[u] = kOne ? 0 : g.solve_of(v);   // one solve: its constants are uniform
    if (sd.frozen && sd.frozen[js[u]]) {   // a solve out of this sweep: nothing to decide
      live[u] = false;
      hi[u] = lo[u];
    }
  }
  // entries and each unit's Sigma sub-table
  // entries: column (coupling flag), weight and, with kCopy, the neighbour's label from the
  // label copy, all read in entry order
  int32_t cr[U], deg[U];
  uint32_t val[U], c[U];
  SubTab tb[U];
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int64_t e = lo[u] + gl;
    const bool has = e < hi[u];
    deg[u] = (int32_t)(hi[u] - lo[u]);
    cr[u] = has ? g.col[e] : 0x7fffffff;
    c[u] = (kCopy && has) ? g.elab[e] : kNone;
    const uint32_t w = (has && g.w) ? (uint32_t)g.w[e] : 1u;
    tb[u].open(sig, gs[u]);
    val[u] = !has ? 0u : (cr[u] < 0 ? 0x80000000u | w : w);
  }
  // a coupling entry of zero weight is no entry; the own community's first probe
  uint32_t hD[U];
  uint64_t eD[U];
  int64_t a[U];
#pragma unroll
  for (int u = 0; u < U; u++) {
    a[u] = sd.a[js[u]];
    const bool ent = val[u] != 0u && (cr[u] >= 0 || a[u] != 0);
    if (!ent) c[u] = kNone;
    else if (!kCopy) c[u] = comm[cr[u] & 0x7fffffff];   // gathered
    if (gl == 0 && kv[u] > 0) eD[u] = tb[u].first(D[u], hD[u]);
  }
  // equal labels merged inside the group in a small LDS table per (group, unit): each entry
  // adds its raw weight (low half) or coupling multiplier (high half) to its label's slot; the
  // lane that claims a slot leads that label.  Three LDS steps instead of G shuffle rounds.
  constexpr int kSlots = 2 * G;   // load at most one half
  uint32_t *sk = lm0_keys + (threadIdx.x >> 6) * (U * 128) + (gbase / G) * kSlots;
  unsigned long long *sv = lm0_vals + (threadIdx.x >> 6) * (U * 128) + (gbase / G) * kSlots;
#pragma unroll
  for (int u = 0; u < U; u++) {
    sk[u * 128 + gl] = 0u;
    sk[u * 128 + gl + G] = 0u;
    sv[u * 128 + gl] = 0ull;
    sv[u * 128 + gl + G] = 0ull;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the clears land before the claims
  bool lead[U];
  int slot[U];
#pragma unroll
  for (int u = 0; u < U; u++) {
    lead[u] = false;
    slot[u] = -1;
    if (c[u] != kNone) {
      const uint32_t key = c[u] + 1;
      uint32_t h = (c[u] * 2654435769u) >> (32 - __builtin_ctz(kSlots));
      for (;;) {
        const uint32_t prev = atomicCAS(sk + u * 128 + h, 0u, key);
        if (prev == 0u || prev == key) {
          lead[u] = prev == 0u;
          break;
        }
        h = (h + 1) & (kSlots - 1);
      }
      slot[u] = (int)h;
      const unsigned long long add =
          (unsigned long long)(val[u] & 0x7fffffffu) << ((val[u] >> 31) ? 32 : 0);
      atomicAdd(sv + u * 128 + h, add);
    }
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0xc07f);
  uint32_t wr[U], wrD[U];
  int nc[U], ncD[U];
#pragma unroll
  for (int u = 0; u < U; u++) {
    wr[u] = 0;
    nc[u] = 0;
    wrD[u] = 0;
    ncD[u] = 0;
    if (lead[u]) {
      const unsigned long long t = sv[u * 128 + slot[u]];
      wr[u] = (uint32_t)t;
      nc[u] = (int)(t >> 32);
    }
    if (gl == 0) {   // the own community's weight
      const uint32_t key = D[u] + 1;
      uint32_t h = (D[u] * 2654435769u) >> (32 - __builtin_ctz(kSlots));
      for (int probes = 0; probes < kSlots; probes++) {
        const uint32_t k = sk[u * 128 + h];
        if (k == key) {
          const unsigned long long t = sv[u * 128 + h];
          wrD[u] = (uint32_t)t;
          ncD[u] = (int)(t >> 32);
          break;
        }
        if (k == 0u) break;
        h = (h + 1) & (kSlots - 1);
      }
    }
  }
  // candidates' first probes, all units together
  bool cand[U];
  uint32_t hc[U];
  uint64_t ec[U];
#pragma unroll
  for (int u = 0; u < U; u++) {
    cand[u] = lead[u] && c[u] != D[u];
    if (cand[u] && kv[u] > 0) ec[u] = tb[u].first(c[u], hc[u]);
  }
  // values, the group's best, the decision
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int j = js[u];
    const int64_t p = sd.p[j], q = sd.q[j], pb = sd.pb[j], b = sd.b[j];
    const int64_t k0 = kv[u];
    const int64_t S0 = k0 > 0 ? sd.S[gs[u]] : 1;
    Score0 best;
    best.g = 0;
    best.lab = kNone;
    if (cand[u]) {
      const int64_t W = b * (int64_t)wr[u] + a[u] * nc[u];
      Score0 s;
      s.lab = c[u];
      s.g = k0 > 0 ? q * S0 * W - pb * (k0 * tb[u].resolve(c[u], hc[u], ec[u])) : q * W;
      if (s.g > best.g || (s.g == best.g && s.lab < best.lab)) best = s;
    }
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) {
      Score0 o;
      o.g = shfl_xor64(best.g, m);
      o.lab = (uint32_t)__shfl_xor((int)best.lab, m, 64);
      if (o.g > best.g || (o.g == best.g && o.lab < best.lab)) best = o;
    }
    if (pc.c) {
      const unsigned long long nk =
          __popcll(__ballot(cand[u] && live[u]) &
                   (((G == 64) ? ~0ull : ((1ull << G) - 1)) << gbase));
      if (gl == 0 && live[u]) {
        atomicAdd(pc.c + 0, 1ull);
        atomicAdd(pc.c + 1, (unsigned long long)deg[u]);
        if (nk) atomicAdd(pc.c + 2, nk);
      }
    }
    if (gl == 0 && live[u]) {
      const int64_t wD = b * (int64_t)wrD[u] + a[u] * ncD[u];
      int64_t stay;
      if (k0 > 0) {
        const int64_t yD = tb[u].resolve(D[u], hD[u], eD[u]);
        stay = q * S0 * wD - pb * (k0 * (yD - k0));
      } else {
        stay = q * wD;
      }
      uint32_t out = kNone;
      if (best.g > stay)
        out = best.lab == kNone ? fresh_of(sd, fresh_base) + (uint32_t)g.uid[pos[u]] : best.lab;
      target[pos[u] - first] = out;
    }
    (void)p;
  }
}

template <class P, class V, int G>
__global__ __launch_bounds__(256) void k_lm_group(V g, SolveDev sd, const int32_t *units,
                                                  int64_t count, const uint32_t *comm,
                                                  SliceTable sig, uint32_t *target,
                                                  uint32_t fresh_base, LmCounters pc) {
  __shared__ uint32_t lk[4 * 128];
  __shared__ int64_t lv[4 * 128];
  lm_group_block<P, V, G>(g, sd, units, count, comm, sig, target, fresh_base, pc, blockIdx.x, lk,
                          lv);
}

template <class P, class V>
__global__ __launch_bounds__(256) void k_lm_wave(V g, SolveDev sd, const int32_t *units,
                                                 int64_t count, const uint32_t *comm,
                                                 SliceTable sig, uint32_t *target,
                                                 uint32_t fresh_base, LmCounters pc) {
  __shared__ uint32_t sk[4][1 << kWaveLg];
  __shared__ int64_t sv[4][1 << kWaveLg];
  __shared__ uint16_t sl[4][kWaveMaxDeg];
  __shared__ int sn[4];
  const int wv = threadIdx.x >> 6;
  const int64_t idx = (int64_t)blockIdx.x * 4 + wv;
  if (idx >= count) return;
  LdsTab tab{sk[wv], sv[wv], kWaveLg, sl[wv], sn + wv};
  uint32_t t = lm_unit<P>(WaveGrp(), tab, g, sd, units[idx], comm, sig, fresh_base,
                          (typename P::Score *)nullptr, pc);
  if ((threadIdx.x & 63) == 0) target[idx] = t;
}

template <class P, class V, int NT, int LG>
__global__ __launch_bounds__(NT) void k_lm_block(V g, SolveDev sd, const int32_t *units,
                                                 int64_t count, const uint32_t *comm,
                                                 SliceTable sig, uint32_t *target,
                                                 uint32_t fresh_base, LmCounters pc) {
  __shared__ uint32_t sk[1 << LG];
  __shared__ int64_t sv[1 << LG];
  __shared__ uint16_t sl[1 << (LG - 1)];   // degree bound of the bin: half the table
  __shared__ int sn;
  __shared__ typename P::Score red[NT / 64];
  __shared__ int64_t hw[NT / 64];
  __shared__ uint32_t hl[NT / 64];
  LdsTab tab{sk, sv, LG, sl, &sn};
  for (int64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
    uint32_t t = lm_unit<P>(BlockGrp(), tab, g, sd, units[idx], comm, sig, fresh_base, red, pc,
                            hw, hl);
    if (threadIdx.x == 0) target[idx] = t;
  }
}

// Bins 0..5 of one colour batch in one launch: consecutive block ranges per bin, each block
// running that bin's code (fewer launches and no per-bin tail).
struct BinSeg {
  const int32_t *units;
  uint32_t *target;
  int64_t count;
  int64_t blk0;     // first block of the segment
  int64_t nbk;      // blocks with work (k_lm_multi: the segment spans nbk rounded up to kXcds)
  int64_t first;    // level 0 in position order: position of the segment's first unit
  int32_t parts;    // latency mode: blocks per unit (candidates split, CandSplit)
  int64_t poff;     // latency mode: the segment's first split-unit slot
};
struct MultiSeg {
  BinSeg s[6];
  int64_t nblk;     // blocks with work (the grid is rounded up to a multiple of kXcds)
};
constexpr int kXcds = 8;   // MI355X: eight accelerator complex dies, each with its own L2

template <class P, class V>
__global__ __launch_bounds__(256) void k_lm_multi(V g, SolveDev sd, MultiSeg ms,
                                                  const uint32_t *comm, SliceTable sig,
                                                  uint32_t fresh_base, LmCounters pc) {
  __shared__ uint32_t sk[1 << kSmallBlockLg];        // 4 wave tables of 512, or one of 2048
  __shared__ int64_t sv[1 << kSmallBlockLg];
  __shared__ uint16_t sl[kSmallBlockMaxDeg];         // 4 lists of 256, or one of 1024
  __shared__ int sn[4];
  __shared__ typename P::Score red[4];
  __shared__ int64_t hw[4];
  __shared__ uint32_t hl[4];
  // XCD-aware order: workgroups are dealt to the 8 XCDs round-robin and every segment starts
  // at a multiple of 8, so within a segment block p serves the (p % 8)-th eighth of the
  // segment's units; units are in id (slice-major) order, so each XCD's L2 sees the labels
  // and Sigma sub-tables of a few slices while every XCD gets an equal share of every bin
  const int64_t b = blockIdx.x;
  int k = 0;
  while (k < 5 && b >= ms.s[k + 1].blk0) k++;
  const BinSeg sg = ms.s[k];
  const int64_t p = b - sg.blk0;
  const int64_t per = (sg.nbk + kXcds - 1) / kXcds;
  const int64_t lb = (p % kXcds) * per + p / kXcds;
  if (lb >= sg.nbk) return;
  switch (k) {
    case 0:
      lm_group_block<P, V, 4>(g, sd, sg.units, sg.count, comm, sig, sg.target, fresh_base, pc, lb,
                               sk, sv);
      break;
    case 1:
      lm_group_block<P, V, 8>(g, sd, sg.units, sg.count, comm, sig, sg.target, fresh_base, pc, lb,
                               sk, sv);
      break;
    case 2:
      lm_group_block<P, V, 16>(g, sd, sg.units, sg.count, comm, sig, sg.target, fresh_base, pc,
                               lb, sk, sv);
      break;
    case 3:
      lm_group_block<P, V, 32>(g, sd, sg.units, sg.count, comm, sig, sg.target, fresh_base, pc,
                               lb, sk, sv);
      break;
    case 4: {
      const int wv = threadIdx.x >> 6;
      const int64_t idx = lb * 4 + wv;
      if (idx >= sg.count) return;
      // a unit of at most 64 entries in fewer than kCoopMinM slices: the wave as one lane group
      // (entries one per lane, labels merged in this wave's LDS region)
      const int64_t v0 = sg.units[idx];
      if (g.degree(v0) <= 64 && g.plen(v0) < kCoopMinM) {
        // lm_group_block addresses 128 slots per wave from the pointer it gets: shift it so
        // that this wave lands on its own 512-slot wave table, which no other wave touches
        lm_group_block<P, V, 64>(g, sd, sg.units, sg.count, comm, sig, sg.target, fresh_base, pc,
                                 lb, sk + (wv << kWaveLg) - wv * 128,
                                 sv + (wv << kWaveLg) - wv * 128);
        break;
      }
      LdsTab tab{sk + (wv << kWaveLg), sv + (wv << kWaveLg), kWaveLg, sl + wv * kWaveMaxDeg,
                 sn + wv};
      uint32_t t = lm_unit<P>(WaveGrp(), tab, g, sd, sg.units[idx], comm, sig, fresh_base,
                              (typename P::Score *)nullptr, pc);
      if ((threadIdx.x & 63) == 0) sg.target[idx] = t;
      break;
    }
    default: {
      LdsTab tab{sk, sv, kSmallBlockLg, sl, sn};
      uint32_t t = lm_unit<P>(BlockGrp(), tab, g, sd, sg.units[lb], comm, sig, fresh_base, red,
                              pc, hw, hl);
      if (threadIdx.x == 0) sg.target[lb] = t;
    }
  }
}

// Bins 0..3 alone (lane groups, one adjacency entry per lane): no LDS, so a large batch runs at
// the occupancy the group code's registers allow, where the fused kernel's LDS tables would
// hold it lower.  Same XCD-aware block order as k_lm_multi.
template <class P, class V>
__global__ __launch_bounds__(256) void k_lm_groups(V g, SolveDev sd, MultiSeg ms,
                                                   const uint32_t *comm, SliceTable sig,
                                                   uint32_t fresh_base, LmCounters pc) {
  __shared__ uint32_t lk[4 * 128];
  __shared__ int64_t lv[4 * 128];
  const int64_t b = blockIdx.x;
  int k = 0;
  while (k < 3 && b >= ms.s[k + 1].blk0) k++;
  const BinSeg sg = ms.s[k];
  const int64_t p = b - sg.blk0;
  const int64_t per = (sg.nbk + kXcds - 1) / kXcds;
  const int64_t lb = (p % kXcds) * per + p / kXcds;
  if (lb >= sg.nbk) return;
  switch (k) {
    case 0:
      lm_group_block<P, V, 4>(g, sd, sg.units, sg.count, comm, sig, sg.target, fresh_base, pc, lb,
                               lk, lv);
      break;
    case 1:
      lm_group_block<P, V, 8>(g, sd, sg.units, sg.count, comm, sig, sg.target, fresh_base, pc, lb,
                               lk, lv);
      break;
    case 2:
      lm_group_block<P, V, 16>(g, sd, sg.units, sg.count, comm, sig, sg.target, fresh_base, pc,
                               lb, lk, lv);
      break;
    default:
      lm_group_block<P, V, 32>(g, sd, sg.units, sg.count, comm, sig, sg.target, fresh_base, pc,
                               lb, lk, lv);
  }
}

// Bins 0..3 of a level-0 colour batch in position order (lm0_lockstep), XCD-aware block order
// as in k_lm_multi; segment k starts at position ms.s[k].first.  kOne: a single solve; kCopy:
// neighbour labels from the label copy.
template <int U, bool kOne, bool kCopy>
__global__ __launch_bounds__(256) void k_lm0_groups(ViewP g, SolveDev sd, MultiSeg ms,
                                                    const uint32_t *comm, SliceTable sig,
                                                    uint32_t fresh_base, LmCounters pc) {
  __shared__ uint32_t keys[4 * U * 128];
  __shared__ unsigned long long vals[4 * U * 128];
  const int64_t b = blockIdx.x;
  int k = 0;
  while (k < 3 && b >= ms.s[k + 1].blk0) k++;
  const BinSeg sg = ms.s[k];
  const int64_t p = b - sg.blk0;
  const int64_t per = (sg.nbk + kXcds - 1) / kXcds;
  const int64_t lb = (p % kXcds) * per + p / kXcds;
  if (lb >= sg.nbk) return;
  switch (k) {
    case 0:
      lm0_lockstep<4, U, kOne, kCopy>(g, sd, sg.first, sg.count, comm, sig, sg.target,
                                        fresh_base, pc, lb, keys, vals);
      break;
    case 1:
      lm0_lockstep<8, U, kOne, kCopy>(g, sd, sg.first, sg.count, comm, sig, sg.target,
                                        fresh_base, pc, lb, keys, vals);
      break;
    case 2:
      lm0_lockstep<16, U, kOne, kCopy>(g, sd, sg.first, sg.count, comm, sig, sg.target,
                                        fresh_base, pc, lb, keys, vals);
      break;
    default:
      lm0_lockstep<32, U, kOne, kCopy>(g, sd, sg.first, sg.count, comm, sig, sg.target,
                                        fresh_base, pc, lb, keys, vals);
  }
}

// Latency mode (aggregated levels, colour batches of few units): every bin below the hub bin
// of both unit classes in one launch.  Occupancy does not matter here, so one kernel carries
// both policies and an LDS table large enough for degree 4096; its blocks have 512 threads,
// which leaves the multi-slice policy the registers it needs without spilling.
struct LatSegs {
  BinSeg s[2 * kBinGtab];   // class (single-slice, multi-slice) x bins 0..kBinGtab-1
  ScoreK *part;             // [split-unit slots x parts] published bests
  uint32_t *done;           // [split-unit slots] finished blocks, 0 between launches
};

template <class P, class V>
__device__ inline void lat_bin(const V &g, const SolveDev &sd, const BinSeg &sg, int bin,
                               int64_t lb, const uint32_t *comm, const SliceTable &sig,
                               uint32_t fresh_base, LmCounters pc, uint32_t *sk, int64_t *sv,
                               uint16_t *sl, int *sn, typename P::Score *red, int64_t *hw,
                               uint32_t *hl, CandSplit cs, ScoreK *ls_part, uint32_t *ls_done) {
  switch (bin) {
    case 0:
      lm_group_block<P, V, 4>(g, sd, sg.units, sg.count, comm, sig, sg.target, fresh_base, pc, lb,
                               sk, sv);
      break;
    case 1:
      lm_group_block<P, V, 8>(g, sd, sg.units, sg.count, comm, sig, sg.target, fresh_base, pc, lb,
                               sk, sv);
      break;
    case 2:
      lm_group_block<P, V, 16>(g, sd, sg.units, sg.count, comm, sig, sg.target, fresh_base, pc,
                               lb, sk, sv);
      break;
    case 3:
      lm_group_block<P, V, 32>(g, sd, sg.units, sg.count, comm, sig, sg.target, fresh_base, pc,
                               lb, sk, sv);
      break;
    default: {   // one unit per block, or sg.parts blocks per unit; table sized by the bin
      const int lg = bin <= 5 ? kSmallBlockLg : kBlockLg;
      LdsTab tab{sk, sv, lg, sl, sn};
      const int64_t unit = lb / sg.parts;
      if (sg.parts > 1) {
        cs.part = (int)(lb % sg.parts);
        cs.B = sg.parts;
        cs.parts = ls_part + (sg.poff + unit) * sg.parts;
        cs.done = ls_done + sg.poff + unit;
      }
      uint32_t t = lm_unit<P>(BlockGrp(), tab, g, sd, sg.units[unit], comm, sig, fresh_base, red,
                              pc, hw, hl, cs);
      if (threadIdx.x == 0 && (sg.parts == 1 || *cs.last)) sg.target[unit] = t;
    }
  }
}

constexpr int kLatThreads = 512;
// Block size of the 8192-slot table kernels: the multi-slice policy needs more than the 128
// registers per lane that 1024-thread blocks allow
template <class P>
constexpr int kBlockThreads = IsMulti<P>::value ? 512 : 1024;

template <class V, class PK>
__global__ __launch_bounds__(kLatThreads) void k_lm_lat(V g, SolveDev sd, LatSegs ls,
                                                        const uint32_t *comm, SliceTable sig,
                                                        uint32_t fresh_base, LmCounters pc) {
  __shared__ uint32_t sk[1 << kBlockLg];
  __shared__ int64_t sv[1 << kBlockLg];
  __shared__ uint16_t sl[kBlockMaxDeg];
  __shared__ int sn;
  __shared__ ScoreK redK[kLatThreads / 64];
  __shared__ Score1 red1[kLatThreads / 64];
  __shared__ int64_t hw[kLatThreads / 64];
  __shared__ uint32_t hl[kLatThreads / 64];
  __shared__ uint16_t sl2[kBlockMaxDeg];
  __shared__ int sn2, slast;
  const int64_t b = blockIdx.x;
  int k = 0;
  while (k < 2 * kBinGtab - 1 && b >= ls.s[k + 1].blk0) k++;
  const BinSeg sg = ls.s[k];
  const int64_t lb = b - sg.blk0;
  const int bin = k % kBinGtab;
  CandSplit cs;
  cs.L2 = sl2;
  cs.n2 = &sn2;
  cs.last = &slast;
  if (k < kBinGtab)
    lat_bin<PolicyK1>(g, sd, sg, bin, lb, comm, sig, fresh_base, pc, sk, sv, sl, &sn, red1, hw,
                      hl, cs, ls.part, ls.done);
  else
    lat_bin<PK>(g, sd, sg, bin, lb, comm, sig, fresh_base, pc, sk, sv, sl, &sn, redK, hw, hl, cs,
                ls.part, ls.done);
}

// Units of very high degree: a global-memory table per unit, slot offsets from a scan.
template <class P, class V>
__global__ __launch_bounds__(256) void k_lm_gtab(V g, SolveDev sd, const int32_t *units,
                                                 int64_t count, const uint32_t *comm,
                                                 SliceTable sig, uint32_t *target,
                                                 uint32_t fresh_base, uint32_t *gk, int64_t *gv,
                                                 const int64_t *goff, const int32_t *glg,
                                                 LmCounters pc) {
  __shared__ typename P::Score red[4];
  __shared__ int64_t hw[4];
  __shared__ uint32_t hl[4];
  for (int64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const int64_t v = units[idx];
    GTab tab{gk + goff[v], gv + goff[v], glg[v]};
    uint32_t t = lm_unit<P>(BlockGrpG(), tab, g, sd, v, comm, sig, fresh_base, red, pc, hw, hl);
    if (threadIdx.x == 0) target[idx] = t;
  }
}

// ------------------------------------------------------------------ hub units
// Units above the block bins are spread over kHubBlocks blocks each (grid = kHubBlocks x
// units): the blocks clear, fill and scan disjoint parts of the unit's global table, each
// scan keeps its best candidate, and one wave per unit reduces those with the same total
// order (value, then label) and compares with staying.  The result equals one group's.
constexpr int kHubBlocks = 16;

__global__ __launch_bounds__(256) void k_hub_clear(const int32_t *units, const int64_t *goff,
                                                   const int32_t *glg, uint32_t *gk, int64_t *gv) {
  const int64_t v = units[blockIdx.y];
  const int64_t size = 1ll << glg[v], base = goff[v];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < size;
       i += (int64_t)gridDim.x * blockDim.x) {
    gk[base + i] = 0;
    gv[base + i] = 0;
  }
}

// A hub's entries mostly fall into few communities, so adding each one to the global table
// would queue thousands of atomics on the same words: each block first sums its share of the
// entries in an LDS table of at most kHubLdsKeys keys (entries of further keys go straight to
// the global table), then adds each LDS key's sum to the global table once.
constexpr int kHubLdsLg = 11;
constexpr int kHubLdsKeys = 1 << (kHubLdsLg - 1);

template <class V>
__global__ __launch_bounds__(256) void k_hub_accum(V g, SolveDev sd, const int32_t *units,
                                                   const uint32_t *comm, const int64_t *goff,
                                                   const int32_t *glg, uint32_t *gk, int64_t *gv,
                                                   LmCounters pc) {
  __shared__ uint32_t sk[1 << kHubLdsLg];
  __shared__ int64_t sv[1 << kHubLdsLg];
  __shared__ int s_claimed;
  const int64_t v = units[blockIdx.y];
  GTab tab{gk + goff[v], gv + goff[v], glg[v]};
  typename V::Row row = g.row(v, sd);
  for (int i = threadIdx.x; i < (1 << kHubLdsLg); i += blockDim.x) {
    sk[i] = 0;
    sv[i] = 0;
  }
  if (threadIdx.x == 0) s_claimed = 0;
  __syncthreads();
  constexpr uint32_t mask = (1u << kHubLdsLg) - 1;
  for (int64_t e = row.lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < row.hi;
       e += (int64_t)gridDim.x * blockDim.x) {
    int64_t w;
    const int64_t x = g.nbr(row, e, w);
    if (w == 0) continue;
    const uint32_t lab = g.lab_at(comm, e, x), key = lab + 1;
    uint32_t h = fib_hash(lab, 32 - kHubLdsLg);
    bool done = false;
    // at most kHubLdsKeys slots are ever claimed, so an empty slot is always reached
    for (;;) {
      const uint32_t k = sk[h];
      if (k == key) {
        atomicAdd(reinterpret_cast<unsigned long long *>(&sv[h]), (unsigned long long)w);
        done = true;
        break;
      }
      if (k == 0) {
        if (atomicAdd(&s_claimed, 1) >= kHubLdsKeys) break;   // LDS table closed to new keys
        const uint32_t prev = atomicCAS(&sk[h], 0u, key);
        if (prev == 0 || prev == key) {
          atomicAdd(reinterpret_cast<unsigned long long *>(&sv[h]), (unsigned long long)w);
          done = true;
          break;
        }
      }
      h = (h + 1) & mask;
    }
    if (!done) tab.add(lab, w);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < (1 << kHubLdsLg); i += blockDim.x)
    if (sk[i] != 0) tab.add(sk[i] - 1, sv[i]);
  if (pc.c && blockIdx.x == 0 && threadIdx.x == 0) {
    atomicAdd(pc.c + 0, 1ull);
    atomicAdd(pc.c + 1, (unsigned long long)(row.hi - row.lo));
  }
}

constexpr int kHubWin = 2048;   // table slots compacted at a time by a hub evaluation block

template <class P, class V>
__global__ __launch_bounds__(256) void k_hub_eval(V g, SolveDev sd, const int32_t *units,
                                                  const uint32_t *comm, SliceTable sig,
                                                  const int64_t *goff, const int32_t *glg,
                                                  const uint32_t *gk, const int64_t *gv,
                                                  typename P::Score *part, LmCounters pc) {
  __shared__ typename P::Score red[4];
  const int64_t v = units[blockIdx.y];
  const uint32_t D = comm[v];
  const uint32_t *K = gk + goff[v];
  const int64_t *Wt = gv + goff[v];
  const int64_t size = 1ll << glg[v];
  const int64_t span = (size + gridDim.x - 1) / gridDim.x;
  const int64_t s0 = (int64_t)blockIdx.x * span, s1 = s0 + span < size ? s0 + span : size;
  const UnitCtx u = unit_ctx(g, sd, v, D);
  typename P::Score best = P::make(g, u, sd, sig, kNone, 0, kEmpty);
  int ncand = 0;
  bool coop = false;
  if constexpr (!V::kLevel0 && IsMulti<P>::value) coop = u.m >= kCoopMinM;
  if (coop) {
    if constexpr (!V::kLevel0 && IsMulti<P>::value) {
      // the block's span of the table is mostly empty slots: each window of kHubWin slots is
      // first compacted into an LDS list of its candidates, and only those take coop turns
      __shared__ int32_t wl[kHubWin];
      __shared__ int wn;
      const CoopLane c = coop_lane(g, u, sd, sig, threadIdx.x);
      const int sub = threadIdx.x / c.mp, nsub = blockDim.x / c.mp;
      for (int64_t w0 = s0; w0 < s1; w0 += kHubWin) {
        const int64_t w1 = w0 + kHubWin < s1 ? w0 + kHubWin : s1;
        if (threadIdx.x == 0) wn = 0;
        __syncthreads();
        for (int64_t i = w0 + threadIdx.x; i < w1; i += blockDim.x) {
          const uint32_t key = K[i];
          if (key != 0 && key - 1 != D) wl[atomicAdd(&wn, 1)] = (int32_t)(i - w0);
        }
        __syncthreads();
        const int nw = wn;
        for (int i0 = 0; i0 < nw; i0 += nsub * kCoopBatch) {
          uint32_t lab[kCoopBatch];
          int64_t W[kCoopBatch], y[kCoopBatch];
          bool ok[kCoopBatch];
          for (int k = 0; k < kCoopBatch; k++) {
            const int ii = i0 + k * nsub + sub;
            const int64_t i = ii < nw ? w0 + wl[ii] : -1;
            const uint32_t key = i >= 0 ? K[i] : 0u;
            lab[k] = key - 1;
            ok[k] = key != 0;
            W[k] = ok[k] ? Wt[i] : 0;
            ok[k] = ok[k] && !P::prunable(u, W[k], best);
          }
          coop_lookup<kCoopBatch>(c, lab, ok, y);
          for (int k = 0; k < kCoopBatch; k++) {
            if (!ok[k]) continue;
            ncand += c.j == 0;
            ScoreK sc = coop_score(u, c, lab[k], W[k], y[k], kTarget);
            if (better<P>(g, u, sd, sig, sc, best)) best = sc;
          }
        }
        __syncthreads();   // the list is rewritten by the next window
      }
    }
  } else {
    for (int64_t i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
      const uint32_t key = K[i];
      if (key == 0 || key - 1 == D) continue;
      const int64_t W = Wt[i];
      if (P::prunable(u, W, best)) continue;
      ncand++;
      typename P::Score sc = P::make(g, u, sd, sig, key - 1, W, kTarget);
      if (better<P>(g, u, sd, sig, sc, best)) best = sc;
    }
  }
  if (pc.c && ncand) atomicAdd(pc.c + 2, (unsigned long long)ncand);
  best = group_best<P>(BlockGrp(), g, u, sd, sig, best, red);
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = best;
}

template <class P, class V>
__global__ __launch_bounds__(64) void k_hub_final(V g, SolveDev sd, const int32_t *units,
                                                  int64_t count, const uint32_t *comm,
                                                  SliceTable sig, const int64_t *goff,
                                                  const int32_t *glg, const uint32_t *gk,
                                                  const int64_t *gv,
                                                  const typename P::Score *part, int nparts,
                                                  uint32_t *target, uint32_t fresh_base) {
  const int64_t idx = blockIdx.x;
  if (idx >= count) return;
  const int lane = threadIdx.x & 63;
  const int64_t v = units[idx];
  const uint32_t D = comm[v];
  const UnitCtx u = unit_ctx(g, sd, v, D);
  typename P::Score best = P::make(g, u, sd, sig, kNone, 0, kEmpty);
  if (lane < nparts) best = part[idx * nparts + lane];
  best = wave_best<P>(g, u, sd, sig, best);
  GTab tab{const_cast<uint32_t *>(gk) + goff[v], const_cast<int64_t *>(gv) + goff[v], glg[v]};
  const int64_t wD = tab.get(D);
  typename P::Score stay;
  bool coop = false;
  if constexpr (!V::kLevel0 && IsMulti<P>::value) coop = u.m >= kCoopMinM;
  if (coop) {
    if constexpr (!V::kLevel0 && IsMulti<P>::value)
      stay = coop_make(u, coop_lane(g, u, sd, sig, lane), D, wD, kStay);
  } else {
    stay = P::make(g, u, sd, sig, D, wD, kStay);
  }
  if (lane == 0) {
    uint32_t out = kNone;
    if (P::cmp(g, u, sd, sig, best, stay) > 0)
      out = best.lab == kNone ? fresh_of(sd, fresh_base) + (uint32_t)g.orig(v) : best.lab;
    target[idx] = out;
  }
}

// Apply the decided moves of one colour batch: new label, Sigma delta for every profile slice.
template <class V>
__global__ __launch_bounds__(256) void k_lm_apply(V g, const int32_t *units, int64_t count,
                                                  const uint32_t *target, uint32_t *comm,
                                                  SliceTable sig, uint32_t *moved,
                                                  const uint8_t *frozen) {
  __shared__ uint32_t s_moves;
  __shared__ int s_j, s_mixed;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool mv = false;
  int j = 0;
  if (threadIdx.x == 0) {
    s_moves = 0;
    s_mixed = 0;
    s_j = g.solve_of(units[i]);   // thread 0's unit always exists
  }
  __syncthreads();
  if (i < count) {
    const uint32_t C = target[i];
    const int64_t v = units[i];
    j = g.solve_of(v);
    if (C != kNone && !frozen[j]) {
      const uint32_t D = comm[v];
      const int m = g.plen(v);
      for (int jj = 0; jj < m; jj++) {
        int gs;
        int64_t k;
        g.pent(v, jj, gs, k);
        tab_add(sig, gs, D, -(int32_t)k);
        tab_add(sig, gs, C, (int32_t)k);
      }
      comm[v] = C;
      if constexpr (std::is_same<V, ViewP>::value) {
        if (g.elab)   // the entries pointing at v see its new label
          for (int64_t e = g.rp[v]; e < g.rp[v + 1]; e++) g.elab[g.prev[e]] = C;
      }
      mv = true;
    }
    if (j != s_j) s_mixed = 1;
    if (mv) atomicAdd(&s_moves, 1u);
  }
  __syncthreads();
  // one atomic per block when all its units belong to one solve (the usual case)
  if (!s_mixed) {
    if (threadIdx.x == 0 && s_moves) atomicAdd(moved + s_j, s_moves);
  } else {
    wave_count(moved, j, mv);
  }
}

// The moves of a small batch, one wave per unit with the lanes over its profile slices (a
// unit of an aggregated level spans up to 64 slices, two Sigma atomics each).
template <class V>
__global__ __launch_bounds__(256) void k_lm_apply_wave(V g, const int32_t *units, int64_t count,
                                                       const uint32_t *target, uint32_t *comm,
                                                       SliceTable sig, uint32_t *moved,
                                                       const uint8_t *frozen) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= count) return;
  const uint32_t C = target[i];
  const int64_t v = units[i];
  const int j = g.solve_of(v);
  if (C == kNone || frozen[j]) return;
  const uint32_t D = comm[v];
  const int m = g.plen(v);
  for (int jj = lane; jj < m; jj += 64) {
    int gs;
    int64_t k;
    g.pent(v, jj, gs, k);
    tab_add(sig, gs, D, -(int32_t)k);
    tab_add(sig, gs, C, (int32_t)k);
  }
  if constexpr (std::is_same<V, ViewP>::value) {
    if (g.elab)
      for (int64_t e = g.rp[v] + lane; e < g.rp[v + 1]; e += 64) g.elab[g.prev[e]] = C;
  }
  if (lane == 0) {
    comm[v] = C;
    atomicAdd(moved + j, 1u);
  }
}

// Profile entries per global slice (how many units of a level can hold a key in the slice's
// Sigma sub-table): an LDS histogram per block when the slices fit, else global atomics.
constexpr int kSliceHistMax = 4096;
__global__ void k_profile_slice_count(const int32_t *ps, int64_t ne, int nslices, int64_t *cnt) {
  __shared__ uint32_t h[kSliceHistMax];
  const bool lds = nslices <= kSliceHistMax;
  if (lds)
    for (int i = threadIdx.x; i < nslices; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ne;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (lds) atomicAdd(&h[ps[i]], 1u);
    else atomicAdd(reinterpret_cast<unsigned long long *>(cnt + ps[i]), 1ull);
  }
  __syncthreads();
  if (lds)
    for (int i = threadIdx.x; i < nslices; i += blockDim.x)
      if (h[i]) atomicAdd(reinterpret_cast<unsigned long long *>(cnt + i), (unsigned long long)h[i]);
}

// Labels of the units of flagged solves back to their copy from the start of the sweep.
template <class V>
__global__ void k_restore_flagged(V g, int64_t n, const uint32_t *snap, const uint32_t *redo,
                                  uint32_t *comm) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && redo[g.usolve[v]]) comm[v] = snap[v];
}

// ------------------------------------------------------------------ level 0 by position
// The level-0 sweeps read the supra-CSR in colour-batch order (ViewP): position i holds unit
// units[i] of the level's sorted batch list.  These kernels lay it out once per level-0 visit.
__global__ void k_pos_of(const int32_t *units, int64_t n, int32_t *pos) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pos[units[i]] = (int32_t)i;
}

// keys ordering the level's units by (batch key, label), ids ascending among equals
__global__ void k_pos_label_keys(const uint32_t *keys, const int32_t *units,
                                 const uint32_t *comm, int64_t n, uint64_t *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = ((uint64_t)keys[i] << 32) | comm[units[i]];
}

// per position: degree (for the row starts), intra degree, slice, solve, labels
__global__ void k_pos_meta(View0 g, const int32_t *units, int64_t n, int64_t *deg, int32_t *pk,
                           int32_t *pslice, int32_t *psolve, int32_t *iota,
                           const uint32_t *comm, uint32_t *pcomm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  if (i == n) {
    deg[n] = 0;
    return;
  }
  const int64_t v = units[i];
  deg[i] = g.degree(v);
  int gs;
  int64_t kk;
  g.pent(v, 0, gs, kk);
  pk[i] = (int32_t)kk;
  pslice[i] = gs;
  if (psolve) psolve[i] = g.solve_of(v);
  iota[i] = (int32_t)i;
  pcomm[i] = comm[v];
}

// entries of one position: neighbour positions with the coupling flag, raw weights
// PosRows: the optional neighbour-label copy (labels of the level's start) and reverse entries
struct PosLabels {
  const uint32_t *comm;   // labels by unit id
  const int64_t *prp;     // row starts by position
  uint32_t *elab;         // nullptr: not built
  int32_t *prev;
};

__device__ inline void pos_row(const View0 &g, const SolveDev &sd, int64_t v, int64_t out,
                               const int32_t *pos, int32_t *pcol, int32_t *pw, int first,
                               int step, const PosLabels &pl) {
  const typename View0::Row r = g.row(v, sd);
  for (int64_t e = r.lo + first; e < r.hi; e += step) {
    const int32_t x = g.col[e];
    const bool coupling = !(x >= r.slo && x < r.shi);
    const int32_t px = pos[x];
    pcol[out + (e - r.lo)] = px | (coupling ? (int32_t)0x80000000 : 0);
    if (pw) pw[out + (e - r.lo)] = g.w[e];
    if (pl.elab) {
      pl.elab[out + (e - r.lo)] = pl.comm[x];
      pl.prev[out + (e - r.lo)] = (int32_t)(pl.prp[px] + g.rev[e]);
    }
  }
}

// rows of at most 32 entries one thread each; longer rows are listed for a wave each
__global__ void k_pos_rows(View0 g, SolveDev sd, const int32_t *units, int64_t n,
                           const int64_t *prp, const int32_t *pos, int32_t *pcol, int32_t *pw,
                           int32_t *wide, uint32_t *nwide, PosLabels pl) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t v = units[i];
  if (g.degree(v) > 32) {
    wide[atomicAdd(nwide, 1u)] = (int32_t)i;
    return;
  }
  pos_row(g, sd, v, prp[i], pos, pcol, pw, 0, 1, pl);
}

__global__ void k_pos_rows_wide(View0 g, SolveDev sd, const int32_t *units, const int64_t *prp,
                                const int32_t *pos, int32_t *pcol, int32_t *pw,
                                const int32_t *wide, const uint32_t *nwide, PosLabels pl) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t k = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); k < *nwide;
       k += nw) {
    const int64_t i = wide[k];
    pos_row(g, sd, units[i], prp[i], pos, pcol, pw, lane, 64, pl);
  }
}

// global-table slots of the hub units, by position
__global__ void k_pos_gtab(const int32_t *hubs, int64_t cnt, const int32_t *pos,
                           const int64_t *goff, const int32_t *glg, int64_t *goffP,
                           int32_t *glgP) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const int64_t u = hubs[i];
  goffP[pos[u]] = goff[u];
  glgP[pos[u]] = glg[u];
}

__global__ void k_pos_labels_back(const int32_t *units, int64_t n, const uint32_t *pcomm,
                                  uint32_t *comm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) comm[units[i]] = pcomm[i];
}

// the label copy made current again after sweeps that did not keep it (entry order)
__global__ void k_pos_elab_refresh(const int32_t *pcol, int64_t nnz, const uint32_t *pcomm,
                                   uint32_t *elab) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nnz) elab[e] = pcomm[pcol[e] & 0x7fffffff];
}

// A refinement round taken again exactly for the solves that raised their redo flag only:
// their units get back the active flags and proposal stamps of the round's start; the other
// solves' units are set aside (inactive, so the proposal kernels skip them) and get their
// flags back afterwards (k_ref_redo_done), keeping their proposals of the first pass.
template <class V>
__global__ void k_ref_redo_prep(V g, int64_t n, const uint32_t *redo, uint8_t *active,
                                const uint8_t *snap_a, uint32_t *propr, const uint32_t *snap_p,
                                uint8_t *keep) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (redo[g.solve_of(v)]) {
    active[v] = snap_a[v];
    propr[v] = snap_p[v];
  } else {
    keep[v] = active[v];
    active[v] = 0;
  }
}
template <class V>
__global__ void k_ref_redo_done(V g, int64_t n, const uint32_t *redo, uint8_t *active,
                                const uint8_t *keep) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && !redo[g.solve_of(v)]) active[v] = keep[v];
}

template <class V>
__global__ void k_sigma_build(V g, int64_t n, const uint32_t *comm, SliceTable sig) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int m = g.plen(v);
  for (int jj = 0; jj < m; jj++) {
    int gs;
    int64_t k;
    g.pent(v, jj, gs, k);
    tab_add(sig, gs, comm[v], (int32_t)k, false);
  }
}

__global__ void k_rebuild_check(const uint32_t *used, const uint32_t *limit, int nslices, int *flag) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nslices && used[s] > limit[s]) atomicOr(flag, 1);
}

// ------------------------------------------------------------------ colouring
// First-fit colouring in decreasing priority (Jones-Plassmann): a unit takes the smallest
// colour unused by its higher-priority neighbours once all of them are coloured.  The
// result equals the sequential greedy colouring in priority order.  Each unit counts its
// higher-priority neighbours once; a round colours the ready frontier and releases the
// lower-priority neighbours, so every row is scanned a constant number of times.
// Frontier lists of a colouring round: units above kJpHeavy neighbours are coloured by a
// whole block (their scans would hold a single wave for long), the others by one wave.
constexpr int kJpHeavy = 512;
struct JpLists {
  int32_t *light[2];
  int32_t *heavy[2];
  uint32_t *counts;   // [0..2] light counters, [3..5] heavy counters (round r uses r % 3)
};

// Rows longer than kJpCountThread entries are counted by a wave (k_jp_count_wide) instead
// of a single thread.
constexpr int kJpCountThread = 64;

template <class V>
__global__ __launch_bounds__(256) void k_jp_count(V g, SolveDev sd, const int32_t *work,
                                                  int64_t nwork, uint32_t *cnt, int32_t *front,
                                                  uint32_t *nfront, int32_t *hfront,
                                                  uint32_t *nhfront, int32_t *wide,
                                                  uint32_t *nwide, int it, int lvl) {
  // one thread per unit; ready units are appended once per wave
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ready = false;
  int64_t v = 0;
  const bool long_row = idx < nwork && g.degree(work[idx]) > kJpCountThread;
  wave_append(wide, nwide, long_row, idx < nwork ? work[idx] : 0);
  if (idx < nwork && !long_row) {
    v = work[idx];
    const int j = g.usolve[v];
    const uint64_t sm = sd.seedmix[j];
    const int64_t off = sd.uoff[j];
    const uint64_t hv = priority(sm, it, lvl, 0, (uint32_t)(v - off));
    typename V::Row row = g.row(v, sd);
    uint32_t c = 0;
    for (int64_t e = row.lo; e < row.hi; e++) {
      int32_t x = g.col[e];
      if (g.wt(row, e, x) == 0) continue;
      uint64_t hx = priority(sm, it, lvl, 0, (uint32_t)(x - off));
      if (outranks(hx, (uint32_t)x, hv, (uint32_t)v)) c++;
    }
    cnt[v] = c;
    ready = c == 0;
  }
  const bool heavy = ready && g.degree(v) > kJpHeavy;
  wave_append(front, nfront, ready && !heavy, (int32_t)v);
  wave_append(hfront, nhfront, heavy, (int32_t)v);
}

// The long rows set aside by k_jp_count, one wave each; their number is read on the device.
template <class V>
__global__ __launch_bounds__(256) void k_jp_count_wide(V g, SolveDev sd, const int32_t *wide,
                                                       const uint32_t *nwide, uint32_t *cnt,
                                                       int32_t *front, uint32_t *nfront,
                                                       int32_t *hfront, uint32_t *nhfront, int it,
                                                       int lvl) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = *nwide;
  for (int64_t idx = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); idx < nw;
       idx += (int64_t)gridDim.x * 4) {
    const int64_t v = wide[idx];
    const int j = g.usolve[v];
    const uint64_t sm = sd.seedmix[j];
    const int64_t off = sd.uoff[j];
    const uint64_t hv = priority(sm, it, lvl, 0, (uint32_t)(v - off));
    typename V::Row row = g.row(v, sd);
    int64_t c = 0;
    for (int64_t e = row.lo + lane; e < row.hi; e += 64) {
      int32_t x = g.col[e];
      if (g.wt(row, e, x) == 0) continue;
      uint64_t hx = priority(sm, it, lvl, 0, (uint32_t)(x - off));
      if (outranks(hx, (uint32_t)x, hv, (uint32_t)v)) c++;
    }
    for (int m = 32; m >= 1; m >>= 1) c += shfl_xor64(c, m);
    if (lane == 0) cnt[v] = (uint32_t)c;
    const bool ready = lane == 0 && c == 0;
    const bool heavy = ready && g.degree(v) > kJpHeavy;
    wave_append(front, nfront, ready && !heavy, (int32_t)v);
    wave_append(hfront, nhfront, heavy, (int32_t)v);
  }
}

// Release the lower-priority neighbours of v over entries [lo, hi) with stride `step`
// starting at this thread's offset; the last release of a neighbour queues it for the next
// round (light or heavy list by degree).  Every thread of the wave must call this.
template <class V>
__device__ inline void jp_release(const V &g, const typename V::Row &row, int64_t first,
                                  int step, int64_t v, uint64_t sm, int64_t off, uint64_t hv,
                                  uint32_t *cnt, WaveStage &sl, WaveStage &sh, int it, int lvl) {
  for (int64_t e0 = row.lo; e0 < row.hi; e0 += step) {
    const int64_t e = e0 + first;
    bool ready = false;
    int32_t x = 0;
    if (e < row.hi) {
      x = g.col[e];
      if (g.wt(row, e, x) != 0) {
        uint64_t hx = priority(sm, it, lvl, 0, (uint32_t)(x - off));
        if (!outranks(hx, (uint32_t)x, hv, (uint32_t)v)) ready = atomicSub(cnt + x, 1u) == 1u;
      }
    }
    const bool heavy = ready && g.degree(x) > kJpHeavy;
    sl.append(ready && !heavy, x);
    sh.append(heavy, x);
  }
}

// Colours of the higher-priority neighbours of v are marked in an LDS bitmap of NW words
// (atomic OR), a window of 64*NW colours at a time; the first clear bit is v's colour.
// sync() orders the bitmap's clear, marks and reads among the threads that share it.
template <int NW, class V, class Sync>
__device__ inline int jp_first_free(const V &g, const typename V::Row &row, int first, int step,
                                    int64_t v, uint64_t sm, int64_t off, uint64_t hv,
                                    const int32_t *colour, int it, int lvl, uint64_t *bits,
                                    Sync sync) {
  const int lane = threadIdx.x & 63;
  int result = -1;
  for (int base = 0; result < 0; base += 64 * NW) {
    for (int i = first; i < NW; i += step) bits[i] = 0;
    sync();
    for (int64_t e = row.lo + first; e < row.hi; e += step) {
      const int32_t x = g.col[e];
      if (g.wt(row, e, x) == 0) continue;
      const uint64_t hx = priority(sm, it, lvl, 0, (uint32_t)(x - off));
      if (!outranks(hx, (uint32_t)x, hv, (uint32_t)v)) continue;
      const int d = colour[x] - base;
      if (d >= 0 && d < 64 * NW) atomicOr((unsigned long long *)(bits + (d >> 6)), 1ull << (d & 63));
    }
    sync();
    // every wave reads the bitmap and finds the same first clear bit
    for (int w0 = 0; w0 < NW && result < 0; w0 += 64) {
      const uint64_t word = w0 + lane < NW ? bits[w0 + lane] : ~0ull;
      const uint64_t freew = __ballot(~word != 0);
      if (freew) {
        const int L = __builtin_ctzll(freew);
        const uint64_t wl = (uint64_t)__shfl((long long)word, L, 64);
        result = base + (w0 + L) * 64 + __builtin_ctzll(~wl);
      }
    }
    sync();
  }
  return result;
}

struct WaveLdsSync {
  // a wave's LDS operations complete in issue order; this only keeps the compiler from
  // moving them across the phases
  __device__ void operator()() const {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
};
struct BlockLdsSync {
  __device__ void operator()() const { __syncthreads(); }
};

// A light unit (at most kJpHeavy entries) has a colour of at most kJpHeavy, inside one
// window of this many bitmap words.
constexpr int kJpLightWords = (kJpHeavy + 64) / 64;
constexpr int kJpBlockWords = 64;

// Colour one light frontier unit with one wave.
template <class V>
__device__ inline void jp_unit(const V &g, const SolveDev &sd, int64_t v, int32_t *colour,
                               uint32_t *cnt, WaveStage &sl, WaveStage &sh, int it, int lvl,
                               uint64_t *bits) {
  const int lane = threadIdx.x & 63;
  const int j = g.usolve[v];
  const uint64_t sm = sd.seedmix[j];
  const int64_t off = sd.uoff[j];
  const uint64_t hv = priority(sm, it, lvl, 0, (uint32_t)(v - off));
  typename V::Row row = g.row(v, sd);
  const int result = jp_first_free<kJpLightWords>(g, row, lane, 64, v, sm, off, hv, colour, it,
                                                  lvl, bits, WaveLdsSync());
  if (lane == 0) colour[v] = result;
  jp_release(g, row, lane, 64, v, sm, off, hv, cnt, sl, sh, it, lvl);
}

// Colour one heavy frontier unit with the whole block (all threads must call this).
template <class V>
__device__ inline void jp_unit_block(const V &g, const SolveDev &sd, int64_t v, int32_t *colour,
                                     uint32_t *cnt, WaveStage &sl, WaveStage &sh, int it,
                                     int lvl, uint64_t *bits) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int j = g.usolve[v];
  const uint64_t sm = sd.seedmix[j];
  const int64_t off = sd.uoff[j];
  const uint64_t hv = priority(sm, it, lvl, 0, (uint32_t)(v - off));
  typename V::Row row = g.row(v, sd);
  const int result = jp_first_free<kJpBlockWords>(g, row, tid, nt, v, sm, off, hv, colour, it,
                                                  lvl, bits, BlockLdsSync());
  if (tid == 0) colour[v] = result;
  jp_release(g, row, tid, nt, v, sm, off, hv, cnt, sl, sh, it, lvl);
}

// One Jones-Plassmann round with its frontier sizes read on the device, so rounds can be
// launched back to back without a host round trip: round r colours the lists of parity r&1
// (sizes counts[r%3] and counts[3 + r%3]), appends the released units to the other lists
// (counters (r+1)%3) and clears the counters of round r+2.  Waves take the light units,
// then whole blocks take the heavy ones.  A round with empty frontiers does nothing.
template <class V>
__global__ __launch_bounds__(256) void k_jp_round(V g, SolveDev sd, JpLists L, int32_t *colour,
                                                  uint32_t *cnt, int r, int it, int lvl) {
  __shared__ uint64_t s_light[4][kJpLightWords];
  __shared__ uint64_t s_block[kJpBlockWords];
  __shared__ int32_t s_stage[4][2][kStage];
  const int64_t nf = L.counts[r % 3], nh = L.counts[3 + r % 3];
  const int p = r & 1;
  const int wv = threadIdx.x >> 6;
  // released units are staged per wave and written out in chunks
  WaveStage sl{s_stage[wv][0], L.light[p ^ 1], L.counts + (r + 1) % 3, 0};
  WaveStage sh{s_stage[wv][1], L.heavy[p ^ 1], L.counts + 3 + (r + 1) % 3, 0};
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    L.counts[(r + 2) % 3] = 0;
    L.counts[3 + (r + 2) % 3] = 0;
  }
  for (int64_t idx = (int64_t)blockIdx.x * 4 + wv; idx < nf; idx += (int64_t)gridDim.x * 4)
    jp_unit(g, sd, (int64_t)L.light[p][idx], colour, cnt, sl, sh, it, lvl, s_light[wv]);
  for (int64_t idx = blockIdx.x; idx < nh; idx += gridDim.x)
    jp_unit_block(g, sd, (int64_t)L.heavy[p][idx], colour, cnt, sl, sh, it, lvl, s_block);
  sl.flush();
  sh.flush();
}

// sort key of a unit for batching: colour, then degree bin
// (inactive: the key of units of solves that sit this iteration out, above every real key)
template <class V>
__global__ void k_batch_keys(V g, int64_t n, const int32_t *colour, const uint8_t *sactive,
                             uint32_t inactive, uint32_t *keys, uint32_t *vals) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  vals[v] = (uint32_t)v;
  if (!sactive[g.usolve[v]]) {
    keys[v] = inactive;
    return;
  }
  keys[v] = ((uint32_t)colour[v] << kBatchShift) | batch_slot(g, v);
}

template <class V>
__global__ void k_bin_keys(V g, int64_t n, const uint8_t *sactive, uint32_t *keys, uint32_t *vals) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  vals[v] = (uint32_t)v;
  uint32_t bin = kNumBins;
  if (sactive[g.usolve[v]]) bin = unit_bin(g, v);
  keys[v] = bin;
}
// first[key] = first position of key in a sorted key array (keys below nkeys only)
__global__ void k_key_bounds(const uint32_t *sk, int64_t n, uint32_t nkeys, int64_t *first) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t k = sk[i];
  if (k < nkeys && (i == 0 || sk[i - 1] != k)) first[k] = i;
}

// per unit of the global-table bin: table size (power of two >= 2*degree), by unit id
template <class V>
__global__ void k_gtab_sizes(V g, const int32_t *units, int64_t count, int64_t *sz, int32_t *lg) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  int64_t v = units[i];
  int64_t d = g.degree(v);
  int l = 4;
  while ((1ll << l) < 2 * d) l++;
  lg[v] = l;
  sz[i] = 1ll << l;
}
__global__ void k_gtab_assign(const int32_t *units, int64_t count, const int64_t *off,
                              int64_t *goff) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) goff[units[i]] = off[i];
}

// ------------------------------------------------------------------ small levels in one block
// For levels with few units the schedule is bounded by launch latency (a hundred colours,
// two launches per colour and sweep).  One workgroup of 1024 threads then runs the whole
// phase: Jones-Plassmann colouring, bucketing by colour, and every colour-batched sweep with
// block barriers between the decisions and the moves of each batch.  The arithmetic and the
// decisions are the same functions as in the multi-launch path.
struct SmallCtl {
  const int32_t *maxsw;    // [J] sweep cap per solve
  uint8_t *frozen;         // [J] solve takes no further moves at this level
  uint32_t *moved;         // [J] moves of the current sweep
  int64_t *sweeps, *moves, *caps;   // [J] per-solve statistics of this level (accumulated)
  int J;
  const uint32_t *limit;   // [slices] rebuild threshold of the Sigma sub-tables
  const uint32_t *nz;      // [slices] key bound after a rebuild
  int nslices;
  int64_t tab_total;
  int smax;                // largest sweep cap of the participating solves
};

constexpr int kSmallThreads = 1024;


constexpr int kSmallWaves = kSmallThreads / 64;

constexpr int kSmallRowThread = 32;   // rows counted by a single thread in a small level
template <class P, class V, bool kSweeps>
__global__ __launch_bounds__(kSmallThreads) void k_small_level(
    V g, SolveDev sd, int64_t n, const int32_t *work, int64_t nwork, uint32_t *comm,
    SliceTable sig, int32_t *colour, uint32_t *cnt, int32_t *fa, int32_t *fb, int32_t *order,
    int64_t *start, uint32_t *target, uint32_t *gk, int64_t *gv, int glg, SmallCtl ctl, int it,
    int lvl, int *ncol_out) {
  __shared__ uint32_t sk[kSmallWaves][1 << kWaveLg];
  __shared__ int64_t sv[kSmallWaves][1 << kWaveLg];
  __shared__ uint16_t sl[kSmallWaves][kWaveMaxDeg];
  __shared__ int sn[kSmallWaves];
  __shared__ uint64_t s_bits[kSmallWaves][kJpLightWords];
  __shared__ int64_t s_part[kSmallThreads];
  __shared__ uint32_t s_nf, s_nn;
  __shared__ int s_maxc, s_any, s_rb;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // ---- colouring: count higher-priority neighbours, then colour ready frontiers
  if (tid == 0) {
    s_nf = 0;
    s_maxc = -1;
  }
  __syncthreads();
  // rows up to kSmallRowThread entries are counted by one thread, longer ones by a wave
  for (int64_t i = wv; i < nwork; i += kSmallWaves) {
    const int64_t v = work[i];
    if (g.degree(v) <= kSmallRowThread) continue;
    const int j = g.usolve[v];
    const uint64_t sm = sd.seedmix[j];
    const int64_t off = sd.uoff[j];
    const uint64_t hv = priority(sm, it, lvl, 0, (uint32_t)(v - off));
    typename V::Row row = g.row(v, sd);
    int64_t c = 0;
    for (int64_t e = row.lo + lane; e < row.hi; e += 64) {
      int32_t x = g.col[e];
      if (g.wt(row, e, x) == 0) continue;
      if (outranks(priority(sm, it, lvl, 0, (uint32_t)(x - off)), (uint32_t)x, hv, (uint32_t)v)) c++;
    }
    for (int m = 32; m >= 1; m >>= 1) c += shfl_xor64(c, m);
    if (lane == 0) {
      cnt[v] = (uint32_t)c;
      colour[v] = -1;
      if (c == 0) fa[atomicAdd(&s_nf, 1u)] = (int32_t)v;
    }
  }
  for (int64_t i = tid; i < nwork; i += kSmallThreads) {
    const int64_t v = work[i];
    if (g.degree(v) > kSmallRowThread) continue;
    const int j = g.usolve[v];
    const uint64_t sm = sd.seedmix[j];
    const int64_t off = sd.uoff[j];
    const uint64_t hv = priority(sm, it, lvl, 0, (uint32_t)(v - off));
    typename V::Row row = g.row(v, sd);
    uint32_t c = 0;
    for (int64_t e = row.lo; e < row.hi; e++) {
      int32_t x = g.col[e];
      if (g.wt(row, e, x) == 0) continue;
      if (outranks(priority(sm, it, lvl, 0, (uint32_t)(x - off)), (uint32_t)x, hv, (uint32_t)v)) c++;
    }
    cnt[v] = c;
    colour[v] = -1;
    if (c == 0) fa[atomicAdd(&s_nf, 1u)] = (int32_t)v;
  }
  block_sync_global();
  int32_t *cur = fa, *nxt = fb;
  while (s_nf > 0) {
    const uint32_t nf = s_nf;
    __syncthreads();
    if (tid == 0) s_nn = 0;
    __syncthreads();
    for (uint32_t idx = wv; idx < nf; idx += kSmallWaves) {
      const int64_t v = cur[idx];
      const int j = g.usolve[v];
      const uint64_t sm = sd.seedmix[j];
      const int64_t off = sd.uoff[j];
      const uint64_t hv = priority(sm, it, lvl, 0, (uint32_t)(v - off));
      typename V::Row row = g.row(v, sd);
      const int result = jp_first_free<kJpLightWords>(g, row, lane, 64, v, sm, off, hv, colour,
                                                      it, lvl, s_bits[wv], WaveLdsSync());
      if (lane == 0) {
        colour[v] = result;
        atomicMax(&s_maxc, result);
      }
      for (int64_t e = row.lo + lane; e < row.hi; e += 64) {
        int32_t x = g.col[e];
        if (g.wt(row, e, x) == 0) continue;
        if (outranks(priority(sm, it, lvl, 0, (uint32_t)(x - off)), (uint32_t)x, hv, (uint32_t)v))
          continue;
        if (atomicSub(cnt + x, 1u) == 1u) nxt[atomicAdd(&s_nn, 1u)] = x;
      }
    }
    block_sync_global();
    if (tid == 0) s_nf = s_nn;
    int32_t *t = cur;
    cur = nxt;
    nxt = t;
    __syncthreads();
  }
  // ---- bucket the units by colour, or by (colour, degree bin) for the multi-launch sweeps
  const int ncol = s_maxc + 1;
  const int nkey = kSweeps ? ncol : kBatchSlots * ncol;
  auto key_of = [&](int64_t v) -> int {
    return kSweeps ? colour[v] : (colour[v] << kBatchShift) | (int)batch_slot(g, v);
  };
  // every hand-over of global memory between waves (plain stores, then atomics or loads of
  // other waves) goes through block_sync_global: a plain barrier does not wait for stores
  for (int c = tid; c <= nkey; c += kSmallThreads) start[c] = 0;
  block_sync_global();
  for (int64_t i = tid; i < nwork; i += kSmallThreads)
    atomicAdd(reinterpret_cast<unsigned long long *>(start + key_of(work[i]) + 1), 1ull);
  block_sync_global();
  // inclusive prefix sum of the key counts start[1..nkey]: contiguous chunks per thread, the
  // chunk totals scanned in LDS
  {
    int64_t *a = start + 1;
    const int64_t chunk = (nkey + kSmallThreads - 1) / kSmallThreads;
    const int64_t c0 = (int64_t)tid * chunk, c1 = c0 + chunk < nkey ? c0 + chunk : nkey;
    int64_t sum = 0;
    for (int64_t c = c0; c < c1; c++) sum += a[c];
    s_part[tid] = sum;
    __syncthreads();
    for (int o = 1; o < kSmallThreads; o <<= 1) {
      const int64_t t = tid >= o ? s_part[tid - o] : 0;
      __syncthreads();
      s_part[tid] += t;
      __syncthreads();
    }
    int64_t run = tid ? s_part[tid - 1] : 0;
    for (int64_t c = c0; c < c1; c++) {
      run += a[c];
      a[c] = run;
    }
  }
  if (tid == 0) *ncol_out = ncol;
  block_sync_global();
  // scatter: decisions inside a batch are independent and moves commute, so the order of
  // units inside a colour does not matter
  for (int c = tid; c < nkey; c += kSmallThreads) cnt[c] = (uint32_t)start[c];
  block_sync_global();
  for (int64_t i = tid; i < nwork; i += kSmallThreads) {
    const int32_t v = work[i];
    order[atomicAdd(cnt + key_of(v), 1u)] = v;
  }
  block_sync_global();
  if (!kSweeps) return;
  // ---- colour-batched sweeps
  LdsTab ltab{sk[wv], sv[wv], kWaveLg, sl[wv], sn + wv};
  const uint32_t gmask_lg = glg;
  for (int t = 0; t < ctl.smax; t++) {
    for (int j = tid; j < ctl.J; j += kSmallThreads) ctl.moved[j] = 0;
    block_sync_global();
    const uint32_t fresh_base = (uint32_t)(n * (int64_t)(1 + t));
    for (int c = 0; c < ncol; c++) {
      const int64_t lo = start[c], hi = start[c + 1];
      for (int64_t idx = lo + wv; idx < hi; idx += kSmallWaves) {
        const int64_t v = order[idx];
        uint32_t tg;
        if (g.degree(v) <= kWaveMaxDeg) {
          tg = lm_unit<P>(WaveGrp(), ltab, g, sd, v, comm, sig, fresh_base,
                          (typename P::Score *)nullptr, LmCounters{nullptr});
        } else {
          GTab gt{gk + ((int64_t)wv << gmask_lg), gv + ((int64_t)wv << gmask_lg), (int)gmask_lg};
          tg = lm_unit<P>(WaveGrp(), gt, g, sd, v, comm, sig, fresh_base,
                          (typename P::Score *)nullptr, LmCounters{nullptr});
        }
        if (lane == 0) target[idx] = tg;
      }
      block_sync_global();
      for (int64_t idx = lo + tid; idx < hi; idx += kSmallThreads) {
        const uint32_t C = target[idx];
        if (C == kNone) continue;
        const int64_t v = order[idx];
        const int j = g.usolve[v];
        if (ctl.frozen[j]) continue;
        const uint32_t D = comm[v];
        const int m = g.plen(v);
        for (int jj = 0; jj < m; jj++) {
          int gs;
          int64_t k;
          g.pent(v, jj, gs, k);
          tab_add(sig, gs, D, -(int32_t)k);
          tab_add(sig, gs, C, (int32_t)k);
        }
        comm[v] = C;
        atomicAdd(ctl.moved + j, 1u);
      }
      block_sync_global();
    }
    // per-solve stopping rules after the sweep
    if (tid == 0) {
      s_any = 0;
      s_rb = 0;
    }
    __syncthreads();
    for (int j = tid; j < ctl.J; j += kSmallThreads) {
      if (ctl.frozen[j]) continue;
      ctl.sweeps[j]++;
      ctl.moves[j] += ctl.moved[j];
      if (ctl.moved[j] == 0) {
        ctl.frozen[j] = 1;
      } else if (t == ctl.maxsw[j] - 1) {
        ctl.caps[j]++;
        ctl.frozen[j] = 1;
      } else {
        s_any = 1;
      }
    }
    for (int s2 = tid; s2 < ctl.nslices; s2 += kSmallThreads)
      if (sig.used[s2] > ctl.limit[s2]) s_rb = 1;
    block_sync_global();
    if (!s_any) break;
    if (s_rb) {   // compact the Sigma table: same contents, fewer dead keys
      for (int64_t i = tid; i < ctl.tab_total; i += kSmallThreads) sig.slots[i] = 0;
      block_sync_global();
      for (int64_t v = tid; v < n; v += kSmallThreads) {
        const int m = g.plen(v);
        for (int jj = 0; jj < m; jj++) {
          int gs;
          int64_t k;
          g.pent(v, jj, gs, k);
          tab_add(sig, gs, comm[v], (int32_t)k, false);
        }
      }
      for (int s2 = tid; s2 < ctl.nslices; s2 += kSmallThreads) sig.used[s2] = ctl.nz[s2];
      block_sync_global();
    }
  }
}

// ------------------------------------------------------------------ work-list segments
// Refinement work lists by degree: lane groups of 4, 8, 16 and 32 lanes (degree up to the
// group size), waves, LDS blocks, global tables.
constexpr int kRefLists = 7;
struct Segs {
  const int32_t *p[kRefLists];
  int64_t pre[kRefLists + 1];   // prefix sums of the segment lengths
  __device__ int seg(int64_t i) const {
    int k = 0;
    while (k < kRefLists - 1 && i >= pre[k + 1]) k++;
    return k;
  }
  __device__ int64_t unit(int64_t i) const {
    const int k = seg(i);
    return p[k][i - pre[k]];
  }
  __device__ int64_t total() const { return pre[kRefLists]; }
};
struct SegOut {
  int32_t *p[kRefLists];
};

// keep the units whose flag is still set, segment by segment
__global__ __launch_bounds__(256) void k_compact_segs(Segs in, const uint8_t *flag, SegOut out,
                                                      uint32_t *cnt) {
  __shared__ uint32_t s_app[256 / 64 + 1];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < in.total();
  const int ks = live ? in.seg(i) : -1;
  // a block may straddle segments: append segment by segment, one atomic per block and list
  for (int k = 0; k < kRefLists; k++) {
    bool keep = false;
    int32_t v = 0;
    if (ks == k) {
      v = (int32_t)in.unit(i);
      keep = flag[v] != 0;
    }
    if (__syncthreads_or(ks == k)) block_append(out.p[k], cnt + k, keep, v, s_app);
  }
}

// ------------------------------------------------------------------ refinement
// Leiden refinement inside each community (Section 3.2 citing Traag et al.): singletons
// that are well connected to their community merge into well-connected sub-communities
// of positive gain; a proposer merges only if it outranks every proposing neighbour of
// its community, so each merge joins a frozen sub-community along an edge and
// sub-communities stay connected.

// Rows up to kRefThreadRow entries are scanned by the unit's own thread; longer ones are set
// aside for a wave each (most units of a refinement pass need no scan at all).
constexpr int kRefThreadRow = 64;

// Refinement starts from singletons: R = id, ext = weight to the own community, slice mask,
// and each unit's Sigma in the refined table.  first/step: this thread's share of the row
// and profile (a thread for a short row, a wave's lanes for a long one).
template <class V>
__device__ inline void ref_init_unit(const V &g, const SolveDev &sd, int64_t v,
                                     const uint32_t *comm, uint32_t *R, int64_t *ext,
                                     uint64_t *mask, SliceTable sr, int first, int step,
                                     bool wave) {
  const uint32_t D = comm[v];
  typename V::Row row = g.row(v, sd);
  int64_t s = 0;
  for (int64_t e = row.lo + first; e < row.hi; e += step) {
    int32_t x = g.col[e];
    if (comm[x] == D) s += g.wt(row, e, x);
  }
  if (wave) s = wave_sum64(s);
  const int m = g.plen(v);
  const int j = g.usolve[v];
  uint64_t mk = 0;
  for (int jj = 0; jj < m; jj++) {
    int gs;
    int64_t k;
    g.pent(v, jj, gs, k);
    mk |= 1ull << (gs - sd.sfirst[j]);
    if (jj % step == first) tab_add(sr, gs, (uint32_t)v, (int32_t)k, false);
  }
  if (first == 0) {
    R[v] = (uint32_t)v;
    ext[v] = s;
    mask[v] = mk;
  }
}

template <class V>
__global__ __launch_bounds__(256) void k_ref_init(V g, SolveDev sd, int64_t n, const uint32_t *comm,
                                                  uint32_t *R, int64_t *ext, uint64_t *mask,
                                                  SliceTable sr, int32_t *wide, uint32_t *nwide) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = v < n;
  const bool defer = live && (g.degree(v) > kRefThreadRow || g.plen(v) > kRefThreadRow);
  if (live && !defer) ref_init_unit(g, sd, v, comm, R, ext, mask, sr, 0, 1, false);
  wave_append(wide, nwide, defer, (int32_t)v);
}

template <class V>
__global__ __launch_bounds__(256) void k_ref_init_wide(V g, SolveDev sd, const int32_t *wide,
                                                       const uint32_t *nwide,
                                                       const uint32_t *comm, uint32_t *R,
                                                       int64_t *ext, uint64_t *mask,
                                                       SliceTable sr) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = *nwide;
  for (int64_t idx = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); idx < nw;
       idx += (int64_t)gridDim.x * 4)
    ref_init_unit(g, sd, (int64_t)wide[idx], comm, R, ext, mask, sr, lane, 64, true);
}

// Well-connectedness of sub-community T within its community K:
//   q*ext(T) - p*b * sum_s x_s (K_s - x_s) / S_s >= 0,  x_s = Sigma_R(T, s), K_s = Sigma(K, s).
template <class V>
__global__ __launch_bounds__(256) void k_ref_wc(V g, SolveDev sd, const int32_t *list,
                                                int64_t count, const uint32_t *comm,
                                                const int64_t *ext, const uint64_t *mask,
                                                SliceTable sr, SliceTable sig, uint8_t *wcT,
                                                uint8_t *active, uint32_t *changed) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int64_t T = list ? list[i] : i;
  if (changed) changed[T] = 0;
  const int j = g.usolve[T];
  const int64_t q = sd.q[j], pb = sd.pb[j];
  const uint32_t K = comm[T];
  const int base = sd.sfirst[j];
  uint64_t mk = mask[T];
  int m = 0;
  int gs0 = 0;
  int64_t c0 = 0;
  double acc = 0, mag = 0;
  for (uint64_t b = mk; b; b &= b - 1) {
    int gs = base + __builtin_ctzll(b);
    int64_t x = tab_get(sr, gs, (uint32_t)T);
    if (x == 0) continue;
    int64_t c = x * ((int64_t)tab_get(sig, gs, K) - x);
    if (m == 0) {
      gs0 = gs;
      c0 = c;
    }
    m++;
    double t = (double)c / (double)sd.S[gs];
    acc += t;
    mag += fabs(t);
  }
  int sign;
  if (m <= 1) {
    i128 val = (i128)q * ext[T] * (m ? sd.S[gs0] : 1) - (i128)pb * c0;
    sign = val < 0 ? -1 : (val > 0 ? 1 : 0);
  } else if (mag == 0.0 || pb == 0) {
    sign = ext[T] > 0 ? 1 : (ext[T] < 0 ? -1 : 0);
  } else {
    double qw = (double)q * (double)ext[T];
    double ap = qw - (double)pb * acc;
    double er = (double)(m + 8) * 0x1p-50 * (fabs(qw) + (double)pb * mag);
    if (fabs(ap) > er) {
      sign = ap > 0 ? 1 : -1;
    } else {
      atomicAdd(reinterpret_cast<unsigned long long *>(sd.fallbacks + j), 1ull);
      ExactAcc ea;
      ea.init();
      for (uint64_t b = mk; b; b &= b - 1) {
        int gs = base + __builtin_ctzll(b);
        int64_t x = tab_get(sr, gs, (uint32_t)T);
        if (x == 0) continue;
        ea.term(x * ((int64_t)tab_get(sig, gs, K) - x), sd.S[gs]);
      }
      sign = ea.sign(q, ext[T], pb);
    }
  }
  wcT[T] = sign >= 0;
  if (active) active[T] = sign >= 0;
}

// Proposal of one active singleton: best well-connected sub-community of positive gain.
template <class P, class V, class Grp, class Tab>
__device__ inline void ref_unit(Grp grp, Tab tab, const V &g, const SolveDev &sd, int64_t v,
                                const uint32_t *comm, const uint32_t *R, const uint8_t *wcT,
                                const SliceTable &sr, uint32_t *prop, uint32_t *propr,
                                uint32_t stamp, int64_t *propw, uint8_t *active,
                                typename P::Score *red, int64_t *sredW = nullptr,
                                uint32_t *sredL = nullptr) {
  const int r = grp.rank(), gsz = grp.size();
  for (int i = r; i < tab.size(); i += gsz) {
    tab.K[i] = 0;
    tab.V[i] = 0;
  }
  tab.reset(r);
  grp.sync();
  const uint32_t D = comm[v];
  typename V::Row row = g.row(v, sd);
  for (int64_t e = row.lo + r; e < row.hi; e += gsz) {
    int32_t x = g.col[e];
    if (comm[x] != D) continue;
    int64_t w = g.wt(row, e, x);
    if (w == 0) continue;
    tab.add(R[x], w);
  }
  grp.sync();
  UnitCtx u = unit_ctx(g, sd, v, D);
  const typename P::Score zero = P::make(g, u, sd, sr, kNone, 0, kEmpty);
  typename P::Score best = zero;
  int64_t hW;
  uint32_t hL;
  group_heaviest(grp, tab, kNone, wcT, hW, hL, sredW, sredL);
  bool coop = false;
  if constexpr (!V::kLevel0 && IsMulti<P>::value) coop = u.m >= kCoopMinM;
  if (coop) {
    if constexpr (!V::kLevel0 && IsMulti<P>::value) {
      // one profile slice per lane, subgroups take the sub-communities in turn (every lane of
      // a subgroup runs the same turns)
      const CoopLane c = coop_lane(g, u, sd, sr, r);
      const int sub = r / c.mp, nsub = gsz / c.mp;
      if (hL != kNone) {
        ScoreK s = coop_make(u, c, hL, hW, kTarget);
        if (P::cmp(g, u, sd, sr, s, zero) > 0) best = s;
      }
      const int nc = tab.count();
      for (int i0 = 0; i0 < nc; i0 += nsub * kCoopBatch) {
        uint32_t lab[kCoopBatch];
        int64_t W[kCoopBatch], y[kCoopBatch];
        bool ok[kCoopBatch];
        for (int k = 0; k < kCoopBatch; k++) {
          const int i = i0 + k * nsub + sub;
          const int h = i < nc ? tab.slot(i) : 0;
          const uint32_t key = i < nc ? tab.K[h] : 0u;
          lab[k] = key - 1;
          ok[k] = key != 0 && key - 1 != hL && wcT[key - 1];
          W[k] = ok[k] ? tab.V[h] : 0;
          ok[k] = ok[k] && !P::prunable(u, W[k], best);
        }
        coop_lookup<kCoopBatch>(c, lab, ok, y);
        for (int k = 0; k < kCoopBatch; k++) {
          if (!ok[k]) continue;
          ScoreK s = coop_score(u, c, lab[k], W[k], y[k], kTarget);
          if (P::cmp(g, u, sd, sr, s, zero) <= 0) continue;
          if (better<P>(g, u, sd, sr, s, best)) best = s;
        }
      }
    }
  } else {
    if (hL != kNone) {
      typename P::Score s = P::make(g, u, sd, sr, hL, hW, kTarget);
      if (P::cmp(g, u, sd, sr, s, zero) > 0) best = s;
    }
    const int nc = tab.count();
    for (int i = r; i < nc; i += gsz) {
      const int h = tab.slot(i);
      uint32_t key = tab.K[h];
      if (key == 0) continue;
      uint32_t T = key - 1;
      if (T == hL || !wcT[T]) continue;
      if (P::prunable(u, tab.V[h], best)) continue;
      typename P::Score s = P::make(g, u, sd, sr, T, tab.V[h], kTarget);
      if (P::cmp(g, u, sd, sr, s, zero) <= 0) continue;
      if (better<P>(g, u, sd, sr, s, best)) best = s;
    }
  }
  best = group_best<P>(grp, g, u, sd, sr, best, red);
  int64_t w = best.lab == kNone ? 0 : tab.get(best.lab);
  grp.sync();
  if (r == 0) {
    if (best.lab == kNone) {
      active[v] = 0;
    } else {
      prop[v] = best.lab;
      propw[v] = w;
      propr[v] = stamp;
    }
  }
}

// Proposals of units of degree <= G with G lanes each: neighbours inside the community are
// merged by sub-community with shuffles, every leader evaluates its sub-community (well
// connected, positive gain), and the group reduces to the best (ties to the lower label).
template <class P, class V, int G>
__global__ __launch_bounds__(256) void k_ref_group(V g, SolveDev sd, const int32_t *units,
                                                   int64_t count, const uint32_t *comm,
                                                   const uint32_t *R, const uint8_t *wcT,
                                                   SliceTable sr, uint32_t *prop, uint32_t *propr,
                                                   uint32_t stamp, int64_t *propw,
                                                   uint8_t *active) {
  const int lane = threadIdx.x & 63;
  const int gl = lane & (G - 1);
  const int gbase = lane & ~(G - 1);
  const int64_t idx = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
  if (idx >= count) return;   // whole groups leave together
  const int64_t v = units[idx];
  if (!active[v]) return;
  const uint32_t D = comm[v];
  typename V::Row row = g.row(v, sd);
  const int64_t e = row.lo + gl;
  uint32_t c = kNone;
  int64_t w = 0;
  if (e < row.hi) {
    const int32_t x = g.col[e];
    if (comm[x] == D) {
      w = g.wt(row, e, x);
      if (w != 0) c = R[x];
    }
  }
  int64_t wsum = 0;
  bool leader = c != kNone;
  for (int j = 0; j < G; j++) {
    const uint32_t cj = (uint32_t)__shfl((int)c, gbase + j, 64);
    const int64_t wj = __shfl(w, gbase + j, 64);
    if (cj == c) {
      wsum += wj;
      if (j < gl) leader = false;
    }
  }
  const UnitCtx u = unit_ctx(g, sd, v, D);
  const typename P::Score zero = P::make(g, u, sd, sr, kNone, 0, kEmpty);
  typename P::Score best = zero;
  if (leader && wcT[c]) {
    typename P::Score s = P::make(g, u, sd, sr, c, wsum, kTarget);
    if (P::cmp(g, u, sd, sr, s, zero) > 0) best = s;
  }
  for (int m = G / 2; m >= 1; m >>= 1) {
    typename P::Score o = P::shfl(best, m);
    if (better<P>(g, u, sd, sr, o, best)) best = o;
  }
  // the weight to the chosen sub-community sits with its leader
  const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << G) - 1)) << gbase;
  const uint64_t bal = __ballot(leader && c == best.lab) & gmask;
  const int src = bal ? __builtin_ctzll(bal) : gbase;
  const int64_t wb = __shfl(wsum, src, 64);
  if (gl == 0) {
    if (best.lab == kNone) {
      active[v] = 0;
    } else {
      prop[v] = best.lab;
      propw[v] = wb;
      propr[v] = stamp;
    }
  }
}

template <class P, class V>
__global__ __launch_bounds__(256) void k_ref_prop_wave(V g, SolveDev sd, const int32_t *units,
                                                       int64_t count, const uint32_t *comm,
                                                       const uint32_t *R, const uint8_t *wcT,
                                                       SliceTable sr, uint32_t *prop, uint32_t *propr,
                                                       uint32_t stamp, int64_t *propw,
                                                       uint8_t *active) {
  __shared__ uint32_t sk[4][1 << kWaveLg];
  __shared__ int64_t sv[4][1 << kWaveLg];
  __shared__ uint16_t sl[4][kWaveMaxDeg];
  __shared__ int sn[4];
  const int wv = threadIdx.x >> 6;
  const int64_t idx = (int64_t)blockIdx.x * 4 + wv;
  if (idx >= count) return;
  const int64_t v = units[idx];
  if (!active[v]) return;
  LdsTab tab{sk[wv], sv[wv], kWaveLg, sl[wv], sn + wv};
  ref_unit<P>(WaveGrp(), tab, g, sd, v, comm, R, wcT, sr, prop, propr, stamp, propw, active,
              (typename P::Score *)nullptr);
}

template <class P, class V, int NT>
__global__ __launch_bounds__(NT) void k_ref_prop_block(V g, SolveDev sd, const int32_t *units,
                                                         int64_t count, const uint32_t *comm,
                                                         const uint32_t *R, const uint8_t *wcT,
                                                         SliceTable sr, uint32_t *prop,
                                                         uint32_t *propr, uint32_t stamp,
                                                         int64_t *propw, uint8_t *active) {
  __shared__ uint32_t sk[1 << kBlockLg];
  __shared__ int64_t sv[1 << kBlockLg];
  __shared__ uint16_t sl[kBlockMaxDeg];
  __shared__ int sn;
  __shared__ typename P::Score red[NT / 64];
  __shared__ int64_t hw[NT / 64];
  __shared__ uint32_t hl[NT / 64];
  LdsTab tab{sk, sv, kBlockLg, sl, &sn};
  for (int64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const int64_t v = units[idx];
    if (!active[v]) continue;
    ref_unit<P>(BlockGrp(), tab, g, sd, v, comm, R, wcT, sr, prop, propr, stamp, propw, active,
                red, hw, hl);
  }
}

template <class P, class V>
__global__ __launch_bounds__(256) void k_ref_prop_gtab(V g, SolveDev sd, const int32_t *units,
                                                       int64_t count, const uint32_t *comm,
                                                       const uint32_t *R, const uint8_t *wcT,
                                                       SliceTable sr, uint32_t *prop, uint32_t *propr,
                                                       uint32_t stamp, int64_t *propw,
                                                       uint8_t *active, uint32_t *gk, int64_t *gv,
                                                       const int64_t *goff, const int32_t *glg) {
  __shared__ typename P::Score red[4];
  __shared__ int64_t hw[4];
  __shared__ uint32_t hl[4];
  for (int64_t idx = blockIdx.x; idx < count; idx += gridDim.x) {
    const int64_t v = units[idx];
    if (!active[v]) continue;
    GTab tab{gk + goff[v], gv + goff[v], glg[v]};
    ref_unit<P>(BlockGrpG(), tab, g, sd, v, comm, R, wcT, sr, prop, propr, stamp, propw, active,
                red, hw, hl);
  }
}

// A proposer merges when its target sub-community keeps all its members this round:
//  (a) the target's founder does not propose (sub-communities with two or more members never
//      propose), or
//  (b) the proposer outranks every proposing neighbour of its community, and the target's
//      founder proposes to a target whose own founder proposes (so the founder cannot move).
// Proposals and eligibility carry the round's stamp instead of being cleared.

template <class V>
__device__ inline bool ref_beaten(const V &g, const SolveDev &sd, int64_t v, const uint32_t *comm,
                                  const uint32_t *propr, uint32_t stamp, int first, int step,
                                  int it, int lvl) {
  const int j = g.usolve[v];
  const uint64_t sm = sd.seedmix[j];
  const int64_t off = sd.uoff[j];
  const uint64_t hv = priority(sm, it, lvl, 1, (uint32_t)(v - off));
  const uint32_t D = comm[v];
  typename V::Row row = g.row(v, sd);
  bool beaten = false;
  for (int64_t e = row.lo + first; e < row.hi; e += step) {
    int32_t x = g.col[e];
    if (comm[x] != D || propr[x] != stamp) continue;
    if (g.wt(row, e, x) == 0) continue;
    uint64_t hx = priority(sm, it, lvl, 1, (uint32_t)(x - off));
    if (outranks(hx, (uint32_t)x, hv, (uint32_t)v)) beaten = true;
  }
  return beaten;
}

template <class V>
__global__ __launch_bounds__(256) void k_ref_eligible(V g, SolveDev sd, Segs segs,
                                                      const uint32_t *comm, const uint32_t *prop,
                                                      const uint32_t *propr, uint32_t stamp,
                                                      uint32_t *elig, int32_t *wide,
                                                      uint32_t *nwide, int it, int lvl) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool defer = false;
  int64_t v = 0;
  if (idx < segs.total()) {
    v = segs.unit(idx);
    if (propr[v] == stamp) {
      const uint32_t T = prop[v];
      if (propr[T] != stamp) {
        elig[v] = stamp;
      } else if (propr[prop[T]] == stamp) {
        if (g.degree(v) > kRefThreadRow) defer = true;
        else if (!ref_beaten(g, sd, v, comm, propr, stamp, 0, 1, it, lvl)) elig[v] = stamp;
      }
    }
  }
  wave_append(wide, nwide, defer, (int32_t)v);
}

// the long rows set aside above, one wave each (their number is read on the device)
template <class V>
__global__ __launch_bounds__(256) void k_ref_eligible_wide(V g, SolveDev sd, const int32_t *wide,
                                                           const uint32_t *nwide,
                                                           const uint32_t *comm,
                                                           const uint32_t *propr, uint32_t stamp,
                                                           uint32_t *elig, int it, int lvl) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = *nwide;
  for (int64_t idx = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); idx < nw;
       idx += (int64_t)gridDim.x * 4) {
    const int64_t v = wide[idx];
    int beaten = ref_beaten(g, sd, v, comm, propr, stamp, lane, 64, it, lvl) ? 1 : 0;
    for (int m = 32; m >= 1; m >>= 1) beaten |= __shfl_xor(beaten, m, 64);
    if (lane == 0 && !beaten) elig[v] = stamp;
  }
}

// Merge every eligible proposer into its target; edges between co-joiners of the same target
// become internal as well.
template <class V>
__device__ inline void ref_merge(const V &g, const SolveDev &sd, int64_t v, const uint32_t *prop,
                                 const int64_t *propw, const uint32_t *elig, uint32_t stamp,
                                 uint32_t *R, int64_t *ext, uint64_t *mask, uint8_t *active,
                                 SliceTable sr, int first, int step, bool wave) {
  const uint32_t T = prop[v];
  typename V::Row row = g.row(v, sd);
  int64_t corr = 0;
  for (int64_t e = row.lo + first; e < row.hi; e += step) {
    int32_t x = g.col[e];
    if (elig[x] == stamp && prop[x] == T) corr += g.wt(row, e, x);
  }
  if (wave) corr = wave_sum64(corr);
  const int m = g.plen(v);
  for (int jj = first; jj < m; jj += step) {
    int gs;
    int64_t k;
    g.pent(v, jj, gs, k);
    tab_add(sr, gs, T, (int32_t)k, false);
  }
  if (first == 0) {
    R[v] = T;
    active[v] = 0;
    active[T] = 0;
    atomicAdd(reinterpret_cast<unsigned long long *>(ext + T),
              (unsigned long long)(ext[v] - 2 * propw[v] - corr));
    atomicOr(reinterpret_cast<unsigned long long *>(mask + T), (unsigned long long)mask[v]);
  }
}

template <class V>
__global__ __launch_bounds__(256) void k_ref_apply(V g, SolveDev sd, Segs segs, const uint32_t *prop,
                                                   const int64_t *propw, const uint32_t *elig,
                                                   uint32_t stamp, uint32_t *R, int64_t *ext,
                                                   uint64_t *mask, uint8_t *active,
                                                   int32_t *wide, uint32_t *nwide, SliceTable sr) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool defer = false;
  int64_t v = 0;
  if (idx < segs.total()) {
    v = segs.unit(idx);
    if (elig[v] == stamp) {
      if (g.degree(v) > kRefThreadRow || g.plen(v) > kRefThreadRow) defer = true;
      else ref_merge(g, sd, v, prop, propw, elig, stamp, R, ext, mask, active, sr, 0, 1, false);
    }
  }
  wave_append(wide, nwide, defer, (int32_t)v);
}

template <class V>
__global__ __launch_bounds__(256) void k_ref_apply_wide(V g, SolveDev sd, const int32_t *wide,
                                                        const uint32_t *nwide,
                                                        const uint32_t *prop,
                                                        const int64_t *propw,
                                                        const uint32_t *elig, uint32_t stamp,
                                                        uint32_t *R, int64_t *ext, uint64_t *mask,
                                                        uint8_t *active, SliceTable sr) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = *nwide;
  for (int64_t idx = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); idx < nw;
       idx += (int64_t)gridDim.x * 4)
    ref_merge(g, sd, (int64_t)wide[idx], prop, propw, elig, stamp, R, ext, mask, active, sr, lane,
              64, true);
}

// merges per solve and the queue of sub-communities that received members (convergent)
template <class V>
__global__ __launch_bounds__(256) void k_ref_post(V g, Segs segs, const uint32_t *prop,
                                                  const uint32_t *elig, uint32_t stamp,
                                                  uint32_t *changed, int32_t *clist,
                                                  uint32_t *ccount, uint32_t *nelig) {
  __shared__ uint32_t s_app[256 / 64 + 1];
  __shared__ uint32_t s_merges;
  __shared__ int s_j, s_mixed;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool merged = false, first = false;
  int j = 0;
  uint32_t T = 0;
  if (threadIdx.x == 0) {
    s_merges = 0;
    s_mixed = 0;
    s_j = -1;
  }
  __syncthreads();
  if (i < segs.total()) {
    const int64_t v = segs.unit(i);
    if (elig[v] == stamp) {
      merged = true;
      j = g.usolve[v];
      T = prop[v];
      first = atomicExch(changed + T, 1u) == 0u;
      atomicAdd(&s_merges, 1u);
      const int prev = atomicCAS(&s_j, -1, j);
      if (prev != -1 && prev != j) s_mixed = 1;
    }
  }
  __syncthreads();
  // one atomic per block when its merges all belong to one solve (the usual case)
  if (!s_mixed) {
    if (threadIdx.x == 0 && s_merges) atomicAdd(nelig + s_j, s_merges);
  } else {
    wave_count(nelig, j, merged);
  }
  block_append(clist, ccount, first, (int32_t)T, s_app);
}

// ------------------------------------------------------------------ aggregation helpers
__global__ void k_minmember(const uint32_t *R, int64_t n, const int32_t *usolve,
                            const uint8_t *cont, uint32_t *minm) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n && cont[usolve[u]]) atomicMin(minm + R[u], (uint32_t)u);
}
__global__ void k_flag_minm(const uint32_t *R, const uint32_t *minm, int64_t n, uint8_t *flag) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u < n) flag[u] = minm[R[u]] == (uint32_t)u;
}
// super-node id of each unit of a continuing solve (kNone for units of finished solves)
__global__ void k_rank_gather(const uint32_t *R, const uint32_t *minm, const int64_t *rank,
                              int64_t n, uint32_t *r) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  uint32_t m = minm[R[u]];
  r[u] = m == kNone ? kNone : (uint32_t)rank[m];
}

// key (r[u], r[x]) of every entry between different super-nodes, written at the entry's own
// position; dropped entries get the all-ones key, which sorts last
constexpr uint64_t kDropKey = ~0ull;
template <class V>
__global__ __launch_bounds__(256) void k_agg_keys(V g, SolveDev sd, int64_t n, const uint32_t *r,
                                                  int shift, uint64_t *keys, int64_t *vals) {
  const int lane = threadIdx.x & 63;
  const int64_t u = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (u >= n) return;
  const uint32_t ru = r[u];
  typename V::Row row = g.row(u, sd);
  for (int64_t e = row.lo + lane; e < row.hi; e += 64) {
    int32_t x = g.col[e];
    int64_t w = g.wt(row, e, x);
    uint32_t rx = ru == kNone ? kNone : r[x];
    bool emit = ru != kNone && w != 0 && rx != ru;
    keys[e] = emit ? (((uint64_t)ru << shift) | rx) : kDropKey;
    vals[e] = emit ? w : 0;
  }
}

// profile entries (r[u], slice) at fixed positions: level 0 one per unit, later pp[u] + j
__device__ inline int64_t prof_pos(const View0 &, int64_t u, int) { return u; }
__device__ inline int64_t prof_pos(const ViewK &g, int64_t u, int j) { return g.pp[u] + j; }
template <class V>
__global__ void k_agg_prof_keys(V g, int64_t n, const uint32_t *r, int shift, uint64_t *keys,
                                int32_t *vals) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n) return;
  int m = g.plen(u);
  if (V::kLevel0 && m == 0) {
    keys[u] = kDropKey;
    vals[u] = 0;
    return;
  }
  for (int jj = 0; jj < m; jj++) {
    int gs;
    int64_t k;
    g.pent(u, jj, gs, k);
    int64_t pos = prof_pos(g, u, jj);
    bool keep = r[u] != kNone;
    keys[pos] = keep ? (((uint64_t)r[u] << shift) | (uint32_t)gs) : kDropKey;
    vals[pos] = keep ? (int32_t)k : 0;
  }
}

// row bounds of a sorted key array (row = high 32 bits): rs[row] = first, re[row] = last + 1
// keys are (row << shift) | column, sorted
__global__ void k_row_bounds(const uint64_t *keys, int64_t m, int shift, int64_t *rs, int64_t *re) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  uint64_t row = keys[i] >> shift;
  if (i == 0 || (keys[i - 1] >> shift) != row) rs[row] = i;
  if (i == m - 1 || (keys[i + 1] >> shift) != row) re[row] = i + 1;
}
__global__ void k_row_cnt(const int64_t *rs, const int64_t *re, int64_t n, int64_t *cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = re[i] - rs[i];
}
__global__ void k_low_bits(const uint64_t *keys, int64_t m, int shift, int32_t *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = (int32_t)(keys[i] & ((1ull << shift) - 1));
}

template <class V>
__global__ void k_scatter_next(V g, int64_t n, const uint32_t *r, const uint32_t *P,
                               uint32_t *Pnext, int32_t *usolve_next) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= n || r[u] == kNone) return;
  Pnext[r[u]] = P[u];
  usolve_next[r[u]] = g.usolve[u];
}

__global__ void k_map_compose(int64_t *map0, const int64_t *lo, const int64_t *hi, int nr,
                              const uint32_t *r) {
  // ranges [lo[k], hi[k]) of level-0 units; grid-stride over their union
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int k = 0; k < nr; k++)
    for (int64_t i = lo[k] + tid; i < hi[k]; i += stride) map0[i] = r[map0[i]];
}

// ------------------------------------------------------------------ canonical labels by sort
__global__ void k_seg_heads(const uint32_t *sk, const uint32_t *sv, int64_t n, uint8_t *head,
                            uint8_t *ismin) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint8_t h = (i == 0 || sk[i] != sk[i - 1]) ? 1 : 0;
  head[i] = h;
  ismin[sv[i]] = h;
}
// segid = inclusive index of the segment (exclusive scan of heads at heads), minOf[seg] = unit
__global__ void k_seg_min(const uint32_t *sv, const uint8_t *head, const int64_t *segx, int64_t n,
                          uint32_t *minof) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && head[i]) minof[segx[i]] = sv[i];
}
__global__ void k_seg_label(const uint32_t *sv, const uint8_t *head, const int64_t *segx,
                            const uint32_t *minof, const int64_t *rank, int64_t n, uint32_t *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t seg = segx[i] + head[i] - 1;
  out[sv[i]] = (uint32_t)rank[minof[seg]];
}
__global__ void k_count_heads(const uint32_t *sv, const uint8_t *head, const int32_t *usolve,
                              int64_t n, uint32_t *cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool h = i < n && head[i];
  wave_count(cnt, h ? usolve[sv[i]] : 0, h);
}
__global__ void k_solve_label_keys(const uint32_t *lab, const int32_t *usolve, int64_t n,
                                   uint64_t *keys, int32_t *vals) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) {
    keys[v] = ((uint64_t)(uint32_t)usolve[v] << 32) | lab[v];
    vals[v] = (int32_t)v;
  }
}
__global__ void k_count_key_heads(const uint64_t *keys, int64_t n, uint32_t *cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool h = i < n && (i == 0 || keys[i] != keys[i - 1]);
  wave_count(cnt, h ? (int)(keys[i] >> 32) : 0, h);
}
__global__ void k_fingerprint(const uint32_t *lab, int64_t n, unsigned long long *acc) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) atomicAdd(acc, (unsigned long long)mix64(((uint64_t)v << 32) | lab[v]));
}
__global__ void k_offset_labels(const int32_t *lab, const int32_t *usolve, const int64_t *uoff,
                                int64_t n, uint32_t *out) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) out[v] = (uint32_t)(uoff[usolve[v]] + lab[v]);
}
// Each solve's labels by first appearance from the union's canonical labels (communities
// ranked by their smallest member over the whole union): the solve's first unit is the
// smallest member of its community, so its rank counts the communities of earlier solves.
__global__ void k_local_labels(const uint32_t *comm, const int32_t *usolve, const int64_t *uoff,
                               int64_t n, int32_t *out) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) out[v] = (int32_t)(comm[v] - comm[uoff[usolve[v]]]);
}
__global__ void k_count_roots_R(const uint32_t *R, const int32_t *usolve, int64_t n, uint32_t *cnt) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool h = u < n && R[u] == (uint32_t)u;
  wave_count(cnt, h ? usolve[u] : 0, h);
}
__global__ void k_count_flags(const uint8_t *flag, const int32_t *usolve, int64_t n, uint32_t *cnt) {
  int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool h = u < n && flag[u];
  wave_count(cnt, h ? usolve[u] : 0, h);
}

// ------------------------------------------------------------------ split into connected parts
__device__ inline int32_t uf_find(int32_t *parent, int32_t x) {
  for (;;) {
    int32_t p = __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p == x) return x;
    int32_t gp = __hip_atomic_load(parent + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (gp != p) __hip_atomic_store(parent + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = p;
  }
}
__device__ inline void uf_unite(int32_t *parent, int32_t a, int32_t b) {
  for (;;) {
    a = uf_find(parent, a);
    b = uf_find(parent, b);
    if (a == b) return;
    if (a < b) {
      int32_t t = a;
      a = b;
      b = t;
    }
    // link the larger root under the smaller one: roots stay component minima
    if (atomicCAS(parent + a, a, b) == a) return;
  }
}

__global__ void k_uf_init(int32_t *parent, const int64_t *lo, const int64_t *hi, int nr) {
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int k = 0; k < nr; k++)
    for (int64_t i = lo[k] + tid; i < hi[k]; i += stride) parent[i] = (int32_t)i;
}

__global__ __launch_bounds__(256) void k_uf_link(View0 g, SolveDev sd, const int64_t *lo,
                                                 const int64_t *hi, int nr, const uint32_t *lab,
                                                 int32_t *parent) {
  const int lane = threadIdx.x & 63;
  int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int k = 0; k < nr; k++)
    for (int64_t v = lo[k] + wid; v < hi[k]; v += nw) {
      View0::Row row = g.row(v, sd);
      const uint32_t L = lab[v];
      for (int64_t e = row.lo + lane; e < row.hi; e += 64) {
        int32_t x = g.col[e];
        if (x <= v || lab[x] != L || g.wt(row, e, x) == 0) continue;
        uf_unite(parent, (int32_t)v, x);
      }
    }
}

// Root of every element into a separate array: other threads' path halving keeps rewriting
// parent[] with ancestors while this runs, so parent[] itself is not a root map afterwards.
__global__ void k_uf_roots(int32_t *parent, const int64_t *lo, const int64_t *hi, int nr,
                           uint8_t *isroot, int32_t *root) {
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int k = 0; k < nr; k++)
    for (int64_t i = lo[k] + tid; i < hi[k]; i += stride) {
      int32_t r = uf_find(parent, (int32_t)i);
      root[i] = r;
      isroot[i] = r == (int32_t)i;
    }
}

// memb[i] = rank of i's root among the roots of its range; root and memb may alias
__global__ void k_label_out(const int32_t *root, const int64_t *rank, const int64_t *lo,
                            const int64_t *hi, const int64_t *roff, int nr, int32_t *memb) {
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int k = 0; k < nr; k++)
    for (int64_t i = lo[k] + tid; i < hi[k]; i += stride)
      memb[i] = (int32_t)(rank[root[i]] - roff[k]);
}

__global__ void k_flatten(const int64_t *map0, const uint32_t *P, const int64_t *lo,
                          const int64_t *hi, int nr, uint32_t *flat) {
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int k = 0; k < nr; k++)
    for (int64_t i = lo[k] + tid; i < hi[k]; i += stride) flat[i] = P[map0[i]];
}

__global__ void k_count_diff(const int32_t *a, const int32_t *b, const int32_t *usolve,
                             const int64_t *lo, const int64_t *hi, int nr, uint32_t *diff) {
  // convergent loops: every lane of a wave runs the same iterations
  const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) & ~63ll;
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int k = 0; k < nr; k++)
    for (int64_t b0 = lo[k] + wave0; b0 < hi[k]; b0 += stride) {
      int64_t i = b0 + lane;
      bool d = i < hi[k] && a[i] != b[i];
      wave_count(diff, d ? usolve[i] : 0, d);
    }
}

// ------------------------------------------------------------------ Q components
// W_s: intra weight inside communities (both directions, unscaled) per global slice; one
// thread per unit, sums merged per wave by slice
__global__ void k_q_w(View0 g, int64_t n, const int32_t *memb, int64_t *W) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t s = 0;
  int gs = 0;
  if (v < n) {
    gs = g.uslice[v];
    const int64_t slo = g.sstart[gs], shi = g.sstart[gs + 1];
    const int32_t L = memb[v];
    for (int64_t e = g.rp[v]; e < g.rp[v + 1]; e++) {
      int32_t x = g.col[e];
      if (x >= slo && x < shi && memb[x] == L) s += g.w ? g.w[e] : 1;
    }
  }
  wave_add64(W, gs, s);
}

// Sigma of a membership: per Sigma slice and label, the sum of the null-model degrees
__global__ void k_sigma_build_memb(View0 g, int64_t n, const int32_t *memb, SliceTable t) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int gs;
  int64_t k;
  g.pent(v, 0, gs, k);
  if (k > 0) tab_add(t, gs, (uint32_t)memb[v], (int32_t)k, false);
}

// Scaled supra-degree of every unit of one solve under the global null model:
// b*k_i^s + a*c with c the unit's coupling entries (1 in the first and last slice, 2 between,
// none for one slice).
__global__ void k_null_degree_global(const int32_t *k, const int64_t *rp, const int32_t *col,
                                     const int32_t *w, int64_t n, int64_t N, int64_t a, int64_t b,
                                     int32_t *out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int64_t lo = (v / N) * N, hi = lo + N;
  int64_t c = 0;   // the copy's coupling multipliers
  for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
    const int32_t x = col[e];
    if (x < lo || x >= hi) c += w ? w[e] : 1;
  }
  out[v] = (int32_t)(b * k[v] + a * c);
}

// CPM node weight: 1 per copy, or 0 for a copy without an intra edge when only present copies
// are coupled (it is then no supra-node)
__global__ void k_cpm_weight(const int32_t *kd, int64_t n, bool present_only, int32_t *out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) out[v] = (!present_only || kd[v] > 0) ? 1 : 0;
}

// SS per Sigma slice: sum over the slice's sub-table of value^2
__global__ void k_q_ss(const uint64_t *slots, const int64_t *base, int nslices, int64_t total,
                       int64_t *SS) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t sq = 0;
  int lo = 0;
  if (i < total) {
    uint64_t e = slots[i];
    int64_t val = (uint32_t)e ? (int32_t)(e >> 32) : 0;
    sq = val * val;
    int hi = nslices;   // base[lo] <= i < base[hi]
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (base[mid] <= i) lo = mid; else hi = mid;
    }
  }
  wave_add64(SS, lo, sq);
}

// I: ordered coupled copy pairs (i,s),(i,s+1) sharing a community, per solve
__global__ void k_q_inter(View0 g, int64_t n, const int32_t *memb, int64_t *I) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t add = 0;
  int j = 0;
  if (v < n) {   // the coupling entries of v (both directions are counted, one per row)
    const int gs = g.uslice[v];
    const int64_t lo = g.sstart[gs], hi = g.sstart[gs + 1];
    j = g.usolve[v];
    for (int64_t e = g.rp[v]; e < g.rp[v + 1]; e++) {
      const int32_t x = g.col[e];
      if ((x < lo || x >= hi) && memb[x] == memb[v]) add += g.w ? g.w[e] : 1;
    }
  }
  wave_add64(I, j, add);
}

// ------------------------------------------------------------------ small utilities
template <class T>
__global__ void k_fill(T *p, T val, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = val;
}
__global__ void k_iota_i32(int32_t *p, int64_t n, int64_t off) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)(i + off);
}
__global__ void k_iota_u32(uint32_t *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (uint32_t)i;
}
__global__ void k_fill_ranges(int32_t *out, const int64_t *lo, const int64_t *hi,
                              const int64_t *outoff, int nr) {
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int k = 0; k < nr; k++)
    for (int64_t i = tid; i < hi[k] - lo[k]; i += stride) out[outoff[k] + i] = (int32_t)(lo[k] + i);
}
__global__ void k_gather_i64(const int64_t *src, const int64_t *idx, int n, int64_t *dst) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}
__global__ void k_compact_flag(const uint8_t *flag, int64_t n, int32_t *out, uint32_t *cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[atomicAdd(cnt, 1u)] = (int32_t)i;
}

}  // namespace mslm
