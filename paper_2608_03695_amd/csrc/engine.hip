// Host driver of the deterministic multislice Leiden schedule (Section 3.2, Eq. 6).
//
// One call runs one or more solves as a disjoint union: every kernel launch covers all
// solves that are still active, and per-solve control (sweep convergence, level breaks,
// iteration stability) is applied from per-solve counters, so each solve follows exactly
// the schedule it would follow alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>

#include "engine.hpp"
#include "kernels.hpp"
#include "prims.hpp"

namespace mslm {

namespace {

constexpr int kBS = 256;

inline unsigned nblk(int64_t n, int bs = kBS) {
  int64_t b = (n + bs - 1) / bs;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 0x7fffffff));
}
inline unsigned nblk_cap(int64_t n, int64_t cap, int bs = kBS) {
  int64_t b = (n + bs - 1) / bs;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}
inline unsigned wblk(int64_t units) { return nblk(units, 4); }

int bits_for(uint64_t x) {
  int b = 1;
  while (b < 64 && (1ull << b) <= x) b++;
  return b;
}

template <class T>
void fill(T *p, T val, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  k_fill<T><<<nblk_cap(n, 65536), kBS, 0, st>>>(p, val, n);
}

template <class T>
void h2d(T *dst, const T *src, int64_t n, hipStream_t st) {
  if (n > 0) MSLM_HIP(hipMemcpyAsync(dst, src, sizeof(T) * n, hipMemcpyHostToDevice, st));
}
template <class T>
void d2h(T *dst, const T *src, int64_t n, hipStream_t st) {
  if (n > 0) MSLM_HIP(hipMemcpyAsync(dst, src, sizeof(T) * n, hipMemcpyDeviceToHost, st));
}

}  // namespace

// ------------------------------------------------------------------ device memory source
namespace {
std::mutex g_alloc_mu;
DevAlloc g_alloc;
}  // namespace

DevAlloc current_allocator() {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  return g_alloc;
}
void set_allocator(const DevAlloc &a) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc = a;
}
Arena *&thread_arena() {
  static thread_local Arena *a = nullptr;
  return a;
}
std::atomic<int64_t> *&thread_account() {
  static thread_local std::atomic<int64_t> *a = nullptr;
  return a;
}

// ------------------------------------------------------------------ workspace
struct LevelBufs {
  Buf rp, col, w, pp, ps, pk, usolve;
};

struct Workspace {
  Buf temp;
  // union level 0
  Buf u_rp, u_col, u_w, u_k, u_uslice, u_usolve, u_sstart, u_pmap, u_rev;
  // per solve / per slice
  Buf s_p, s_q, s_pb, s_a, s_b, s_seed, s_uoff, s_sfirst, s_slast, s_S, s_frozen, s_cnt, s_cnt2;
  Buf fallbacks;
  // state
  Buf pcur, pnew, comm, comm2, map0, pflat, parent, isroot, rank0;
  Buf colour, work0, work1, nwork, bkeys, bvals, bkeys2, bvals2, hist, target;
  Buf gk, gv, goff, glg;
  Buf sig_slots, sig_base, sig_shift, sig_used, sig_limit, sr_slots, sr_used, flag;
  Buf R, ext, mask, active, wcT, elig, changed, clist, ccount, prop, propr, propw;
  Buf r, minm, flag8, rank, akeys, avals, akeys2, avals2, nuniq, rowcnt, pkeys, pvals, pkeys2,
      pvals2, pnext;
  Buf ckeys, cvals, ckeys2, cvals2, head, ismin, segx, minof, crank;
  Buf qW, qSS, qI, ranges_lo, ranges_hi, ranges_off;
  Buf sm_maxsw, sm_stat, sm_nz, sm_start;
  Buf b_src, b_dst, b_w, b_off, b_twom;   // graph build inputs and per-slice sums
  Buf b_pairs, b_present;                 // coupled slice pairs, present copies (build)
  Buf hubpart;                            // per-block best candidates of hub units
  Buf jph0, jph1;                         // heavy frontier lists of the colouring
  Buf sig_count;                          // profile entries per slice of a level
  Buf comm_snap;                          // labels at the start of a sweep (for a redo)
  Buf s_redo;                             // per-solve redo flags of a sweep
  Buf ref_wide, ref_wcnt;                 // refinement units with long rows, and their count
  Buf ref_snap_a, ref_snap_p;             // active flags and proposal stamps before a round
  Buf ref_keep;                           // active flags of solves that skip a round's redo
  Buf lat_part, lat_done;                 // latency mode: candidates split among blocks
  // sweeps replayed from HIP graphs: a private stream (default priority) joined to the solve
  // stream by events, the fresh-label base on the device, and a switch that turns graphs off
  // after a failed capture
  hipStream_t gstream = nullptr;
  hipEvent_t gev0 = nullptr, gev1 = nullptr;
  bool graphs_off = false;
  Buf fresh;
  // level 0 in colour-batch order (local-moving sweeps)
  Buf p_pos, p_deg, p_rp, p_col, p_w, p_k, p_slice, p_solve, p_iota, p_comm, p_goff, p_glg,
      p_wide, p_nwide, p_sk, p_sk2, p_units, p_elab, p_prev;
  LevelBufs lvA, lvB;
  std::vector<hipEvent_t> evpool;
};

Workspace *workspace_new() { return new Workspace(); }
void workspace_free(Workspace *ws) {
  if (!ws) return;
  for (auto e : ws->evpool) (void)hipEventDestroy(e);
  if (ws->gev0) (void)hipEventDestroy(ws->gev0);
  if (ws->gev1) (void)hipEventDestroy(ws->gev1);
  if (ws->gstream) (void)hipStreamDestroy(ws->gstream);
  delete ws;
}

void workspace_release_build(Workspace *ws) {
  if (!ws) return;
  for (Buf *b : {&ws->b_src, &ws->b_dst, &ws->b_w, &ws->akeys, &ws->akeys2, &ws->avals,
                 &ws->avals2, &ws->temp, &ws->b_pairs, &ws->b_present})
    b->release();
}

static void *temp_get(void *ctx, size_t bytes) {
  return static_cast<Workspace *>(ctx)->temp.ensure(bytes);
}

static TempAlloc temp_alloc(Workspace *ws) { return TempAlloc{temp_get, ws}; }

#define MSLM_PRIM(call) MSLM_HIP(call)

// ------------------------------------------------------------------ graph build (Eq. 3)
namespace {

__global__ void k_build_validate(const int32_t *src, const int32_t *dst, const int32_t *w,
                                 int64_t E, int32_t N, int *bad) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  int32_t u = src[e], x = dst[e];
  if (u < 0 || u >= N || x < 0 || x >= N || u == x || (w && w[e] < 1)) atomicOr(bad, 1);
}

// every intra edge in both directions, keyed (row, col); the slice comes from the offsets
__global__ void k_build_intra(const int32_t *src, const int32_t *dst, const int32_t *w,
                              const int64_t *off, int32_t T, int32_t N, int64_t E, int shift,
                              uint64_t *keys, int64_t *vals) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  int lo = 0, hi = T;   // off[lo] <= e < off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= e) lo = mid; else hi = mid;
  }
  int64_t base = (int64_t)lo * N;
  uint64_t u = (uint64_t)(base + src[e]), x = (uint64_t)(base + dst[e]);
  int64_t ww = w ? w[e] : 1;
  keys[2 * e] = (u << shift) | x;
  vals[2 * e] = ww;
  keys[2 * e + 1] = (x << shift) | u;
  vals[2 * e + 1] = ww;
}

// copies with an intra edge (present): both ends of every edge of a slice
__global__ void k_mark_present(const int32_t *src, const int32_t *dst, const int64_t *off,
                               int32_t T, int32_t N, int64_t E, uint8_t *present) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  int lo = 0, hi = T;   // off[lo] <= e < off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= e) lo = mid; else hi = mid;
  }
  present[(int64_t)lo * N + src[e]] = 1;
  present[(int64_t)lo * N + dst[e]] = 1;
}

// coupling entries (i,s)<->(i,r) of the coupled slice pairs p = (ps[p], pr[p], c[p]), raw weight
// c_sr (scaled by a at use); with `present`, a pair of copies not both present gets the key
// all-ones in the sort's 2*shift bits (never an entry: it would be a self-loop), which sorts
// last and is dropped
__global__ void k_build_inter(int32_t N, int64_t P, const int32_t *ps, const int32_t *pr,
                              const int32_t *pc, const uint8_t *present, int shift,
                              uint64_t *keys, int64_t *vals) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)N * P) return;
  const int64_t p = t / N, i = t - p * N;
  uint64_t v = (uint64_t)((int64_t)ps[p] * N + i), x = (uint64_t)((int64_t)pr[p] * N + i);
  int64_t c = pc[p];
  if (present && !(present[v] && present[x])) {
    v = x = (1ull << shift) - 1;
    c = 0;
  }
  keys[2 * t] = (v << shift) | x;
  vals[2 * t] = c;
  keys[2 * t + 1] = (x << shift) | v;
  vals[2 * t + 1] = c;
}

// coupling total: sum of the raw coupling weights over all entries (both directions)
__global__ void k_coupling_total(const int64_t *rp, const int32_t *col, const int32_t *w,
                                 int64_t n, int32_t N, unsigned long long *out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long t = 0;
  if (v < n) {
    const int64_t lo = (v / N) * N, hi = lo + N;
    for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
      const int32_t x = col[e];
      if (x < lo || x >= hi) t += (unsigned long long)w[e];
    }
  }
  for (int m = 32; m >= 1; m >>= 1) t += __shfl_xor(t, m, 64);
  if ((threadIdx.x & 63) == 0 && t) atomicAdd(out, t);
}

__global__ void k_build_csr(const uint64_t *keys, const int64_t *vals, int64_t m, int shift,
                            int32_t *col, int32_t *w, int64_t *rowcnt, int *nonunit) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  uint64_t k = keys[i];
  col[i] = (int32_t)(k & ((1ull << shift) - 1));
  int64_t v = vals[i];
  w[i] = (int32_t)v;
  if (v > 1) atomicOr(nonunit, 1);
  atomicAdd(reinterpret_cast<unsigned long long *>(rowcnt + (k >> shift)), 1ull);
}

// Reverse entries: entry e = (u, x) (its sorted unique key) finds (x, u) in x's row, whose
// columns ascend, by binary search; the offset within x's row is stored.  The supra-graph is
// symmetric, so the search always succeeds.
__global__ void k_build_rev(const uint64_t *keys, int64_t m, int shift, const int64_t *rp,
                            const int32_t *col, int32_t *rev) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const uint64_t k = keys[e];
  const int32_t u = (int32_t)(k >> shift);
  const int64_t x = (int64_t)(k & ((1ull << shift) - 1));
  const int64_t r0 = rp[x];
  int64_t lo = r0, hi = rp[x + 1];   // col[lo] <= u < col[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (col[mid] <= u) lo = mid;
    else hi = mid;
  }
  rev[e] = (int32_t)(lo - r0);
}

// Intra degree of every unit and, per slice, 2m_s and the count of units with nonzero degree.
// A wave's units are consecutive, so they nearly always lie in one slice: the wave sums first
// and issues one atomic per counter (one atomic per unit on 64 addresses serialises).
__global__ void k_build_degree(const int64_t *rp, const int32_t *col, const int32_t *w, int64_t n,
                               int32_t N, int32_t *kdeg, int64_t *twom, int64_t *nz) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = v < n;
  const int64_t s = live ? v / N : -1;
  int64_t d = 0;
  if (live) {
    const int64_t lo = s * N, hi = lo + N;
    for (int64_t e = rp[v]; e < rp[v + 1]; e++) {
      int32_t x = col[e];
      if (x >= lo && x < hi) d += w[e];
    }
    kdeg[v] = (int32_t)(d < 0x7fffffff ? d : 0x7fffffff);
  }
  // lane 0 holds the wave's smallest unit, so it is live whenever any lane is
  const int64_t s0 = __shfl(s, 0, 64);
  if (__all(!live || s == s0)) {
    int64_t dd = d, z = d != 0;
    for (int m = 32; m >= 1; m >>= 1) {
      dd += shfl_xor64(dd, m);
      z += shfl_xor64(z, m);
    }
    if ((threadIdx.x & 63) == 0 && dd) {
      atomicAdd(reinterpret_cast<unsigned long long *>(twom + s0), (unsigned long long)dd);
      atomicAdd(reinterpret_cast<unsigned long long *>(nz + s0), (unsigned long long)z);
    }
  } else if (d) {
    atomicAdd(reinterpret_cast<unsigned long long *>(twom + s), (unsigned long long)d);
    atomicAdd(reinterpret_cast<unsigned long long *>(nz + s), 1ull);
  }
}

__global__ void k_max_degree(const int64_t *rp, int64_t n, int *mx) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int d = v < n ? (int)std::min<int64_t>(rp[v + 1] - rp[v], 0x7fffffff) : 0;
  for (int m = 32; m >= 1; m >>= 1) d = max(d, __shfl_xor(d, m, 64));
  if ((threadIdx.x & 63) == 0 && d > 0) atomicMax(mx, d);
}

}  // namespace

void build_graph(GraphDev &g, const mslm_graph_desc &d, hipStream_t st, Workspace *ws) {
  const int32_t N = d.n_nodes, T = d.n_slices;
  const int64_t E = d.slice_offsets[T];
  const int64_t n = (int64_t)N * T;
  // the coupled slice pairs (s < r, c_sr > 0) of the coupling matrix
  const std::vector<int32_t> cm = api_coupling_matrix(&d);
  std::vector<int32_t> hps, hpr, hpc;
  for (int s = 0; s < T; s++)
    for (int r = s + 1; r < T; r++)
      if (cm[(size_t)s * T + r]) {
        hps.push_back(s);
        hpr.push_back(r);
        hpc.push_back(cm[(size_t)s * T + r]);
      }
  const int64_t P = (int64_t)hps.size();
  const int64_t ninter = (int64_t)N * P;
  const int64_t mraw = 2 * E + 2 * ninter;
  const bool on_dev = d.flags & MSLM_INPUT_ON_DEVICE;
  const bool present_only = d.flags & MSLM_COUPLE_PRESENT;
  g.N = N;
  g.T = T;
  g.n = n;
  g.crow = api_coupling_rows(cm, T);
  g.present_only = present_only;
  // edge lists on the device (workspace buffers: repeated builds allocate nothing new)
  const int32_t *src = d.src, *dst = d.dst, *w = d.weight;
  if (!on_dev) {
    src = ws->b_src.get<int32_t>(E);
    dst = ws->b_dst.get<int32_t>(E);
    h2d(const_cast<int32_t *>(src), d.src, E, st);
    h2d(const_cast<int32_t *>(dst), d.dst, E, st);
    if (d.weight) {
      w = ws->b_w.get<int32_t>(E);
      h2d(const_cast<int32_t *>(w), d.weight, E, st);
    }
  }
  int64_t *off = ws->b_off.get<int64_t>(T + 1);
  h2d(off, d.slice_offsets, T + 1, st);
  if (on_dev && E > 0) {   // host validation covers host inputs; device inputs are checked here
    int *bad = ws->flag.get<int>(1);
    MSLM_HIP(hipMemsetAsync(bad, 0, sizeof(int), st));
    k_build_validate<<<nblk(E), kBS, 0, st>>>(src, dst, w, E, N, bad);
    int hbad = 0;
    d2h(&hbad, bad, 1, st);
    MSLM_HIP(hipStreamSynchronize(st));
    if (hbad) throw Error(MSLM_EINVAL, "edge list has an id out of range, a self-loop or a weight < 1");
  }
  // keys (row << b) | column with b the bits of n: the sort covers the bits in use
  const int shift = bits_for((uint64_t)n);
  uint64_t *k1 = ws->akeys.get<uint64_t>(mraw);
  int64_t *v1 = ws->avals.get<int64_t>(mraw);
  if (E > 0) k_build_intra<<<nblk(E), kBS, 0, st>>>(src, dst, w, off, T, N, E, shift, k1, v1);
  if (ninter > 0) {
    int32_t *dp = ws->b_pairs.get<int32_t>(3 * P);
    h2d(dp, hps.data(), P, st);
    h2d(dp + P, hpr.data(), P, st);
    h2d(dp + 2 * P, hpc.data(), P, st);
    uint8_t *pres = nullptr;
    if (present_only) {
      pres = ws->b_present.get<uint8_t>(n);
      MSLM_HIP(hipMemsetAsync(pres, 0, n, st));
      if (E > 0) k_mark_present<<<nblk(E), kBS, 0, st>>>(src, dst, off, T, N, E, pres);
    }
    k_build_inter<<<nblk(ninter), kBS, 0, st>>>(N, P, dp, dp + P, dp + 2 * P, pres, shift,
                                                k1 + 2 * E, v1 + 2 * E);
  }
  uint64_t *k2 = ws->akeys2.get<uint64_t>(mraw);
  int64_t *v2 = ws->avals2.get<int64_t>(mraw);
  MSLM_PRIM(sort_pairs_u64_i64(k1, k2, v1, v2, mraw, 2 * shift, st, temp_alloc(ws)));
  int64_t *dn = ws->nuniq.get<int64_t>(1);
  MSLM_PRIM(reduce_by_key_u64_i64(k2, k1, v2, v1, dn, mraw, st, temp_alloc(ws)));
  int64_t m = 0;
  d2h(&m, dn, 1, st);
  MSLM_HIP(hipStreamSynchronize(st));
  if (present_only && m > 0) {   // the dropped pairs' key sorts last
    uint64_t last = 0;
    d2h(&last, k1 + m - 1, 1, st);
    MSLM_HIP(hipStreamSynchronize(st));
    const uint64_t drop = (2 * shift >= 64) ? ~0ull : ((1ull << (2 * shift)) - 1);
    if (last == drop) m--;
  }
  g.nnz = m;
  int32_t *col = g.col.get<int32_t>(m);
  int32_t *wv = g.w.get<int32_t>(m);
  int64_t *cnt = ws->rowcnt.get<int64_t>(n + 1);
  int *flags = ws->flag.get<int>(2);
  MSLM_HIP(hipMemsetAsync(cnt, 0, sizeof(int64_t) * (n + 1), st));
  MSLM_HIP(hipMemsetAsync(flags, 0, sizeof(int) * 2, st));
  if (m > 0) k_build_csr<<<nblk(m), kBS, 0, st>>>(k1, v1, m, shift, col, wv, cnt, flags);
  int64_t *rp = g.rp.get<int64_t>(n + 1);
  MSLM_PRIM(exclusive_sum_i64(cnt, rp, n + 1, st, temp_alloc(ws)));
  int32_t *rev = g.rev.get<int32_t>(m);
  if (m > 0) k_build_rev<<<nblk(m), kBS, 0, st>>>(k1, m, shift, rp, col, rev);
  int32_t *kd = g.k.get<int32_t>(n);
  int64_t *twom = ws->b_twom.get<int64_t>(2 * T);
  MSLM_HIP(hipMemsetAsync(twom, 0, sizeof(int64_t) * 2 * T, st));
  k_build_degree<<<nblk(n), kBS, 0, st>>>(rp, col, wv, n, N, kd, twom, twom + T);
  k_max_degree<<<nblk(n), kBS, 0, st>>>(rp, n, flags + 1);
  unsigned long long *ct = reinterpret_cast<unsigned long long *>(ws->nuniq.get<int64_t>(1));
  MSLM_HIP(hipMemsetAsync(ct, 0, sizeof(unsigned long long), st));
  k_coupling_total<<<nblk(n), kBS, 0, st>>>(rp, col, wv, n, N, ct);
  std::vector<int64_t> h(2 * T);
  int hf[2] = {0, 0};
  unsigned long long hct = 0;
  d2h(h.data(), twom, 2 * T, st);
  d2h(hf, flags, 2, st);
  d2h(&hct, ct, 1, st);
  MSLM_HIP(hipStreamSynchronize(st));
  g.ctot = (int64_t)hct;
  g.twom.assign(h.begin(), h.begin() + T);
  g.nzslice.assign(h.begin() + T, h.end());
  for (int s = 0; s < T; s++)
    if (g.twom[s] >= (int64_t)1 << 31)
      throw Error(MSLM_EOVERFLOW, "a slice's total degree 2m_s reaches 2^31");
  g.unit = hf[0] == 0;
  g.maxdeg = hf[1];
}

namespace {
__global__ void k_iota_i64_ranges(int64_t *p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}
__global__ void k_union_rows(const int64_t *rp, int64_t n, int64_t eoff, int64_t *out, int) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n) out[i] = rp[i] + eoff;
}
__global__ void k_union_cols(const int32_t *col, int64_t m, int32_t u0, int32_t *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = col[i] + u0;
}
__global__ void k_unit_ids(int32_t *uslice, int32_t *usolve, int64_t n, int32_t N, int32_t sfirst,
                           int32_t j) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uslice[i] = sfirst + (int32_t)(i / N);
  usolve[i] = j;
}
}  // namespace

#include "engine_solve.inc"

}  // namespace mslm
