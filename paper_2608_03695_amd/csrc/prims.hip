// Device-wide primitives written for gfx950: exclusive scan, stable LSD radix sort of
// key/value pairs, and reduce-by-key over sorted keys.
//
// Scan: every block reduces a tile, one block scans the tile sums, every block rescans its
// tile with its offset (read twice, written once).
//
// Radix sort: 8-bit digits over the bits in use, one pass per digit, each pass three launches:
//   histogram  - a block counts the digits of its tile in LDS and writes them digit-major
//                (count[d * B + b]), so one exclusive scan of that array gives every (digit,
//                block) its first output position;
//   scan       - the device scan above;
//   scatter    - a block ranks its keys stably: each wave walks its contiguous part of the
//                tile 64 keys at a time, finds the lanes holding the same digit with eight
//                ballots (one per digit bit), takes its rank among them from the popcount of
//                the lower lanes and adds the group's size to the wave's running count of that
//                digit in LDS; per-digit prefixes over the waves and over the digits place
//                every key in an LDS copy of the tile sorted by digit, from which consecutive
//                threads write each digit's run to consecutive output positions.
// Within a wave the LDS read of a digit's running count and the group leader's write of the
// new count are issued in program order, so every lane of the group sees the count before it.
//
// Reduce-by-key: a segmented scan.  Every item is summarised by (is it a segment head, its
// value); pairs (heads, sum since the last head) combine associatively, so one scan gives
// every item its segment's index and running sum, and the last item of each segment writes
// the segment out.  Three launches (tile pairs, one block scanning them, tiles rescanned and
// written); no atomics, integer sums in the items' order.
#include "prims.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace mslm {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kScanItems = 8;                       // scan tile: 2048 items
constexpr int64_t kScanTile = (int64_t)kThreads * kScanItems;
constexpr int kSortItems = 8;                       // radix tile: 2048 keys
constexpr int64_t kSortTile = (int64_t)kThreads * kSortItems;
constexpr int kDigitBits = 8;
constexpr int kDigits = 1 << kDigitBits;
constexpr int kMaxBlockSums = 1 << 20;              // tile sums scanned by one block: 2^31 items
static_assert(kThreads == kDigits, "the scatter kernel gives each thread one digit");

// ------------------------------------------------------------------ small helpers
struct Carve {   // sub-allocates one temp-storage request
  char *p;
  size_t used = 0;
  template <class T>
  T *take(int64_t n) {
    used = (used + 255) & ~(size_t)255;
    T *r = reinterpret_cast<T *>(p + used);
    used += sizeof(T) * (size_t)std::max<int64_t>(n, 1);
    return r;
  }
  static size_t need(std::initializer_list<size_t> parts) {
    size_t s = 0;
    for (size_t x : parts) s = ((s + 255) & ~(size_t)255) + std::max<size_t>(x, 1);
    return s + 256;
  }
};

inline unsigned grid_for(int64_t n, int64_t tile) {
  return (unsigned)std::max<int64_t>(1, (n + tile - 1) / tile);
}

__device__ inline int64_t wave_incl_sum(int64_t x) {
  const int lane = threadIdx.x & 63;
  for (int o = 1; o < 64; o <<= 1) {
    int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Exclusive prefix of x over the block (all threads call it); total in *tot.
__device__ inline int64_t block_excl_sum(int64_t x, int64_t *sh, int64_t *tot) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t inc = wave_incl_sum(x);
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  int64_t before = 0, all = 0;
  for (int i = 0; i < kWaves; i++) {
    if (i < w) before += sh[i];
    all += sh[i];
  }
  __syncthreads();
  if (tot) *tot = all;
  return before + inc - x;
}

// ------------------------------------------------------------------ scan
template <class T>
__global__ __launch_bounds__(kThreads) void k_scan_tiles(const T *in, int64_t n, int64_t *sums) {
  __shared__ int64_t sh[kWaves];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t s = 0;
  for (int i = 0; i < kScanItems; i++)
    if (base + i < n) s += (int64_t)in[base + i];
  int64_t tot = 0;
  block_excl_sum(s, sh, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// One block: exclusive scan of the tile sums in place (nb <= kMaxBlockSums).
__global__ __launch_bounds__(1024) void k_scan_sums(int64_t *sums, int64_t nb) {
  __shared__ int64_t sh[16];
  const int per = (int)((nb + 1023) / 1024);
  const int64_t lo = (int64_t)threadIdx.x * per;
  int64_t s = 0;
  for (int64_t i = lo; i < lo + per && i < nb; i++) s += sums[i];
  // block-wide exclusive prefix (1024 threads = 16 waves)
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t inc = wave_incl_sum(s);
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  int64_t before = 0;
  for (int i = 0; i < w; i++) before += sh[i];
  int64_t run = before + inc - s;
  for (int64_t i = lo; i < lo + per && i < nb; i++) {
    const int64_t x = sums[i];
    sums[i] = run;
    run += x;
  }
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_scan_apply(const T *in, int64_t *out, int64_t n,
                                                         const int64_t *sums) {
  __shared__ int64_t sh[kWaves];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t s = 0;
  for (int i = 0; i < kScanItems; i++) {
    v[i] = base + i < n ? (int64_t)in[base + i] : 0;
    s += v[i];
  }
  int64_t run = sums[blockIdx.x] + block_excl_sum(s, sh, nullptr);
  for (int i = 0; i < kScanItems; i++) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
}

template <class T>
size_t scan_temp(int64_t n) {
  return Carve::need({sizeof(int64_t) * (size_t)grid_for(n, kScanTile)});
}

// out[i] = sum of in[0..i-1]; `tmp` holds the tile sums.
template <class T>
hipError_t scan_run(const T *in, int64_t *out, int64_t n, hipStream_t st, Carve &tmp) {
  if (n <= 0) return hipSuccess;
  const unsigned nb = grid_for(n, kScanTile);
  if (nb > kMaxBlockSums) return hipErrorInvalidValue;
  int64_t *sums = tmp.take<int64_t>(nb);
  k_scan_tiles<T><<<nb, kThreads, 0, st>>>(in, n, sums);
  k_scan_sums<<<1, 1024, 0, st>>>(sums, nb);
  k_scan_apply<T><<<nb, kThreads, 0, st>>>(in, out, n, sums);
  return hipGetLastError();
}

template <class T>
hipError_t exclusive_sum(const T *in, int64_t *out, int64_t n, hipStream_t st, TempAlloc ta) {
  if (n <= 0) return hipSuccess;
  void *p = ta.get(ta.ctx, scan_temp<T>(n));
  if (!p) return hipErrorOutOfMemory;
  Carve c{static_cast<char *>(p)};
  return scan_run<T>(in, out, n, st, c);
}

// ------------------------------------------------------------------ radix sort
template <class K>
__device__ inline uint32_t digit_of(K k, int bit) {
  return (uint32_t)(k >> bit) & (kDigits - 1);
}

template <class K>
__global__ __launch_bounds__(kThreads) void k_rs_hist(const K *keys, int64_t n, int bit,
                                                      int64_t *count, int64_t nb) {
  __shared__ uint32_t h[kDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int i = 0; i < kSortItems; i++) {
    const int64_t j = base + (int64_t)i * kThreads + threadIdx.x;
    if (j < n) atomicAdd(&h[digit_of(keys[j], bit)], 1u);
  }
  __syncthreads();
  count[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

template <class K, class V>
__global__ __launch_bounds__(kThreads) void k_rs_scatter(const K *kin, const V *vin, K *kout,
                                                         V *vout, int64_t n, int bit,
                                                         const int64_t *offs, int64_t nb) {
  __shared__ uint32_t wcnt[kWaves][kDigits];   // running count per wave and digit
  __shared__ uint32_t tstart[kDigits];         // first slot of each digit in the sorted tile
  __shared__ int64_t gofs[kDigits];            // first output position of each digit
  __shared__ K sk[kSortTile];                  // the tile, sorted by digit
  __shared__ V sv[kSortTile];
  __shared__ int64_t shc[kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = 0; i < kWaves; i++) wcnt[i][threadIdx.x] = 0;
  gofs[threadIdx.x] = offs[(int64_t)threadIdx.x * nb + blockIdx.x];
  __syncthreads();
  // wave w walks keys [base + w*512, base + (w+1)*512) in rounds of 64
  const int64_t tile = (int64_t)blockIdx.x * kSortTile;
  const int64_t base = tile + (int64_t)w * 64 * kSortItems;
  const uint64_t below = (1ull << lane) - 1;
  K kk[kSortItems];
  V vv[kSortItems];
  uint32_t dg[kSortItems], rk[kSortItems];
  for (int r = 0; r < kSortItems; r++) {
    const int64_t j = base + (int64_t)r * 64 + lane;
    const bool live = j < n;
    kk[r] = live ? kin[j] : K(0);
    vv[r] = live ? vin[j] : V(0);
    const uint32_t d = digit_of(kk[r], bit);
    dg[r] = d;
    uint64_t peers = __ballot(live);
    for (int b = 0; b < kDigitBits; b++) {
      const uint64_t ones = __ballot(live && ((d >> b) & 1u));
      peers &= ((d >> b) & 1u) ? ones : ~ones;
    }
    const uint32_t before = wcnt[w][d];            // every lane of the group reads first
    rk[r] = before + (uint32_t)__popcll(peers & below);
    if (live && (peers & below) == 0) wcnt[w][d] = before + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // per digit: keys of earlier waves first; digits in order inside the tile
  uint32_t pre[kWaves];
  uint32_t cnt = 0;
  for (int i = 0; i < kWaves; i++) {
    pre[i] = cnt;
    cnt += wcnt[i][threadIdx.x];
  }
  int64_t tot = 0;
  const uint32_t start = (uint32_t)block_excl_sum((int64_t)cnt, shc, &tot);
  tstart[threadIdx.x] = start;
  for (int i = 0; i < kWaves; i++) wcnt[i][threadIdx.x] = start + pre[i];
  __syncthreads();
  for (int r = 0; r < kSortItems; r++) {
    const int64_t j = base + (int64_t)r * 64 + lane;
    if (j >= n) continue;
    const uint32_t slot = wcnt[w][dg[r]] + rk[r];
    sk[slot] = kk[r];
    sv[slot] = vv[r];
  }
  __syncthreads();
  // consecutive threads write consecutive positions inside each digit's run
  const int live = (int)(n - tile < kSortTile ? n - tile : kSortTile);
  for (int s = threadIdx.x; s < live; s += kThreads) {
    const uint32_t d = digit_of(sk[s], bit);
    const int64_t pos = gofs[d] + (s - (int64_t)tstart[d]);
    kout[pos] = sk[s];
    vout[pos] = sv[s];
  }
}

template <class K, class V>
hipError_t radix_sort(const K *kin, K *kout, const V *vin, V *vout, int64_t n, int end_bit,
                      hipStream_t st, TempAlloc ta) {
  if (n <= 0) return hipSuccess;
  end_bit = std::max(0, std::min<int>(end_bit, (int)(8 * sizeof(K))));
  const int passes = (end_bit + kDigitBits - 1) / kDigitBits;
  if (passes == 0) {
    hipError_t e = hipMemcpyAsync(kout, kin, sizeof(K) * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(vout, vin, sizeof(V) * n, hipMemcpyDeviceToDevice, st);
  }
  const int64_t nb = grid_for(n, kSortTile);
  const int64_t nc = nb * kDigits;
  const size_t bytes = Carve::need({sizeof(int64_t) * (size_t)nc, sizeof(int64_t) * (size_t)nc,
                                    passes > 1 ? sizeof(K) * (size_t)n : 1,
                                    passes > 1 ? sizeof(V) * (size_t)n : 1}) +
                       scan_temp<int64_t>(nc);
  void *p = ta.get(ta.ctx, bytes);
  if (!p) return hipErrorOutOfMemory;
  Carve c{static_cast<char *>(p)};
  int64_t *count = c.take<int64_t>(nc);
  int64_t *offs = c.take<int64_t>(nc);
  K *tk = passes > 1 ? c.take<K>(n) : nullptr;
  V *tv = passes > 1 ? c.take<V>(n) : nullptr;
  const K *sk = kin;
  const V *sv = vin;
  for (int ps = 0; ps < passes; ps++) {
    // the last pass lands in the output; earlier passes alternate so that it does
    const bool to_out = ((passes - 1 - ps) % 2) == 0;
    K *dk = to_out ? kout : tk;
    V *dv = to_out ? vout : tv;
    const int bit = ps * kDigitBits;
    k_rs_hist<K><<<(unsigned)nb, kThreads, 0, st>>>(sk, n, bit, count, nb);
    Carve cs = c;
    hipError_t e = scan_run<int64_t>(count, offs, nc, st, cs);
    if (e != hipSuccess) return e;
    k_rs_scatter<K, V><<<(unsigned)nb, kThreads, 0, st>>>(sk, sv, dk, dv, n, bit, offs, nb);
    sk = dk;
    sv = dv;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ reduce by key
// A pair (c, s) summarises a run of items: c heads among them, s the sum of the items after
// the last head (all of them when c == 0).  Pairs combine associatively:
//   (c1, s1) then (c2, s2) = (c1 + c2, c2 ? s2 : s1 + s2),
// so a scan of pairs gives every item the number of segments before it and the running sum
// of its segment.
template <class V>
struct SegPair {
  int64_t c;
  V s;
};

template <class V>
__device__ inline SegPair<V> seg_combine(const SegPair<V> &a, const SegPair<V> &b) {
  return SegPair<V>{a.c + b.c, b.c ? b.s : (V)(a.s + b.s)};
}

// exclusive scan of pairs over the block; the block's total in *tot
template <class V>
__device__ inline SegPair<V> block_excl_pairs(SegPair<V> x, int64_t *shc, V *shs,
                                              SegPair<V> *tot) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  SegPair<V> inc = x;
  for (int o = 1; o < 64; o <<= 1) {
    SegPair<V> y{__shfl_up(inc.c, o, 64), __shfl_up(inc.s, o, 64)};
    if (lane >= o) inc = seg_combine(y, inc);
  }
  if (lane == 63) {
    shc[w] = inc.c;
    shs[w] = inc.s;
  }
  __syncthreads();
  SegPair<V> before{0, 0}, all{0, 0};
  for (int i = 0; i < kWaves; i++) {
    const SegPair<V> p{shc[i], shs[i]};
    if (i < w) before = seg_combine(before, p);
    all = seg_combine(all, p);
  }
  __syncthreads();
  if (tot) *tot = all;
  // exclusive: everything before this lane
  SegPair<V> prev{__shfl_up(inc.c, 1, 64), __shfl_up(inc.s, 1, 64)};
  if (lane == 0) prev = SegPair<V>{0, 0};
  return seg_combine(before, prev);
}

// The block's tile of keys and values, loaded with coalesced reads into LDS; item i of the
// tile is sk[i]; prev/next are the keys just before and after the tile (or a copy of the
// first/last key when there is none, which never marks a head).
template <class K, class V>
struct RbkTile {
  K sk[kSortTile];
  V sv[kSortTile];
  K prev, next;
};

template <class K, class V>
__device__ inline int64_t load_tile(const K *keys, const V *vals, int64_t n, RbkTile<K, V> &t) {
  const int64_t tile = (int64_t)blockIdx.x * kSortTile;
  const int64_t len = n - tile < kSortTile ? n - tile : kSortTile;
  for (int64_t i = threadIdx.x; i < len; i += kThreads) {
    t.sk[i] = keys[tile + i];
    t.sv[i] = vals[tile + i];
  }
  if (threadIdx.x == 0) {
    t.prev = tile > 0 ? keys[tile - 1] : keys[0];
    t.next = tile + len < n ? keys[tile + len] : keys[tile + len - 1];
  }
  __syncthreads();
  return len;
}

template <class K, class V>
__device__ inline bool tile_head(const RbkTile<K, V> &t, int64_t i, int64_t tile) {
  const K before = i > 0 ? t.sk[i - 1] : t.prev;
  return (tile + i == 0) || t.sk[i] != before;
}

template <class K, class V>
__device__ inline SegPair<V> thread_pair(const RbkTile<K, V> &t, int64_t lo, int64_t hi,
                                         int64_t tile) {
  SegPair<V> p{0, 0};
  for (int64_t i = lo; i < hi; i++)
    p = seg_combine(p, SegPair<V>{tile_head(t, i, tile) ? 1 : 0, t.sv[i]});
  return p;
}

template <class K, class V>
__global__ __launch_bounds__(kThreads) void k_rbk_tiles(const K *keys, const V *vals, int64_t n,
                                                        int64_t *tc, V *ts) {
  __shared__ RbkTile<K, V> t;
  __shared__ int64_t shc[kWaves];
  __shared__ V shs[kWaves];
  const int64_t tile = (int64_t)blockIdx.x * kSortTile;
  const int64_t len = load_tile(keys, vals, n, t);
  const int64_t lo = (int64_t)threadIdx.x * kSortItems;
  const int64_t hi = lo + kSortItems < len ? lo + kSortItems : len;
  SegPair<V> tot;
  block_excl_pairs<V>(thread_pair(t, lo, hi, tile), shc, shs, &tot);
  if (threadIdx.x == 0) {
    tc[blockIdx.x] = tot.c;
    ts[blockIdx.x] = tot.s;
  }
}

// one block: exclusive scan of the tile pairs in place (nb <= kMaxBlockSums); the total
// count of segments into *nout
template <class V>
__global__ __launch_bounds__(1024) void k_rbk_scan_tiles(int64_t *tc, V *ts, int64_t nb,
                                                         int64_t *nout) {
  __shared__ int64_t shc[16];
  __shared__ V shs[16];
  const int per = (int)((nb + 1023) / 1024);
  const int64_t lo = (int64_t)threadIdx.x * per;
  SegPair<V> x{0, 0};
  for (int64_t i = lo; i < lo + per && i < nb; i++) x = seg_combine(x, SegPair<V>{tc[i], ts[i]});
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  SegPair<V> inc = x;
  for (int o = 1; o < 64; o <<= 1) {
    SegPair<V> y{__shfl_up(inc.c, o, 64), __shfl_up(inc.s, o, 64)};
    if (lane >= o) inc = seg_combine(y, inc);
  }
  if (lane == 63) {
    shc[w] = inc.c;
    shs[w] = inc.s;
  }
  __syncthreads();
  SegPair<V> run{0, 0};
  for (int i = 0; i < w; i++) run = seg_combine(run, SegPair<V>{shc[i], shs[i]});
  SegPair<V> prev{__shfl_up(inc.c, 1, 64), __shfl_up(inc.s, 1, 64)};
  if (lane == 0) prev = SegPair<V>{0, 0};
  run = seg_combine(run, prev);
  for (int64_t i = lo; i < lo + per && i < nb; i++) {
    const SegPair<V> t{tc[i], ts[i]};
    tc[i] = run.c;
    ts[i] = run.s;
    run = seg_combine(run, t);
  }
  if (threadIdx.x == 1023) *nout = run.c;
}

// every item knows the segments before it and its segment's running sum; the last item of a
// segment writes the segment's key and sum
template <class K, class V>
__global__ __launch_bounds__(kThreads) void k_rbk_emit(const K *keys, const V *vals, int64_t n,
                                                       const int64_t *tc, const V *ts, K *kout,
                                                       V *vout) {
  __shared__ RbkTile<K, V> t;
  __shared__ int64_t shc[kWaves];
  __shared__ V shs[kWaves];
  const int64_t tile = (int64_t)blockIdx.x * kSortTile;
  const int64_t len = load_tile(keys, vals, n, t);
  const int64_t lo = (int64_t)threadIdx.x * kSortItems;
  const int64_t hi = lo + kSortItems < len ? lo + kSortItems : len;
  SegPair<V> run = block_excl_pairs<V>(thread_pair(t, lo, hi, tile), shc, shs, nullptr);
  run = seg_combine(SegPair<V>{tc[blockIdx.x], ts[blockIdx.x]}, run);
  for (int64_t i = lo; i < hi; i++) {
    run = seg_combine(run, SegPair<V>{tile_head(t, i, tile) ? 1 : 0, t.sv[i]});
    const bool last = tile + i + 1 == n || (i + 1 < len ? t.sk[i + 1] : t.next) != t.sk[i];
    if (last) {
      kout[run.c - 1] = t.sk[i];
      vout[run.c - 1] = run.s;
    }
  }
}

template <class K, class V>
hipError_t reduce_by_key(const K *kin, K *kout, const V *vin, V *vout, int64_t *nout, int64_t n,
                         hipStream_t st, TempAlloc ta) {
  if (n <= 0) return hipMemsetAsync(nout, 0, sizeof(int64_t), st);
  const int64_t nb = grid_for(n, kSortTile);
  if (nb > kMaxBlockSums) return hipErrorInvalidValue;
  void *p = ta.get(ta.ctx, Carve::need({sizeof(int64_t) * (size_t)nb, sizeof(V) * (size_t)nb}));
  if (!p) return hipErrorOutOfMemory;
  Carve c{static_cast<char *>(p)};
  int64_t *tc = c.take<int64_t>(nb);
  V *ts = c.take<V>(nb);
  k_rbk_tiles<K, V><<<(unsigned)nb, kThreads, 0, st>>>(kin, vin, n, tc, ts);
  k_rbk_scan_tiles<V><<<1, 1024, 0, st>>>(tc, ts, nb, nout);
  k_rbk_emit<K, V><<<(unsigned)nb, kThreads, 0, st>>>(kin, vin, n, tc, ts, kout, vout);
  return hipGetLastError();
}

}  // namespace

hipError_t sort_pairs_u32_u32(const uint32_t *kin, uint32_t *kout, const uint32_t *vin,
                              uint32_t *vout, int64_t n, int end_bit, hipStream_t st,
                              TempAlloc ta) {
  return radix_sort<uint32_t, uint32_t>(kin, kout, vin, vout, n, end_bit, st, ta);
}

hipError_t sort_pairs_u64_i64(const uint64_t *kin, uint64_t *kout, const int64_t *vin,
                              int64_t *vout, int64_t n, int end_bit, hipStream_t st,
                              TempAlloc ta) {
  return radix_sort<uint64_t, int64_t>(kin, kout, vin, vout, n, end_bit, st, ta);
}

hipError_t sort_pairs_u64_i32(const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                              int32_t *vout, int64_t n, int end_bit, hipStream_t st,
                              TempAlloc ta) {
  return radix_sort<uint64_t, int32_t>(kin, kout, vin, vout, n, end_bit, st, ta);
}

hipError_t reduce_by_key_u64_i64(const uint64_t *kin, uint64_t *kout, const int64_t *vin,
                                 int64_t *vout, int64_t *nout, int64_t n, hipStream_t st,
                                 TempAlloc ta) {
  return reduce_by_key<uint64_t, int64_t>(kin, kout, vin, vout, nout, n, st, ta);
}

hipError_t reduce_by_key_u64_i32(const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                                 int32_t *vout, int64_t *nout, int64_t n, hipStream_t st,
                                 TempAlloc ta) {
  return reduce_by_key<uint64_t, int32_t>(kin, kout, vin, vout, nout, n, st, ta);
}

hipError_t exclusive_sum_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t st,
                             TempAlloc ta) {
  return exclusive_sum<int64_t>(in, out, n, st, ta);
}

hipError_t exclusive_sum_u8_i64(const uint8_t *in, int64_t *out, int64_t n, hipStream_t st,
                                TempAlloc ta) {
  return exclusive_sum<uint8_t>(in, out, n, st, ta);
}

hipError_t exclusive_sum_u32_i64(const uint32_t *in, int64_t *out, int64_t n, hipStream_t st,
                                 TempAlloc ta) {
  return exclusive_sum<uint32_t>(in, out, n, st, ta);
}

}  // namespace mslm
