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
//                digit in LDS; per-digit prefixes over the waves then place every key.
// Within a wave the LDS read of a digit's running count and the group leader's write of the
// new count are issued in program order, so every lane of the group sees the count before it.
//
// Reduce-by-key: head flags, a scan of them (segment index of every item), then each thread
// sums the runs of its eight consecutive items: runs that start inside its range are stored
// whole (the thread owns their head), the run it continues from the previous thread is kept
// aside and added to its segment with an atomic in a second launch, after every owner's store.
// Integer sums, so the result does not depend on the order of the additions.
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
  __shared__ int64_t gofs[kDigits];            // first output position of each digit
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = 0; i < kWaves; i++) wcnt[i][threadIdx.x] = 0;
  gofs[threadIdx.x] = offs[(int64_t)threadIdx.x * nb + blockIdx.x];
  __syncthreads();
  // wave w walks keys [base + w*512, base + (w+1)*512) in rounds of 64
  const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)w * 64 * kSortItems;
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
  // per digit, the keys of earlier waves come first
  uint32_t pre[kWaves];
  {
    uint32_t run = 0;
    for (int i = 0; i < kWaves; i++) {
      pre[i] = run;
      run += wcnt[i][threadIdx.x];
    }
  }
  __syncthreads();
  for (int i = 0; i < kWaves; i++) wcnt[i][threadIdx.x] = pre[i];
  __syncthreads();
  for (int r = 0; r < kSortItems; r++) {
    const int64_t j = base + (int64_t)r * 64 + lane;
    if (j >= n) continue;
    const int64_t pos = gofs[dg[r]] + wcnt[w][dg[r]] + rk[r];
    kout[pos] = kk[r];
    vout[pos] = vv[r];
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
template <class K>
__global__ __launch_bounds__(kThreads) void k_rbk_heads(const K *keys, int64_t n, uint8_t *head) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

template <class K, class V>
__global__ __launch_bounds__(kThreads) void k_rbk_sum(const K *keys, const V *vals,
                                                      const uint8_t *head, const int64_t *seg,
                                                      int64_t n, K *kout, V *vout,
                                                      int64_t *cseg, V *cval) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t lo = t * kSortItems;
  if (lo >= n) return;
  const int64_t hi = std::min<int64_t>(lo + kSortItems, n);
  cseg[t] = -1;
  int64_t i = lo;
  if (!head[lo]) {   // the run continued from the previous thread: added after the stores
    V s = 0;
    while (i < hi && !head[i]) s += vals[i++];
    cseg[t] = seg[lo] - 1;   // seg counts the heads before lo, its run's head included
    cval[t] = s;
  }
  while (i < hi) {   // runs whose head this thread holds
    const int64_t sg = seg[i];
    const K k = keys[i];
    V s = vals[i++];
    while (i < hi && !head[i]) s += vals[i++];
    kout[sg] = k;
    vout[sg] = s;
  }
}

template <class V>
__global__ __launch_bounds__(kThreads) void k_rbk_carry(const int64_t *cseg, const V *cval,
                                                        int64_t nt, V *vout);

template <>
__global__ __launch_bounds__(kThreads) void k_rbk_carry<int64_t>(const int64_t *cseg,
                                                                 const int64_t *cval, int64_t nt,
                                                                 int64_t *vout) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t < nt && cseg[t] >= 0)
    atomicAdd(reinterpret_cast<unsigned long long *>(vout + cseg[t]),
              (unsigned long long)cval[t]);
}

template <>
__global__ __launch_bounds__(kThreads) void k_rbk_carry<int32_t>(const int64_t *cseg,
                                                                 const int32_t *cval, int64_t nt,
                                                                 int32_t *vout) {
  const int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (t < nt && cseg[t] >= 0) atomicAdd(vout + cseg[t], cval[t]);
}

__global__ void k_rbk_count(const uint8_t *head, const int64_t *seg, int64_t n, int64_t *nout) {
  *nout = seg[n - 1] + head[n - 1];
}

template <class K, class V>
hipError_t reduce_by_key(const K *kin, K *kout, const V *vin, V *vout, int64_t *nout, int64_t n,
                         hipStream_t st, TempAlloc ta) {
  if (n <= 0) return hipMemsetAsync(nout, 0, sizeof(int64_t), st);
  const int64_t nt = (n + kSortItems - 1) / kSortItems;
  const size_t bytes = Carve::need({(size_t)n, sizeof(int64_t) * (size_t)n,
                                    sizeof(int64_t) * (size_t)nt, sizeof(V) * (size_t)nt}) +
                       scan_temp<uint8_t>(n);
  void *p = ta.get(ta.ctx, bytes);
  if (!p) return hipErrorOutOfMemory;
  Carve c{static_cast<char *>(p)};
  uint8_t *head = c.take<uint8_t>(n);
  int64_t *seg = c.take<int64_t>(n);
  int64_t *cseg = c.take<int64_t>(nt);
  V *cval = c.take<V>(nt);
  k_rbk_heads<K><<<grid_for(n, kThreads), kThreads, 0, st>>>(kin, n, head);
  hipError_t e = scan_run<uint8_t>(head, seg, n, st, c);
  if (e != hipSuccess) return e;
  k_rbk_sum<K, V><<<grid_for(nt, kThreads), kThreads, 0, st>>>(kin, vin, head, seg, n, kout, vout,
                                                              cseg, cval);
  k_rbk_carry<V><<<grid_for(nt, kThreads), kThreads, 0, st>>>(cseg, cval, nt, vout);
  k_rbk_count<<<1, 1, 0, st>>>(head, seg, n, nout);
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
