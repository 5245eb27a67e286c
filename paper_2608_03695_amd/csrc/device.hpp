// Device building blocks of the multislice Leiden path for gfx950 (CDNA4, wave64).
//
//  * priority hash (SplitMix64 output function, Steele-Lea-Flood 2014) for colouring and
//    refinement eligibility;
//  * the slice-partitioned community-degree table Sigma[(C, s)] (Eq. 6's per-slice null
//    model needs the total slice-s degree of every community): one open-addressing
//    sub-table per slice so that a colour batch, processed in slice-major order, touches
//    one slice's sub-table at a time (it stays resident in L2 / Infinity Cache);
//  * per-wave LDS accumulation tables for neighbour-community weights;
//  * exact comparison of multi-slice gains: a double filter with a rigorous error bound,
//    then fixed-width two's-complement big integers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mslm {

constexpr uint32_t kNone = 0xffffffffu;   // "no label" / the empty-community sentinel
constexpr int kMaxSlices = 64;

// ------------------------------------------------------------------ hashing

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

// seedmix = mix64(seed); key packs the solve-local unit id, phase, level and iteration.
__host__ __device__ inline uint64_t priority(uint64_t seedmix, int it, int lvl, int phase,
                                            uint32_t local) {
  uint64_t key = (uint64_t)local | ((uint64_t)phase << 32) | ((uint64_t)lvl << 40) |
                 ((uint64_t)it << 48);
  return mix64(key ^ seedmix);
}

// (h_u, u) > (h_v, v) lexicographically
__device__ inline bool outranks(uint64_t hu, uint32_t u, uint64_t hv, uint32_t v) {
  return hu > hv || (hu == hv && u > v);
}

__host__ __device__ inline uint32_t fib_hash(uint32_t x, int shift) {
  return (uint32_t)((x * 2654435769u) >> shift);
}

// ------------------------------------------------------------------ wave helpers

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ inline int64_t shfl_xor64(int64_t v, int m) { return __shfl_xor(v, m, 64); }
__device__ inline uint32_t shfl_xor32(uint32_t v, int m) { return (uint32_t)__shfl_xor((int)v, m, 64); }

__device__ inline int64_t wave_sum64(int64_t v) {
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor64(v, m);
  return v;
}

// Keyed counters with one atomic per distinct key present in the wave.  Every lane of the
// wave must call these together (no lane may have left the kernel).
__device__ inline void wave_count(uint32_t *ctr, int key, bool inc) {
  const int lane = threadIdx.x & 63;
  uint64_t m = __ballot(inc);
  while (m) {
    int leader = __builtin_ctzll(m);
    int k = __shfl(key, leader, 64);
    uint64_t same = __ballot(inc && key == k);
    if (lane == leader) atomicAdd(ctr + k, (uint32_t)__popcll(same));
    m &= ~same;
  }
}
__device__ inline void wave_add64(int64_t *ctr, int key, int64_t val) {
  const int lane = threadIdx.x & 63;
  uint64_t m = __ballot(val != 0);
  while (m) {
    int leader = __builtin_ctzll(m);
    int k = __shfl(key, leader, 64);
    bool mine = val != 0 && key == k;
    int64_t v = wave_sum64(mine ? val : 0);
    if (lane == leader) atomicAdd(reinterpret_cast<unsigned long long *>(ctr + k), (unsigned long long)v);
    m &= ~__ballot(mine);
  }
}

// Append val to out[] for every lane with flag set: one atomic per wave (convergent code).
__device__ inline void wave_append(int32_t *out, uint32_t *ctr, bool flag, int32_t val) {
  const int lane = threadIdx.x & 63;
  uint64_t bal = __ballot(flag);
  if (!bal) return;
  const int leader = __builtin_ctzll(bal);
  uint32_t base = 0;
  if (lane == leader) base = atomicAdd(ctr, (uint32_t)__popcll(bal));
  base = (uint32_t)__shfl((int)base, leader, 64);
  if (flag) out[base + __popcll(bal & ((1ull << lane) - 1))] = val;
}

// Appends gathered in a wave-private LDS buffer and written out in chunks: one global atomic
// per chunk instead of one per call (a frontier counter is shared by the whole grid, and
// atomics on one word serialise).  n is the same on every lane of the wave.
constexpr int kStage = 512;
struct WaveStage {
  int32_t *buf;     // LDS, kStage entries, private to the wave
  int32_t *out;     // global list
  uint32_t *ctr;    // its length
  uint32_t n;       // entries held
  __device__ void flush() {
    if (n == 0) return;
    wave_sync();
    const int lane = threadIdx.x & 63;
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(ctr, n);
    base = (uint32_t)__shfl((int)base, 0, 64);
    for (uint32_t i = lane; i < n; i += 64) out[base + i] = buf[i];
    wave_sync();
    n = 0;
  }
  // every lane of the wave must call this
  __device__ void append(bool flag, int32_t val) {
    const uint64_t bal = __ballot(flag);
    if (!bal) return;
    const int lane = threadIdx.x & 63;
    if (flag) buf[n + __popcll(bal & ((1ull << lane) - 1))] = val;
    n += (uint32_t)__popcll(bal);
    if (n > kStage - 64) flush();
  }
};

// Appends of a whole block written with one global atomic: every thread of the block calls
// this (s holds blockDim.x / 64 + 1 words of LDS).
__device__ inline void block_append(int32_t *out, uint32_t *ctr, bool flag, int32_t val,
                                    uint32_t *s) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint64_t bal = __ballot(flag);
  if (lane == 0) s[wv] = (uint32_t)__popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int w = 0; w < nw; w++) {
      const uint32_t c = s[w];
      s[w] = tot;
      tot += c;
    }
    s[nw] = tot ? atomicAdd(ctr, tot) : 0u;
  }
  __syncthreads();
  if (flag) out[s[nw] + s[wv] + __popcll(bal & ((1ull << lane) - 1))] = val;
  __syncthreads();
}

// ------------------------------------------------------------------ Sigma table
// Slot layout: 64-bit word, low half = key (label + 1, 0 = empty), high half = value.
// Values are slice degrees (< 2^31 by the create-time precondition).

struct SliceTable {
  uint64_t *slots;
  const int64_t *base;     // [slices] first slot of the slice's sub-table
  const int32_t *shift;    // [slices] 32 - log2(capacity)
  uint32_t *used;          // [slices] keys claimed (for the rebuild rule)
};

__device__ inline int32_t tab_get(const SliceTable &t, int s, uint32_t label) {
  const int sh = t.shift[s];
  const uint32_t mask = 0xffffffffu >> sh;
  const uint64_t *sub = t.slots + t.base[s];
  const uint32_t key = label + 1;
  uint32_t h = fib_hash(label, sh);
  for (;;) {
    uint64_t e = sub[h];
    uint32_t k = (uint32_t)e;
    if (k == key) return (int32_t)(e >> 32);
    if (k == 0) return 0;
    h = (h + 1) & mask;
  }
}

// count_new: bump the slice's key counter when a new key is claimed (only the sweeps need
// it, for the rebuild rule; full builds set the counters from known bounds instead)
__device__ inline void tab_add(const SliceTable &t, int s, uint32_t label, int32_t delta,
                               bool count_new = true) {
  const int sh = t.shift[s];
  const uint32_t mask = 0xffffffffu >> sh;
  uint64_t *sub = t.slots + t.base[s];
  const uint32_t key = label + 1;
  uint32_t h = fib_hash(label, sh);
  for (;;) {
    uint32_t *kp = reinterpret_cast<uint32_t *>(sub + h);
    uint32_t k = __hip_atomic_load(kp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (k == 0) {
      uint32_t prev = atomicCAS(kp, 0u, key);
      if (prev == 0) {
        if (count_new) atomicAdd(t.used + s, 1u);
        k = key;
      } else {
        k = prev;
      }
    }
    if (k == key) {
      atomicAdd(reinterpret_cast<int32_t *>(kp) + 1, delta);
      return;
    }
    h = (h + 1) & mask;
  }
}

// ------------------------------------------------------------------ LDS accumulation
// Open addressing over a power-of-two table in LDS; keys are label + 1.

__device__ inline void lds_add(uint32_t *K, int64_t *V, int lg, uint32_t label, int64_t w) {
  const uint32_t key = label + 1, mask = (1u << lg) - 1;
  uint32_t h = fib_hash(label, 32 - lg);
  for (;;) {
    uint32_t prev = atomicCAS(&K[h], 0u, key);
    if (prev == 0 || prev == key) {
      atomicAdd(reinterpret_cast<unsigned long long *>(&V[h]), (unsigned long long)w);
      return;
    }
    h = (h + 1) & mask;
  }
}

// As lds_add; the first insertion of a key also appends its slot to the list L (length *n),
// so that scans visit the occupied slots only.
__device__ inline void lds_add_listed(uint32_t *K, int64_t *V, int lg, uint32_t label, int64_t w,
                                      uint16_t *L, int *n) {
  const uint32_t key = label + 1, mask = (1u << lg) - 1;
  uint32_t h = fib_hash(label, 32 - lg);
  for (;;) {
    uint32_t prev = atomicCAS(&K[h], 0u, key);
    if (prev == 0 || prev == key) {
      if (prev == 0) L[atomicAdd(n, 1)] = (uint16_t)h;
      atomicAdd(reinterpret_cast<unsigned long long *>(&V[h]), (unsigned long long)w);
      return;
    }
    h = (h + 1) & mask;
  }
}

__device__ inline int64_t lds_get(const uint32_t *K, const int64_t *V, int lg, uint32_t label) {
  const uint32_t key = label + 1, mask = (1u << lg) - 1;
  uint32_t h = fib_hash(label, 32 - lg);
  for (;;) {
    uint32_t k = K[h];
    if (k == key) return V[h];
    if (k == 0) return 0;
    h = (h + 1) & mask;
  }
}

// global-memory version for units whose neighbourhood exceeds the LDS table
__device__ inline void gtab_add(uint32_t *K, int64_t *V, uint32_t mask, int shift, uint32_t label,
                                int64_t w) {
  const uint32_t key = label + 1;
  uint32_t h = fib_hash(label, shift);
  for (;;) {
    uint32_t prev = atomicCAS(&K[h], 0u, key);
    if (prev == 0 || prev == key) {
      atomicAdd(reinterpret_cast<unsigned long long *>(&V[h]), (unsigned long long)w);
      return;
    }
    h = (h + 1) & mask;
  }
}

__device__ inline int64_t gtab_get(const uint32_t *K, const int64_t *V, uint32_t mask, int shift,
                                   uint32_t label) {
  const uint32_t key = label + 1;
  uint32_t h = fib_hash(label, shift);
  for (;;) {
    uint32_t k = K[h];
    if (k == key) return V[h];
    if (k == 0) return 0;
    h = (h + 1) & mask;
  }
}

// ------------------------------------------------------------------ solve coefficients
// gamma = p/q, omega = a/b reduced; scaled weights: intra b*w, coupling a.
// Gains are ordered through   q*W - p*b * sum_s k_s * y_s / S_s   (S_s = 2m_s or 1).
struct Coef {
  int64_t p, q, a, b, pb;
  const int64_t *S;        // [slices] device
};

// ------------------------------------------------------------------ exact comparison
// Fixed-width two's-complement integers of kLimbs 32-bit limbs (2304 bits): enough for
// q*W*prod(S) with 64 slice denominators below 2^31 plus the summed null terms.
constexpr int kLimbs = 72;

struct Big {
  uint32_t d[kLimbs];
};

__device__ inline void big_set(Big &x, int64_t v) {
  uint32_t ext = v < 0 ? 0xffffffffu : 0u;
  x.d[0] = (uint32_t)v;
  x.d[1] = (uint32_t)((uint64_t)v >> 32);
  for (int i = 2; i < kLimbs; i++) x.d[i] = ext;
}
__device__ inline void big_mul_u32(Big &x, uint32_t m) {
  uint64_t c = 0;
  for (int i = 0; i < kLimbs; i++) {
    uint64_t t = (uint64_t)x.d[i] * m + c;
    x.d[i] = (uint32_t)t;
    c = t >> 32;
  }
}
// x += y * m  (or x -= y * m when neg), m < 2^32, y read as kLimbs - shift unsigned limbs
// placed shift limbs up; in place, modulo 2^2304
__device__ inline void big_addmul_u32(Big &x, const Big &y, uint32_t m, int shift, bool neg) {
  uint64_t pc = 0;   // carry of the product stream
  int64_t ac = 0;    // carry or borrow of the sum, -1..1
  for (int i = shift; i < kLimbs; i++) {
    const uint64_t p = (uint64_t)y.d[i - shift] * m + pc;
    pc = p >> 32;
    const int64_t pl = (int64_t)(uint32_t)p;
    const int64_t t = (int64_t)x.d[i] + (neg ? -pl : pl) + ac;
    x.d[i] = (uint32_t)t;
    ac = t >> 32;
  }
}

// Streaming evaluator of  q*Wd*Pi - pb*sum_j c_j/S_j * Pi  where Pi is the product of the
// denominators of the terms fed in (terms with c_j == 0 are skipped entirely).  Only the
// running numerator and Pi are stored; every update works in place, limb by limb.
struct ExactAcc {
  Big num, den;
  __device__ void init() {
    big_set(num, 0);
    big_set(den, 1);
  }
  // S in [1, 2^31) (a slice's 2m, or 1 for an empty slice)
  __device__ void term(int64_t c, int64_t S) {
    if (c == 0) return;
    // num/den + c/S = (num*S + c*den) / (den*S)
    big_mul_u32(num, (uint32_t)S);
    const bool neg = c < 0;
    const uint64_t a = neg ? (uint64_t)0 - (uint64_t)c : (uint64_t)c;
    big_addmul_u32(num, den, (uint32_t)a, 0, neg);
    if (a >> 32) big_addmul_u32(num, den, (uint32_t)(a >> 32), 1, neg);
    big_mul_u32(den, (uint32_t)S);
  }
  // sign of q*Wd*den - pb*num, produced limb by limb with a 128-bit carry (|q*Wd| < 2^95,
  // 0 <= pb < 2^64): the low 2304 bits of the exact value, whose top bit is its sign
  __device__ int sign(int64_t q, int64_t Wd, int64_t pb) {
    const __int128 a = (__int128)q * Wd;
    const bool aneg = a < 0;
    const unsigned __int128 ua = aneg ? (unsigned __int128)0 - (unsigned __int128)a
                                      : (unsigned __int128)a;
    const uint64_t A0 = (uint32_t)ua, A1 = (uint32_t)(ua >> 32), A2 = (uint32_t)(ua >> 64);
    const uint64_t B0 = (uint32_t)(uint64_t)pb, B1 = (uint32_t)((uint64_t)pb >> 32);
    __int128 acc = 0;
    uint32_t any = 0, top = 0;
    for (int i = 0; i < kLimbs; i++) {
      __int128 sa = (__int128)(den.d[i] * A0);
      __int128 sb = (__int128)(num.d[i] * B0);
      if (i >= 1) {
        sa += (__int128)(den.d[i - 1] * A1);
        sb += (__int128)(num.d[i - 1] * B1);
      }
      if (i >= 2) sa += (__int128)(den.d[i - 2] * A2);
      acc += (aneg ? -sa : sa) - sb;
      top = (uint32_t)acc;
      any |= top;
      acc >>= 32;
    }
    return (top >> 31) ? -1 : (any ? 1 : 0);
  }
};

// Double-precision estimate of  q*W - pb * sum_j c_j / S_j  with a rigorous bound on its
// error: every int64 -> double conversion, division, product and addition contributes at
// most one half-ulp, so (m + 8) * 2^-50 * (|q*W| + pb * sum |c_j| / S_j) is a safe cover.
struct Approx {
  double val, err;
};

}  // namespace mslm
