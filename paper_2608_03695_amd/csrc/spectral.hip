// The Bethe-Hessian spectral pathway (Section 3.1, the paragraphs after Eq. 4) on a resident
// supra-graph: H(r) = (r^2 - 1) I - r A + D (A the supra-adjacency of Eq. 3, D its degrees),
// the k algebraically smallest eigenpairs by Lanczos with full reorthogonalisation, and
// k-means on the rows of the embedding.
//
// Kernels: the operator (16 lanes per row), block-partial dot products with a fixed grid (the
// same sums in the same order on every run), a multi-vector dot / update pair for the
// reorthogonalisation, a one-workgroup implicit-QR eigensolver for the small tridiagonal
// matrix (rotations found by one thread, applied by one thread per row), the Ritz vectors, and k-means
// (maximin start, Lloyd steps; distances rounded operation by operation, centroid sums exact in
// fixed point through integer atomics, so the labels do not depend on the order of the sums).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mslm.h"
#include "device.hpp"
#include "engine.hpp"
#include "handles.hpp"
#include "host.hpp"

namespace mslm {
namespace {

constexpr int kSB = 256;          // threads per block
constexpr int kDotBlocks = 512;   // fixed grid of the reductions
constexpr int kMdotBlocks = 1024; // row ranges of the reorthogonalisation dot products
constexpr int kMdotVec = 4;       // vectors per block (a timing sweep of 4/8/16)
constexpr int kMaxK = 32;         // eigenvectors / clusters
constexpr int kMaxSteps = 256;    // Krylov dimension
constexpr int kFixShift = 40;     // fixed-point scale of the k-means sums
constexpr int kSplit = 20;        // a fixed-point value as hi * 2^20 + lo, 0 <= lo < 2^20

inline unsigned blocks(int64_t n, int bs = kSB) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + bs - 1) / bs, 1 << 30));
}

struct SpecGraph {
  const int64_t *rp;
  const int32_t *col;
  const int32_t *w;   // raw weight (intra w, coupling c_sr) or nullptr: all 1
  int64_t n, N;
  double omega;
};

// weighted degree of every supra-node: intra weights plus omega * c_sr of the coupling entries
__global__ void k_bh_degree(SpecGraph g, double *d) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= g.n) return;
  const int64_t lo = (v / g.N) * g.N, hi = lo + g.N;
  double s = 0.0;
  for (int64_t e = g.rp[v]; e < g.rp[v + 1]; e++) {
    const int32_t x = g.col[e];
    const double raw = g.w ? (double)g.w[e] : 1.0;
    s += (x >= lo && x < hi) ? raw : g.omega * raw;
  }
  d[v] = s;
}

// y = H(r) x = (r^2 - 1 + d) x - r A x, 16 lanes per row
__global__ void k_bh_apply(SpecGraph g, const double *d, double r, const double *x, double *y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t v = t >> 4;
  const int sl = (int)(t & 15);
  double acc = 0.0;
  if (v < g.n) {
    const int64_t lo = (v / g.N) * g.N, hi = lo + g.N;
    for (int64_t e = g.rp[v] + sl; e < g.rp[v + 1]; e += 16) {
      const int32_t x_ = g.col[e];
      const double raw = g.w ? (double)g.w[e] : 1.0;
      acc += ((x_ >= lo && x_ < hi) ? raw : g.omega * raw) * x[x_];
    }
  }
  for (int m = 8; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
  if (v < g.n && sl == 0) y[v] = (r * r - 1.0 + d[v]) * x[v] - r * acc;
}

__device__ inline double block_sum(double v, double *sh) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[wv] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); i++) s += sh[i];
  __syncthreads();
  return s;
}

// partial[b] = sum over block b's grid-stride share of x*y (x == y for a squared norm);
// d2 optional: sum of d^2 into partial2[b]
__global__ void k_dot_partial(const double *x, const double *y, int64_t n, double *partial) {
  __shared__ double sh[kSB / 64];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    s += x[i] * y[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
// out[i] = sum over b of partial[b * cnt + i]: one block per i (the same order every run);
// gate as for k_mdot_partial
__global__ void k_sum_partials(const double *partial, int nb, int cnt, const int *gate,
                               double *out) {
  if (gate && *gate == 0) return;
  __shared__ double sh[kSB / 64];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) s += partial[(int64_t)b * cnt + i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[i] = s;
}

// sum of d and of d^2 (the default r)
__global__ void k_deg_moments(const double *d, int64_t n, double *partial) {
  __shared__ double sh[kSB / 64];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    s1 += d[i];
    s2 += d[i] * d[i];
  }
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s1;
    partial[2 * blockIdx.x + 1] = s2;
  }
}

// y = a*x + b*y
__global__ void k_axpby(double a, const double *x, double b, double *y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}
// y = a*x (y is not read: it may hold anything, even non-finite values)
__global__ void k_scale_into(double a, const double *x, double *y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// w -= alpha * v_j + beta * v_{j-1}
__global__ void k_lanczos_sub(double *w, const double *vj, const double *vp, double alpha,
                              double beta, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double t = w[i] - alpha * vj[i];
  if (vp) t -= beta * vp[i];
  w[i] = t;
}

// partial[b * stride + i] = block b's share of V_i . w for i < cnt and, with norm, of w . w at
// i = cnt (stride = cnt + norm; V column-major, n per vector).  Block (b, y) takes the
// contiguous row range b and the four vectors 4y..4y+3 (a grid of kMdotBlocks x
// ceil(stride / 4) blocks): many short blocks keep enough loads in flight.
__global__ __launch_bounds__(kSB) void k_mdot_partial(const double *V, int cnt, const double *w,
                                                     int64_t n, int norm, const int *gate,
                                                     double *partial) {
  if (gate && *gate == 0) return;
  __shared__ double sh[kMdotVec][kSB / 64];
  const int stride = cnt + norm;
  const int i0 = blockIdx.y * kMdotVec;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = std::min<int64_t>(n, lo + per);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double s[kMdotVec];
#pragma unroll
  for (int u = 0; u < kMdotVec; u++) s[u] = 0.0;
#pragma unroll 4
  for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
    const double wk = w[k];
#pragma unroll
    for (int u = 0; u < kMdotVec; u++) {
      const int i = i0 + u;
      if (i < cnt) s[u] += V[(int64_t)i * n + k] * wk;
      else if (i == cnt && norm) s[u] += wk * wk;
    }
  }
  // the block's sums: wave shuffles, then the four waves in index order
#pragma unroll
  for (int u = 0; u < kMdotVec; u++) {
    double v = s[u];
    for (int msk = 32; msk >= 1; msk >>= 1) v += __shfl_xor(v, msk, 64);
    if (lane == 0) sh[u][wv] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < kMdotVec && i0 + (int)threadIdx.x < stride) {
    double v = 0.0;
    for (int q = 0; q < kSB / 64; q++) v += sh[threadIdx.x][q];
    partial[(int64_t)blockIdx.x * stride + i0 + threadIdx.x] = v;
  }
}

// w -= V h (cnt vectors); gate as for k_mdot_partial
__global__ void k_msub(const double *V, int cnt, const double *h, const int *gate, double *w,
                       int64_t n) {
  if (gate && *gate == 0) return;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s = 0.0;
  for (int i = 0; i < cnt; i++) s += V[(int64_t)i * n + k] * h[i];
  w[k] -= s;
}

// The second reorthogonalisation pass is needed when the first removed more than half of
// w's squared norm (||w - V h|| < ||w|| / sqrt(2), Daniel, Gragg, Kaufman and Stewart 1976):
// flag = (sum h_i^2 > ||w||^2 / 2), from h[0..cnt) and ||w||^2 in h[cnt]; count[0] counts them
__global__ void k_reorth_gate(const double *h, int cnt, int *flag, int *count) {
  if (threadIdx.x != 0) return;
  double hh = 0.0;
  for (int i = 0; i < cnt; i++) hh += h[i] * h[i];
  const int f = hh > 0.5 * h[cnt];
  *flag = f;
  count[0] += f;
}

// deterministic start vector: SplitMix64 of (seed, i) as a uniform value in [-1, 1)
__global__ void k_start_vector(double *v, int64_t n, uint64_t seedmix) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t z = mix64(seedmix ^ (uint64_t)i);
  v[i] = (double)(z >> 11) * 0x1p-52 - 1.0;
}

// Eigen-decomposition of the symmetric tridiagonal matrix with diagonal a[0..m) and
// off-diagonal b[0..m-1) by implicit QR steps with the Wilkinson shift (Golub & Van Loan,
// Section 8.3).  Wave 0 finds the trailing unreduced block, thread 0 chases the bulge of one
// step through it and keeps the step's rotations in LDS; then thread t applies them, in order, to
// row t of the eigenvector matrix Z (column-major, Z[c * m + t]: the same column for every
// thread, so the accesses are coalesced).  Off-diagonal entries at or below 2^-52 times the
// sum of their two diagonal neighbours are set to zero.  The entries must be scaled to
// magnitudes of at most 1 (the caller scales by a power of two).  Ends with the eigenvalues in eval[]
// (column c of Z belongs to eval[c]), their ascending order (ties to the lower index) in
// order[], and the number of QR steps in *steps_out (-1 when max_steps did not converge).
constexpr int kQrThreads = kMaxSteps;   // one thread per row of Z
__global__ __launch_bounds__(kQrThreads) void k_tridiag_qr(const double *a, const double *b, int m,
                                                          int max_steps, double *Z, double *eval,
                                                          int *order, int *steps_out) {
  __shared__ double dd[kMaxSteps], ee[kMaxSteps];
  __shared__ double cs[kMaxSteps], sn[kMaxSteps];
  __shared__ int blk_lo, blk_hi, state;   // state 0: a step to apply, 1: converged, 2: failed
  const double eps = 0x1p-52;
  const int t = threadIdx.x;
  for (int i = t; i < m; i += blockDim.x) {
    dd[i] = a[i];
    ee[i] = i + 1 < m ? b[i] : 0.0;
  }
  for (int i = t; i < m * m; i += blockDim.x) Z[i] = (i / m == i % m) ? 1.0 : 0.0;
  __syncthreads();
  // hi and steps are kept alike by every lane of wave 0, which searches for the block together
  int steps = 0, hi = m - 1;
  auto negligible = [&](int j) {   // ee[j] against its diagonal neighbours
    return fabs(ee[j]) <= eps * (fabs(dd[j]) + fabs(dd[j + 1]));
  };
  for (;;) {
    if (t < 64) {
      int st = 1;
      while (hi > 0) {
        if (negligible(hi - 1)) {   // deflate
          if (t == 0) ee[hi - 1] = 0.0;
          hi--;
          continue;
        }
        // lo: one past the largest j < hi - 1 with a negligible ee[j] (0 when there is none),
        // 64 entries per ballot
        int lo = 0;
        for (int base = hi - 2; base >= 0; base -= 64) {
          const int j = base - t;
          const unsigned long long bal = __ballot(j >= 0 && negligible(j));
          if (bal) {
            lo = base - (__ffsll(bal) - 1) + 1;
            break;
          }
        }
        if (steps >= max_steps) {
          st = 2;
          break;
        }
        steps++;
        st = 0;
        if (t != 0) break;
        if (lo > 0) ee[lo - 1] = 0.0;
        // the shift: the eigenvalue of the trailing 2 x 2 block nearer its last entry
        const double p = dd[hi - 1], q = ee[hi - 1], r = dd[hi];
        const double del = 0.5 * (p - r);
        const double mu = r - q * q / (del + copysign(hypot(del, q), del));
        double x = dd[lo] - mu, z = ee[lo];
        // ak, bk: T[k][k] and T[k][k+1] as the previous rotation left them (kept in registers,
        // so the chain of rotations waits on no LDS load)
        double ak = dd[lo], bk = ee[lo];
        for (int k = lo; k < hi; k++) {
          const double ck = dd[k + 1], f = k + 1 < hi ? ee[k + 1] : 0.0;
          // G = [[c, s], [-s, c]] on (k, k+1) zeroes z against x; T <- G^T T G.  The matrix
          // comes scaled to entries of magnitude at most 1, so x^2 + z^2 cannot overflow
          const double q2 = x * x + z * z;
          const double rh = q2 > 0.0 ? rsqrt(q2) : 0.0;
          const double h = q2 * rh;
          const double c = q2 > 0.0 ? x * rh : 1.0, s = -z * rh;
          if (k > lo) ee[k - 1] = h;
          const double ek = c * s * (ak - ck) + (c * c - s * s) * bk;
          dd[k] = c * c * ak - 2.0 * c * s * bk + s * s * ck;
          ee[k] = ek;
          ak = s * s * ak + 2.0 * c * s * bk + c * c * ck;   // T[k+1][k+1]
          bk = c * f;                                        // T[k+1][k+2]
          z = -s * f;                                        // the bulge at (k, k+2)
          x = ek;
          cs[k] = c;
          sn[k] = s;
        }
        dd[hi] = ak;
        blk_lo = lo;
        blk_hi = hi;
        break;
      }
      if (t == 0) state = st;
    }
    __syncthreads();
    if (state != 0) break;
    const int lo = blk_lo, h2 = blk_hi;
    if (t < m) {   // Z <- Z G_lo G_lo+1 ... on row t, the next 16 columns loaded ahead
      constexpr int kAhead = 16;
      double carry = Z[(int64_t)lo * m + t];
      for (int k0 = lo; k0 < h2; k0 += kAhead) {
        double nx[kAhead];
#pragma unroll
        for (int u = 0; u < kAhead; u++)
          nx[u] = k0 + 1 + u <= h2 ? Z[(int64_t)(k0 + 1 + u) * m + t] : 0.0;
#pragma unroll
        for (int u = 0; u < kAhead; u++) {
          const int k = k0 + u;
          if (k < h2) {
            Z[(int64_t)k * m + t] = cs[k] * carry - sn[k] * nx[u];
            carry = sn[k] * carry + cs[k] * nx[u];
          }
        }
      }
      Z[(int64_t)h2 * m + t] = carry;
    }
    __syncthreads();
  }
  if (t == 0) {
    for (int i = 0; i < m; i++) {
      eval[i] = dd[i];
      order[i] = i;
    }
    for (int i = 1; i < m; i++) {   // insertion sort by eigenvalue, stable
      const int o = order[i];
      int j = i - 1;
      while (j >= 0 && eval[order[j]] > eval[o]) {
        order[j + 1] = order[j];
        j--;
      }
      order[j + 1] = o;
    }
    *steps_out = state == 2 ? -1 : steps;
  }
}

// Ritz vectors: Y[v * K + c] = sum_i V_i[v] Z[i, order[c]] (Z column-major)
__global__ void k_ritz(const double *V, int msteps, const double *Z, int m, const int *order,
                       int K, int64_t n, double *Y) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double acc[kMaxK];
#pragma unroll
  for (int c = 0; c < kMaxK; c++) acc[c] = 0.0;
  for (int i = 0; i < msteps; i++) {
    const double x = V[(int64_t)i * n + v];
#pragma unroll
    for (int c = 0; c < kMaxK; c++)
      if (c < K) acc[c] += x * Z[(int64_t)order[c] * m + i];
  }
#pragma unroll
  for (int c = 0; c < kMaxK; c++)
    if (c < K) Y[v * K + c] = acc[c];
}

__global__ void k_column(const double *Y, int K, int c, int64_t n, double *x) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) x[v] = Y[v * K + c];
}

// ------------------------------------------------------------------ k-means
__device__ inline double sqdist(const double *p, const double *c, int dim) {
  double d = 0.0;
  for (int j = 0; j < dim; j++) {
    const double t = p[j] - c[j];
    d = d + t * t;   // separate rounding of product and sum (contraction is off)
  }
  return d;
}

__global__ void k_to_fixed(const double *P, int64_t cnt, int64_t *Q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) Q[i] = (int64_t)rint(ldexp(P[i], kFixShift));
}

__global__ void k_km_near_init(const double *P, int64_t n, int dim, const double *c, double *near) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) near[v] = sqdist(P + v * dim, c, dim);
}
__global__ void k_km_near_min(const double *P, int64_t n, int dim, const double *c, double *near) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) near[v] = fmin(near[v], sqdist(P + v * dim, c, dim));
}

// argmax of near (the first index of the largest value): block partials, then one block
__device__ inline void better_pair(double &bv, int64_t &bi, double v, int64_t i) {
  if (v > bv || (v == bv && i < bi)) {
    bv = v;
    bi = i;
  }
}
__global__ void k_argmax_partial(const double *x, int64_t n, double *pv, int64_t *pi) {
  __shared__ double sv[kSB];
  __shared__ int64_t si[kSB];
  double bv = -INFINITY;
  int64_t bi = INT64_MAX;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    better_pair(bv, bi, x[i], i);
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = blockDim.x / 2; s >= 1; s >>= 1) {
    if ((int)threadIdx.x < s) {
      double v = sv[threadIdx.x];
      int64_t i = si[threadIdx.x];
      better_pair(v, i, sv[threadIdx.x + s], si[threadIdx.x + s]);
      sv[threadIdx.x] = v;
      si[threadIdx.x] = i;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = sv[0];
    pi[blockIdx.x] = si[0];
  }
}
// the winner's point becomes centroid c
__global__ void k_argmax_final(const double *pv, const int64_t *pi, int nb, const double *P,
                               int dim, double *C, int c) {
  __shared__ int64_t win;
  if (threadIdx.x == 0) {
    double bv = -INFINITY;
    int64_t bi = INT64_MAX;
    for (int b = 0; b < nb; b++) better_pair(bv, bi, pv[b], pi[b]);
    win = bi;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < dim; j += blockDim.x) C[c * dim + j] = P[win * dim + j];
}
__global__ void k_copy_row(const double *P, int64_t row, int dim, double *dst) {
  for (int j = threadIdx.x; j < dim; j += blockDim.x) dst[j] = P[row * dim + j];
}

// nearest centroid (strictly smaller distance wins, so ties stay with the lower index)
__global__ void k_km_assign(const double *P, int64_t n, int dim, const double *C, int k,
                            int32_t *labels, unsigned long long *changed) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ch = false;
  if (v < n) {
    // the point's coordinates are loaded once (registers), then compared with every centroid;
    // the distance is the same sum in the same order as sqdist
    double p[kMaxK];
#pragma unroll
    for (int j = 0; j < kMaxK; j++) p[j] = j < dim ? P[v * dim + j] : 0.0;
    double best = INFINITY;
    int lab = 0;
    for (int c = 0; c < k; c++) {
      const double *cc = C + c * dim;
      double d = 0.0;
#pragma unroll
      for (int j = 0; j < kMaxK; j++) {
        if (j < dim) {
          const double t = p[j] - cc[j];
          d = d + t * t;
        }
      }
      if (d < best) {
        best = d;
        lab = c;
      }
    }
    ch = labels[v] != lab;
    labels[v] = lab;
  }
  const unsigned long long b = __ballot(ch);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(changed, (unsigned long long)__popcll(b));
}

// exact fixed-point sums per (cluster, coordinate): each value split as hi * 2^20 + lo,
// 0 <= lo < 2^20, both parts summed in int64 (block shares in LDS, then global atomics)
__global__ void k_km_accum(const int64_t *Q, const int32_t *labels, int64_t n, int dim, int k,
                           unsigned long long *Sh, unsigned long long *Sl,
                           unsigned long long *cnt) {
  __shared__ unsigned long long lh[kMaxK * kMaxK], ll[kMaxK * kMaxK], lc[kMaxK];
  const int kd = k * dim;
  for (int i = threadIdx.x; i < kd; i += blockDim.x) {
    lh[i] = 0ull;
    ll[i] = 0ull;
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) lc[i] = 0ull;
  __syncthreads();
  // a grid-stride share per block (a few hundred blocks), so the global atomics below stay
  // few per address
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int c = labels[v];
    atomicAdd(&lc[c], 1ull);
    for (int j = 0; j < dim; j++) {
      const int64_t q = Q[v * dim + j];
      const int64_t hi = q >> kSplit;                   // floor
      const int64_t lo = q - (hi << kSplit);            // 0 <= lo < 2^20
      atomicAdd(&lh[c * dim + j], (unsigned long long)hi);
      atomicAdd(&ll[c * dim + j], (unsigned long long)lo);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kd; i += blockDim.x) {
    if (lh[i]) atomicAdd(&Sh[i], lh[i]);
    if (ll[i]) atomicAdd(&Sl[i], ll[i]);
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x)
    if (lc[i]) atomicAdd(&cnt[i], lc[i]);
}

// centroid = (hi * 2^20 + lo) / count * 2^-40; an empty cluster keeps its centroid
__global__ void k_km_centroids(const unsigned long long *Sh, const unsigned long long *Sl,
                               const unsigned long long *cnt, int k, int dim, double *C) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k * dim) return;
  const unsigned long long c = cnt[i / dim];
  if (c == 0) return;
  const double s = (double)(int64_t)Sh[i] * 1048576.0 + (double)(int64_t)Sl[i];
  C[i] = ldexp(s / (double)c, -kFixShift);
}

__global__ void k_spec_fill_i32(int32_t *p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st) {
  if (n > 0) k_spec_fill_i32<<<blocks(n), kSB, 0, st>>>(p, v, n);
}

template <class T>
struct DevVec {
  Buf b;
  T *get(int64_t n) { return b.get<T>(std::max<int64_t>(n, 1)); }
};

void h2d_raw(void *d, const void *h, size_t bytes, hipStream_t st) {
  if (bytes) MSLM_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st));
}
void d2h_raw(void *h, const void *d, size_t bytes, hipStream_t st) {
  if (bytes) MSLM_HIP(hipMemcpyAsync(h, d, bytes, hipMemcpyDeviceToHost, st));
}

double dot_dev(const double *x, const double *y, int64_t n, double *partial, double *out,
               hipStream_t st) {
  k_dot_partial<<<kDotBlocks, kSB, 0, st>>>(x, y, n, partial);
  k_sum_partials<<<1, kSB, 0, st>>>(partial, kDotBlocks, 1, nullptr, out);
  double h = 0.0;
  d2h_raw(&h, out, sizeof(double), st);
  MSLM_HIP(hipStreamSynchronize(st));
  return h;
}

// k-means of n points (device, row-major n x dim) into labels / centroids; returns iterations
int kmeans_dev(const double *P, int64_t n, int dim, int k, int max_iter, int32_t *labels,
               double *C, hipStream_t st) {
  DevVec<int64_t> bQ;
  DevVec<double> bnear, bpv;
  DevVec<int64_t> bpi;
  DevVec<unsigned long long> bacc;
  int64_t *Q = bQ.get(n * dim);
  double *near = bnear.get(n);
  double *pv = bpv.get(kDotBlocks);
  int64_t *pi = bpi.get(kDotBlocks);
  unsigned long long *acc = bacc.get(2 * (int64_t)k * dim + k + 1);
  unsigned long long *Sh = acc, *Sl = acc + k * dim, *cnt = acc + 2 * k * dim,
                     *changed = cnt + k;
  k_to_fixed<<<blocks(n * dim), kSB, 0, st>>>(P, n * dim, Q);
  // maximin start: point 0, then the farthest point from the chosen ones, k - 1 times
  k_copy_row<<<1, 64, 0, st>>>(P, 0, dim, C);
  k_km_near_init<<<blocks(n), kSB, 0, st>>>(P, n, dim, C, near);
  for (int c = 1; c < k; c++) {
    k_argmax_partial<<<kDotBlocks, kSB, 0, st>>>(near, n, pv, pi);
    k_argmax_final<<<1, 64, 0, st>>>(pv, pi, kDotBlocks, P, dim, C, c);
    k_km_near_min<<<blocks(n), kSB, 0, st>>>(P, n, dim, C + c * dim, near);
  }
  fill_i32(labels, -1, n, st);
  int it = 0;
  for (it = 1; it <= max_iter; it++) {
    MSLM_HIP(hipMemsetAsync(acc, 0, sizeof(unsigned long long) * (2 * k * dim + k + 1), st));
    k_km_assign<<<blocks(n), kSB, 0, st>>>(P, n, dim, C, k, labels, changed);
    k_km_accum<<<std::min<unsigned>(blocks(n), kDotBlocks), kSB, 0, st>>>(Q, labels, n, dim, k,
                                                                         Sh, Sl, cnt);
    k_km_centroids<<<blocks(k * dim), kSB, 0, st>>>(Sh, Sl, cnt, k, dim, C);
    unsigned long long h = 0;
    d2h_raw(&h, changed, sizeof(h), st);
    MSLM_HIP(hipStreamSynchronize(st));
    if (h == 0) break;
  }
  return std::min(it, max_iter);
}

struct Spectral {
  double r = 1.0, residual_max = 0.0, ms_spmv = 0.0;
  int steps = 0, sweeps = 0, km_iters = 0, second_passes = 0;
  int64_t spmv_launches = 0;
};

// The pathway on graph g: eigenvalues (host, K), optional embedding (host n x K) and labels.
Spectral bethe_hessian_run(const GraphDev &gd, hipStream_t st, double omega, double r_in, int K,
                           int msteps, int km_iter, uint64_t seed, double *eigenvalues,
                           double *embedding, int32_t *labels_host) {
  Spectral out;
  const int64_t n = gd.n;
  SpecGraph g{gd.rp.as<int64_t>(), gd.col.as<int32_t>(),
              gd.unit ? nullptr : gd.w.as<int32_t>(), n, gd.N, omega};
  DevVec<double> bd, bpart, bout, bV, bW, bT, bZ, beval, bY, bx, by;
  DevVec<int> bord, bsw;
  double *d = bd.get(n);
  double *partial = bpart.get((int64_t)kMdotBlocks * (kMaxSteps + 2));
  double *dout = bout.get(kMaxSteps + 2);
  k_bh_degree<<<blocks(n), kSB, 0, st>>>(g, d);
  double r = r_in;
  if (r <= 0.0) {   // sqrt(<d^2>/<d> - 1), or 1 when that is not above 1
    k_deg_moments<<<kDotBlocks, kSB, 0, st>>>(d, n, partial);
    k_sum_partials<<<2, kSB, 0, st>>>(partial, kDotBlocks, 2, nullptr, dout);
    double m2[2] = {0.0, 0.0};
    d2h_raw(m2, dout, sizeof(m2), st);
    MSLM_HIP(hipStreamSynchronize(st));
    const double x = m2[0] > 0.0 ? m2[1] / m2[0] - 1.0 : 0.0;
    r = x > 1.0 ? std::sqrt(x) : 1.0;
  }
  out.r = r;
  // Lanczos with full reorthogonalisation (classical Gram-Schmidt, twice)
  double *V = bV.get((int64_t)(msteps + 1) * n);
  double *w = bW.get(n);
  k_start_vector<<<blocks(n), kSB, 0, st>>>(V, n, mix64(seed));
  {
    const double nv = std::sqrt(dot_dev(V, V, n, partial, dout, st));
    k_scale_into<<<blocks(n), kSB, 0, st>>>(1.0 / nv, V, V, n);
  }
  std::vector<double> alpha, beta(1, 0.0);
  int *flag = bsw.get(3);   // [0] second pass wanted, [1] second passes taken, [2] QR steps
  fill_i32(flag, 0, 3, st);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  MSLM_HIP(hipEventCreate(&e0));
  MSLM_HIP(hipEventCreate(&e1));
  int steps = msteps;
  for (int j = 0; j < msteps; j++) {
    const double *vj = V + (int64_t)j * n;
    MSLM_HIP(hipEventRecord(e0, st));
    k_bh_apply<<<blocks(n * 16), kSB, 0, st>>>(g, d, r, vj, w);
    MSLM_HIP(hipEventRecord(e1, st));
    const double a = dot_dev(vj, w, n, partial, dout, st);   // synchronises the stream
    if (!std::isfinite(a)) throw Error(MSLM_EHIP, "Lanczos: a non-finite Rayleigh quotient");
    float ms = 0.f;
    MSLM_HIP(hipEventElapsedTime(&ms, e0, e1));
    out.ms_spmv += ms;
    out.spmv_launches++;
    alpha.push_back(a);
    k_lanczos_sub<<<blocks(n), kSB, 0, st>>>(w, vj, j ? V + (int64_t)(j - 1) * n : nullptr, a,
                                              beta[j], n);
    // classical Gram-Schmidt against every Lanczos vector, a second time when the first
    // pass cancelled most of w
    const dim3 g1(kMdotBlocks, (j + 2 + kMdotVec - 1) / kMdotVec);
    const dim3 g2(kMdotBlocks, (j + 1 + kMdotVec - 1) / kMdotVec);
    k_mdot_partial<<<g1, kSB, 0, st>>>(V, j + 1, w, n, 1, nullptr, partial);
    k_sum_partials<<<j + 2, kSB, 0, st>>>(partial, kMdotBlocks, j + 2, nullptr, dout);
    k_msub<<<blocks(n), kSB, 0, st>>>(V, j + 1, dout, nullptr, w, n);
    k_reorth_gate<<<1, 64, 0, st>>>(dout, j + 1, flag, flag + 1);
    k_mdot_partial<<<g2, kSB, 0, st>>>(V, j + 1, w, n, 0, flag, partial);
    k_sum_partials<<<j + 1, kSB, 0, st>>>(partial, kMdotBlocks, j + 1, flag, dout);
    k_msub<<<blocks(n), kSB, 0, st>>>(V, j + 1, dout, flag, w, n);
    if (j == msteps - 1) break;
    const double b = std::sqrt(dot_dev(w, w, n, partial, dout, st));
    if (!std::isfinite(b)) throw Error(MSLM_EHIP, "Lanczos: a non-finite residual norm");
    if (!(b > 1e-12 * std::max(1.0, std::fabs(a)))) {   // an invariant subspace: stop
      steps = j + 1;
      break;
    }
    beta.push_back(b);
    k_scale_into<<<blocks(n), kSB, 0, st>>>(1.0 / b, w, V + (int64_t)(j + 1) * n, n);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  out.steps = steps;
  if (K > steps) throw Error(MSLM_EUNSUPPORTED, "the Krylov space closed before k vectors");
  // the tridiagonal matrix's eigenpairs (one workgroup), the K smallest
  double *T = bT.get(2 * (int64_t)steps);
  double *Z = bZ.get((int64_t)steps * steps);
  double *eval = beval.get(steps);
  int *order = bord.get(steps);
  int *sw = flag + 2;
  // scaled by a power of two (exact) to entries of magnitude at most 1
  double big = 0.0;
  for (int i = 0; i < steps; i++) big = std::max(big, std::fabs(alpha[i]));
  for (int i = 1; i < steps; i++) big = std::max(big, std::fabs(beta[i]));
  const int ex = big > 0.0 ? std::ilogb(big) + 1 : 0;
  std::vector<double> tri(2 * (size_t)steps, 0.0);
  for (int i = 0; i < steps; i++) tri[i] = std::ldexp(alpha[i], -ex);
  for (int i = 1; i < steps; i++) tri[steps + i - 1] = std::ldexp(beta[i], -ex);
  h2d_raw(T, tri.data(), sizeof(double) * tri.size(), st);
  k_tridiag_qr<<<1, kQrThreads, 0, st>>>(T, T + steps, steps, 30 * steps, Z, eval, order, sw);
  std::vector<double> ev(steps);
  std::vector<int> ord(steps);
  d2h_raw(ev.data(), eval, sizeof(double) * steps, st);
  d2h_raw(ord.data(), order, sizeof(int) * steps, st);
  d2h_raw(&out.sweeps, sw, sizeof(int), st);
  d2h_raw(&out.second_passes, flag + 1, sizeof(int), st);
  MSLM_HIP(hipStreamSynchronize(st));
  if (out.sweeps < 0) throw Error(MSLM_EHIP, "the tridiagonal eigensolver did not converge");
  for (int c = 0; c < K; c++) eigenvalues[c] = std::ldexp(ev[ord[c]], ex);
  double *Y = bY.get(n * K);
  k_ritz<<<blocks(n), kSB, 0, st>>>(V, steps, Z, steps, order, K, n, Y);
  // residuals ||H y - lambda y|| of the returned pairs
  double *x = bx.get(n), *y = by.get(n);
  for (int c = 0; c < K; c++) {
    k_column<<<blocks(n), kSB, 0, st>>>(Y, K, c, n, x);
    k_bh_apply<<<blocks(n * 16), kSB, 0, st>>>(g, d, r, x, y);
    k_axpby<<<blocks(n), kSB, 0, st>>>(-eigenvalues[c], x, 1.0, y, n);
    out.residual_max = std::max(out.residual_max, std::sqrt(dot_dev(y, y, n, partial, dout, st)));
  }
  if (embedding) {
    d2h_raw(embedding, Y, sizeof(double) * n * K, st);
    MSLM_HIP(hipStreamSynchronize(st));
  }
  if (labels_host) {
    DevVec<int32_t> blab;
    DevVec<double> bC;
    int32_t *lab = blab.get(n);
    double *C = bC.get((int64_t)K * K);
    out.km_iters = kmeans_dev(Y, n, K, K, km_iter, lab, C, st);
    d2h_raw(labels_host, lab, sizeof(int32_t) * n, st);
    MSLM_HIP(hipStreamSynchronize(st));
  }
  return out;
}

}  // namespace
}  // namespace mslm

using namespace mslm;

extern "C" {

mslm_status mslm_kmeans(const double *points, int64_t n, int32_t dim, int32_t k,
                        int32_t max_iterations, int32_t *labels, double *centroids,
                        int32_t *iterations, void *hip_stream) {
  if (!points || !labels || n < 1 || dim < 1 || dim > kMaxK || k < 1 || k > kMaxK || k > n)
    return api_fail(MSLM_EINVAL, "k-means: need points, labels, n >= k >= 1, 1 <= dim, k <= 32");
  if (max_iterations <= 0) max_iterations = 100;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  try {
    DevVec<double> bP, bC;
    DevVec<int32_t> bl;
    double *P = bP.get(n * dim);
    double *C = bC.get((int64_t)k * dim);
    int32_t *lab = bl.get(n);
    h2d_raw(P, points, sizeof(double) * n * dim, st);
    const int it = kmeans_dev(P, n, dim, k, max_iterations, lab, C, st);
    d2h_raw(labels, lab, sizeof(int32_t) * n, st);
    if (centroids) d2h_raw(centroids, C, sizeof(double) * k * dim, st);
    MSLM_HIP(hipStreamSynchronize(st));
    if (iterations) *iterations = it;
  } catch (const Error &e) {
    return api_fail(e.status, e.what());
  } catch (const std::exception &e) {
    return api_fail(MSLM_ENOMEM, e.what());
  }
  api_clear_error();
  return MSLM_OK;
}

mslm_status mslm_bh_apply(mslm_graph *g, double r, int64_t omega_num, int64_t omega_den,
                          const double *x, double *y) {
  if (!g || !x || !y) return api_fail(MSLM_EINVAL, "graph, x or y is NULL");
  int64_t on = g->g.omega_num, od = g->g.omega_den;
  if (omega_den != 0) {
    mslm_status s = api_check_fraction(omega_num, omega_den, "omega");
    if (s != MSLM_OK) return s;
    on = omega_num;
    od = omega_den;
  }
  const int64_t n = g->g.n;
  hipStream_t st = g->st;
  try {
    SpecGraph sg{g->g.rp.as<int64_t>(), g->g.col.as<int32_t>(),
                 g->g.unit ? nullptr : g->g.w.as<int32_t>(), n, g->g.N, (double)on / (double)od};
    DevVec<double> bd, bx, by;
    double *d = bd.get(n), *dx = bx.get(n), *dy = by.get(n);
    k_bh_degree<<<blocks(n), kSB, 0, st>>>(sg, d);
    h2d_raw(dx, x, sizeof(double) * n, st);
    k_bh_apply<<<blocks(n * 16), kSB, 0, st>>>(sg, d, r, dx, dy);
    d2h_raw(y, dy, sizeof(double) * n, st);
    MSLM_HIP(hipStreamSynchronize(st));
  } catch (const Error &e) {
    return api_fail(e.status, e.what());
  } catch (const std::exception &e) {
    return api_fail(MSLM_ENOMEM, e.what());
  }
  api_clear_error();
  return MSLM_OK;
}

mslm_status mslm_bethe_hessian(mslm_graph *g, const mslm_spectral_params *p, double *eigenvalues,
                               double *embedding, int32_t *labels, mslm_spectral_result *res) {
  if (!g || !p || !eigenvalues) return api_fail(MSLM_EINVAL, "graph, params or eigenvalues is NULL");
  const int64_t n = g->g.n;
  const int K = p->k;
  if (K < 1 || K > kMaxK || K >= n)
    return api_fail(MSLM_EINVAL, "k must lie in 1..32 and below the number of supra-nodes");
  int m = p->lanczos_steps;
  if (m == 0) m = (int)std::min<int64_t>(n, std::min(kMaxSteps, std::max(4 * K, K + 152)));
  if (m < K || m > kMaxSteps || m > n)
    return api_fail(MSLM_EINVAL, "lanczos_steps must lie in k..min(256, supra-nodes)");
  int64_t on = g->g.omega_num, od = g->g.omega_den;
  if (p->omega_den != 0) {
    mslm_status s = api_check_fraction(p->omega_num, p->omega_den, "omega");
    if (s != MSLM_OK) return s;
    on = p->omega_num;
    od = p->omega_den;
  }
  if (!(p->r >= 0.0) || !std::isfinite(p->r)) return api_fail(MSLM_EINVAL, "r must be >= 0");
  const auto t0 = std::chrono::steady_clock::now();
  try {
    Spectral s = bethe_hessian_run(g->g, g->st, (double)on / (double)od, p->r, K, m,
                                   p->kmeans_iterations > 0 ? p->kmeans_iterations : 100, p->seed,
                                   eigenvalues, embedding, labels);
    if (res) {
      std::memset(res, 0, sizeof(*res));
      res->r = s.r;
      res->residual_max = s.residual_max;
      res->lanczos_steps = s.steps;
      res->tridiagonal_steps = s.sweeps;
      res->second_passes = s.second_passes;
      res->kmeans_iterations = s.km_iters;
      res->spmv_ms = s.ms_spmv;
      res->spmv_launches = s.spmv_launches;
      res->ms_total =
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
  } catch (const Error &e) {
    return api_fail(e.status, e.what());
  } catch (const std::exception &e) {
    return api_fail(MSLM_ENOMEM, e.what());
  }
  api_clear_error();
  return MSLM_OK;
}

}  // extern "C"
