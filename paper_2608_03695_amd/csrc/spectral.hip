// The Bethe-Hessian spectral pathway (Section 3.1, the paragraphs after Eq. 4) on a resident
// supra-graph: H(r) = (r^2 - 1) I - r A + D (A the supra-adjacency of Eq. 3, D its degrees),
// the k algebraically smallest eigenpairs by Lanczos with full reorthogonalisation, and
// k-means on the rows of the embedding.
//
// Kernels: the operator (16 lanes per row), block-partial dot products with a fixed grid (the
// same sums in the same order on every run), a multi-vector dot / update pair for the
// reorthogonalisation, a one-workgroup parallel Jacobi eigensolver for the small tridiagonal
// matrix (disjoint rotations per round, round-robin pairing), the Ritz vectors, and k-means
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
constexpr int kMdotBlocks = 4096; // grid of the reorthogonalisation dot products (8 per CU)
constexpr int kMaxK = 32;         // eigenvectors / clusters
constexpr int kMaxSteps = 256;    // Krylov dimension
constexpr int kFixShift = 40;     // fixed-point scale of the k-means sums
constexpr int kSplit = 20;        // a fixed-point value as hi * 2^20 + lo, 0 <= lo < 2^20
constexpr int kJacobiThreads = 1024;

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
// out[i] = sum over b of partial[b * cnt + i]: one block per i (the same order every run)
__global__ void k_sum_partials(const double *partial, int nb, int cnt, double *out) {
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

// partial[b * cnt + i] = block b's share of V_i . w, i < cnt (V column-major, n per vector);
// four vectors per pass over the block's rows, so w is read once per four
__global__ void k_mdot_partial(const double *V, int cnt, const double *w, int64_t n,
                               double *partial) {
  __shared__ double sh[kSB / 64];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per, hi = std::min<int64_t>(n, lo + per);
  for (int i0 = 0; i0 < cnt; i0 += 4) {
    const int q = std::min(4, cnt - i0);
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
      const double wk = w[k];
#pragma unroll
      for (int u = 0; u < 4; u++)
        if (u < q) s[u] += V[(int64_t)(i0 + u) * n + k] * wk;
    }
    for (int u = 0; u < q; u++) {
      const double t = block_sum(s[u], sh);
      if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * cnt + i0 + u] = t;
    }
  }
}

// w -= V h (cnt vectors)
__global__ void k_msub(const double *V, int cnt, const double *h, double *w, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s = 0.0;
  for (int i = 0; i < cnt; i++) s += V[(int64_t)i * n + k] * h[i];
  w[k] -= s;
}

// deterministic start vector: SplitMix64 of (seed, i) as a uniform value in [-1, 1)
__global__ void k_start_vector(double *v, int64_t n, uint64_t seedmix) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t z = mix64(seedmix ^ (uint64_t)i);
  v[i] = (double)(z >> 11) * 0x1p-52 - 1.0;
}

// Parallel cyclic Jacobi on the symmetric m x m matrix A (row-major, global memory), one
// workgroup: every round applies m/2 disjoint rotations (round-robin pairing of the indices,
// with a dummy when m is odd) to the rows, then to the columns and to the eigenvector matrix Z;
// sweeps until the off-diagonal norm is below tol times the matrix norm.  Ends with the
// eigenvalue order (ascending, ties to the lower index) in order[].
__global__ __launch_bounds__(kJacobiThreads) void k_jacobi(double *A, double *Z, int m, double tol,
                                                          int max_sweeps, int *order,
                                                          double *eval, int *sweeps_out) {
  __shared__ int pp[kMaxSteps / 2 + 1], qq[kMaxSteps / 2 + 1];
  __shared__ double cs[kMaxSteps / 2 + 1], sn[kMaxSteps / 2 + 1];
  __shared__ int player[kMaxSteps + 1];
  __shared__ double red[kJacobiThreads / 64];
  __shared__ int done;
  const int M = m + (m & 1);   // players, a dummy index m when m is odd
  for (int i = threadIdx.x; i < m * m; i += blockDim.x) Z[i] = (i / m == i % m) ? 1.0 : 0.0;
  __syncthreads();
  int sweep = 0;
  for (; sweep < max_sweeps; sweep++) {
    double off = 0.0, tot = 0.0;
    for (int i = threadIdx.x; i < m * m; i += blockDim.x) {
      const double a = A[i];
      tot += a * a;
      if (i / m != i % m) off += a * a;
    }
    off = block_sum(off, red);
    tot = block_sum(tot, red);
    if (threadIdx.x == 0) done = !(off > tol * tol * tot);
    __syncthreads();
    if (done) break;
    for (int i = threadIdx.x; i < M; i += blockDim.x) player[i] = i;
    __syncthreads();
    for (int round = 0; round < M - 1; round++) {
      // pairs (player[i], player[M-1-i]); rotation parameters from the current matrix
      for (int i = threadIdx.x; i < M / 2; i += blockDim.x) {
        int p = player[i], q = player[M - 1 - i];
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < m) {
          const double apq = A[p * m + q];
          if (apq != 0.0) {
            const double th = (A[q * m + q] - A[p * m + p]) / (2.0 * apq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        pp[i] = p;
        qq[i] = q;
        cs[i] = c;
        sn[i] = s;
      }
      __syncthreads();
      // rows p, q of every pair (A <- J^T A)
      for (int t = threadIdx.x; t < (M / 2) * m; t += blockDim.x) {
        const int i = t / m, k = t % m;
        const int p = pp[i], q = qq[i];
        if (q >= m || sn[i] == 0.0) continue;
        const double a = A[p * m + k], b = A[q * m + k];
        A[p * m + k] = cs[i] * a - sn[i] * b;
        A[q * m + k] = sn[i] * a + cs[i] * b;
      }
      __syncthreads();
      // columns p, q (A <- A J) and the eigenvectors (Z <- Z J)
      for (int t = threadIdx.x; t < (M / 2) * m; t += blockDim.x) {
        const int i = t / m, k = t % m;
        const int p = pp[i], q = qq[i];
        if (q >= m || sn[i] == 0.0) continue;
        const double a = A[k * m + p], b = A[k * m + q];
        A[k * m + p] = cs[i] * a - sn[i] * b;
        A[k * m + q] = sn[i] * a + cs[i] * b;
        const double za = Z[k * m + p], zb = Z[k * m + q];
        Z[k * m + p] = cs[i] * za - sn[i] * zb;
        Z[k * m + q] = sn[i] * za + cs[i] * zb;
      }
      __syncthreads();
      // next round: player 0 stays, the others rotate by one place
      if (threadIdx.x == 0) {
        const int last = player[M - 1];
        for (int i = M - 1; i > 1; i--) player[i] = player[i - 1];
        player[1] = last;
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    for (int i = 0; i < m; i++) {
      eval[i] = A[i * m + i];
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
    *sweeps_out = sweep;
  }
}

// Ritz vectors: Y[v * K + c] = sum_i V_i[v] Z[i, order[c]]
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
      if (c < K) acc[c] += x * Z[i * m + order[c]];
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
    double best = INFINITY;
    int lab = 0;
    for (int c = 0; c < k; c++) {
      const double d = sqdist(P + v * dim, C + c * dim, dim);
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
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) {
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
  k_sum_partials<<<1, kSB, 0, st>>>(partial, kDotBlocks, 1, out);
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
    k_km_accum<<<blocks(n), kSB, 0, st>>>(Q, labels, n, dim, k, Sh, Sl, cnt);
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
  int steps = 0, sweeps = 0, km_iters = 0;
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
    k_sum_partials<<<2, kSB, 0, st>>>(partial, kDotBlocks, 2, dout);
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
    for (int pass = 0; pass < 2; pass++) {
      k_mdot_partial<<<kMdotBlocks, kSB, 0, st>>>(V, j + 1, w, n, partial);
      k_sum_partials<<<j + 1, kSB, 0, st>>>(partial, kMdotBlocks, j + 1, dout);
      k_msub<<<blocks(n), kSB, 0, st>>>(V, j + 1, dout, w, n);
    }
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
  // the tridiagonal matrix, its eigenpairs (one workgroup), the K smallest
  std::vector<double> Th((size_t)steps * steps, 0.0);
  for (int i = 0; i < steps; i++) {
    Th[(size_t)i * steps + i] = alpha[i];
    if (i + 1 < steps) {
      Th[(size_t)i * steps + i + 1] = beta[i + 1];
      Th[(size_t)(i + 1) * steps + i] = beta[i + 1];
    }
  }
  double *T = bT.get((int64_t)steps * steps);
  double *Z = bZ.get((int64_t)steps * steps);
  double *eval = beval.get(steps);
  int *order = bord.get(steps);
  int *sw = bsw.get(1);
  h2d_raw(T, Th.data(), sizeof(double) * Th.size(), st);
  k_jacobi<<<1, kJacobiThreads, 0, st>>>(T, Z, steps, 1e-15, 60, order, eval, sw);
  std::vector<double> ev(steps);
  std::vector<int> ord(steps);
  d2h_raw(ev.data(), eval, sizeof(double) * steps, st);
  d2h_raw(ord.data(), order, sizeof(int) * steps, st);
  d2h_raw(&out.sweeps, sw, sizeof(int), st);
  MSLM_HIP(hipStreamSynchronize(st));
  for (int c = 0; c < K; c++) eigenvalues[c] = ev[ord[c]];
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
      res->jacobi_sweeps = s.sweeps;
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
