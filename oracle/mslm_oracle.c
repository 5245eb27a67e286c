/*
 * Plain sequential reference of the multislice-modularity Leiden schedule.
 *
 * TEST INFRASTRUCTURE ONLY: this oracle is built and called by the tests, the smoke check
 * and the benchmark's CPU baseline.  The product library never links or calls it, and it
 * shares no source with the HIP path.
 *
 * What it computes
 *   - The supra-graph of Eq. 3 (Section 3.1): per-snapshot adjacency on the diagonal, ordinal
 *     coupling omega between copies (i,s) and (i,s+1) of every node by default; in general
 *     omega^(sr) = omega * c_sr for a given integer matrix c (Eq. 6), and optionally only
 *     between copies present in both slices (a copy is present when it has an edge there).
 *   - Leiden optimisation (Section 3.2, citing Traag et al. 2019: local moving, refinement that
 *     keeps communities well connected, aggregation) of the multislice modularity Q_MS of Eq. 6
 *     with its per-slice null model gamma k_i^s k_j^s / 2m^s, made fully deterministic:
 *       * synchronous colour-batched local moving (first-fit colouring in decreasing hash
 *         priority), exact gains, argmax with ties to the lowest community label, moves only
 *         on strict improvement;
 *       * round-synchronous refinement in which a singleton proposes its best well-connected
 *         sub-community of positive gain and merges when it outranks every proposing
 *         neighbour of its community;
 *       * aggregation by refined sub-communities, super-nodes carrying per-slice degree
 *         profiles, the local-moving partition as the next level's start;
 *       * after the levels: communities split into connected components, labels by first
 *         appearance in supra-node order v = s*N + i.
 *   - Variants of the objective (Eq. 6 in its full generality, Section 3.2): a resolution
 *     gamma^(s) per slice; the global null model of Eq. 5 over the supra-graph; the multislice
 *     CPM (null term gamma^(s) n_i n_j with node weight 1 per supra-node); and a start
 *     partition for the first iteration (warm start / resume).
 *   - Exact arithmetic: integer weights are scaled by the coupling denominator b (omega = a/b)
 *     so all weights are integers; gains are compared as exact rationals (int128 when a unit
 *     lies in one slice, an own arbitrary-precision integer otherwise).  Nothing is rounded.
 *
 * Every parameter, reading and tie rule is listed in the design notes of the repository.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2
#define ORC_EOVERFLOW -3
#define ORC_EUNSUPPORTED -4

#define NONE_LABEL 0xffffffffu
#define MAX_SLICES 64
#define DEFAULT_SWEEPS 32
#define MAX_REFINE_ROUNDS 256
#define MAX_ITER_CAP 32

/* ------------------------------------------------------------------ small exact integers */
/* Sign-magnitude integers of up to BN_CAP 32-bit limbs, enough for a product of 64 slice
 * denominators below 2^62 (a resolution denominator times 2m_s) times a 2^125 numerator. */
#define BN_CAP 136
typedef struct { int neg; int len; uint32_t d[BN_CAP]; } bn_t;

static void bn_zero(bn_t *x) { x->neg = 0; x->len = 0; }
static void bn_trim(bn_t *x) { while (x->len > 0 && x->d[x->len - 1] == 0) x->len--; if (!x->len) x->neg = 0; }
static void bn_from_u64(bn_t *x, uint64_t v) {
  x->neg = 0; x->len = 0;
  while (v) { x->d[x->len++] = (uint32_t)v; v >>= 32; }
}
/* |x| *= m */
static void bn_mul_u64(bn_t *x, uint64_t m) {
  if (m == 0 || x->len == 0) { bn_zero(x); return; }
  unsigned __int128 carry = 0;
  for (int i = 0; i < x->len; i++) {
    unsigned __int128 t = (unsigned __int128)x->d[i] * m + carry;
    x->d[i] = (uint32_t)t;
    carry = t >> 32;
  }
  while (carry) {
    if (x->len >= BN_CAP) { fprintf(stderr, "oracle bignum overflow\n"); abort(); }
    x->d[x->len++] = (uint32_t)carry;
    carry >>= 32;
  }
}
static int bn_cmp_mag(const bn_t *a, const bn_t *b) {
  if (a->len != b->len) return a->len < b->len ? -1 : 1;
  for (int i = a->len - 1; i >= 0; i--)
    if (a->d[i] != b->d[i]) return a->d[i] < b->d[i] ? -1 : 1;
  return 0;
}
/* r = |a| + |b| (magnitudes) */
static void bn_add_mag(bn_t *r, const bn_t *a, const bn_t *b) {
  int n = a->len > b->len ? a->len : b->len;
  uint64_t c = 0;
  for (int i = 0; i < n; i++) {
    uint64_t s = c + (i < a->len ? a->d[i] : 0) + (i < b->len ? b->d[i] : 0);
    r->d[i] = (uint32_t)s; c = s >> 32;
  }
  r->len = n;
  if (c) { if (n >= BN_CAP) { fprintf(stderr, "oracle bignum overflow\n"); abort(); } r->d[r->len++] = (uint32_t)c; }
}
/* r = |a| - |b|, requires |a| >= |b| */
static void bn_sub_mag(bn_t *r, const bn_t *a, const bn_t *b) {
  int64_t br = 0;
  for (int i = 0; i < a->len; i++) {
    int64_t s = (int64_t)a->d[i] - (i < b->len ? b->d[i] : 0) - br;
    br = s < 0; if (s < 0) s += ((int64_t)1 << 32);
    r->d[i] = (uint32_t)s;
  }
  r->len = a->len; bn_trim(r);
}
/* r = a + (negate_b ? -b : b), signed */
static void bn_add(bn_t *r, const bn_t *a, const bn_t *b, int negate_b) {
  int bneg = b->len ? (b->neg ^ negate_b) : 0;
  bn_t t;
  if (a->neg == bneg) { bn_add_mag(&t, a, b); t.neg = a->neg; }
  else if (bn_cmp_mag(a, b) >= 0) { bn_sub_mag(&t, a, b); t.neg = a->neg; }
  else { bn_sub_mag(&t, b, a); t.neg = bneg; }
  bn_trim(&t);
  *r = t;
}
static int bn_cmp(const bn_t *a, const bn_t *b) {
  if (a->neg != b->neg) return a->neg ? -1 : 1;
  int m = bn_cmp_mag(a, b);
  return a->neg ? -m : m;
}

/* ------------------------------------------------------------------ hashing */
/* SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014). */
uint64_t orc_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}
uint64_t orc_priority(uint64_t seed, int it, int lvl, int phase, uint32_t v) {
  uint64_t key = (uint64_t)v | ((uint64_t)phase << 32) | ((uint64_t)lvl << 40) | ((uint64_t)it << 48);
  return orc_mix64(key ^ orc_mix64(seed));
}

/* ------------------------------------------------------------------ (label, slice) -> value map */
typedef struct { uint64_t *key; int64_t *val; uint64_t cap, used; } map_t;
#define MAP_EMPTY 0xffffffffffffffffULL
static uint64_t mkey(uint32_t label, int32_t s) { return ((uint64_t)label << 8) | (uint64_t)s; }
static int map_init(map_t *m, uint64_t want) {
  uint64_t cap = 16; while (cap < 2 * want + 16) cap <<= 1;
  m->key = malloc(cap * sizeof(uint64_t)); m->val = malloc(cap * sizeof(int64_t));
  if (!m->key || !m->val) return ORC_ENOMEM;
  memset(m->key, 0xff, cap * sizeof(uint64_t)); m->cap = cap; m->used = 0; return ORC_OK;
}
static void map_free(map_t *m) { free(m->key); free(m->val); m->key = NULL; m->val = NULL; }
static uint64_t map_slot(const map_t *m, uint64_t k) {
  uint64_t h = orc_mix64(k) & (m->cap - 1);
  while (m->key[h] != MAP_EMPTY && m->key[h] != k) h = (h + 1) & (m->cap - 1);
  return h;
}
static int64_t map_get(const map_t *m, uint32_t label, int32_t s) {
  uint64_t h = map_slot(m, mkey(label, s));
  return m->key[h] == MAP_EMPTY ? 0 : m->val[h];
}
static void map_add(map_t *m, uint32_t label, int32_t s, int64_t v) {
  if (2 * (m->used + 1) > m->cap) {
    map_t n2; uint64_t cap = m->cap * 2;
    n2.key = malloc(cap * sizeof(uint64_t)); n2.val = malloc(cap * sizeof(int64_t));
    if (!n2.key || !n2.val) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    memset(n2.key, 0xff, cap * sizeof(uint64_t)); n2.cap = cap; n2.used = 0;
    for (uint64_t i = 0; i < m->cap; i++) if (m->key[i] != MAP_EMPTY) {
      uint64_t h = map_slot(&n2, m->key[i]); n2.key[h] = m->key[i]; n2.val[h] = m->val[i]; n2.used++;
    }
    map_free(m); *m = n2;
  }
  uint64_t k = mkey(label, s), h = map_slot(m, k);
  if (m->key[h] == MAP_EMPTY) { m->key[h] = k; m->val[h] = 0; m->used++; }
  m->val[h] += v;
}

/* ------------------------------------------------------------------ graphs */
typedef struct {
  int64_t n, nnz;
  int64_t *rp; int32_t *col; int64_t *w;     /* CSR of scaled weights, no self entries */
  int64_t *pp; int32_t *ps; int64_t *pk;     /* per-unit slice profile (nonzero degrees) */
} level_t;

typedef struct orc_graph {
  int32_t N, T;
  int64_t a, b;                /* omega = a/b, reduced */
  int64_t twom[MAX_SLICES];    /* 2m_s, unscaled */
  level_t g0;
  int32_t *raw;                /* level-0 raw intra weight per entry, 0 for coupling entries */
  int32_t cmat[MAX_SLICES * MAX_SLICES];   /* coupling multipliers c_sr (omega^(sr) = omega c_sr) */
  int present_only;            /* coupling only between copies present in both slices */
  char *present;               /* [N*T] copy (i,s) has an intra edge */
  int64_t ctot;                /* sum of c_sr over the ordered coupled copy pairs */
} orc_graph;

/* The coupling multiplier of copies (i,s) and (i,r), 0 when they are not coupled. */
static int64_t coupled(const orc_graph *g, int32_t i, int32_t s, int32_t r) {
  if (s == r) return 0;
  int64_t c = g->cmat[s * g->T + r];
  if (c && g->present_only &&
      !(g->present[(int64_t)s * g->N + i] && g->present[(int64_t)r * g->N + i]))
    return 0;
  return c;
}

static void level_free(level_t *g) {
  free(g->rp); free(g->col); free(g->w); free(g->pp); free(g->ps); free(g->pk);
  memset(g, 0, sizeof(*g));
}

typedef struct { int64_t row; int32_t col; int32_t raw; int32_t inter; } ent_t;
static int ent_cmp(const void *x, const void *y) {
  const ent_t *a = x, *b = y;
  if (a->row != b->row) return a->row < b->row ? -1 : 1;
  if (a->col != b->col) return a->col < b->col ? -1 : 1;
  return 0;
}

static int64_t gcd64(int64_t x, int64_t y) { while (y) { int64_t t = x % y; x = y; y = t; } return x; }

void orc_destroy(orc_graph *g);

/* coupling: T*T multipliers c_sr >= 0 (symmetric, zero diagonal; NULL: 1 for |s-r| = 1, the
 * ordinal coupling); present_only: coupling entries only between copies that have an edge in
 * their slices. */
int orc_create(int32_t N, int32_t T, const int64_t *off, const int32_t *src, const int32_t *dst,
               const int32_t *w, int64_t omega_num, int64_t omega_den, const int32_t *coupling,
               int32_t present_only, orc_graph **out) {
  *out = NULL;
  if (N < 1 || T < 1 || T > MAX_SLICES || omega_num < 0 || omega_den < 1) return ORC_EINVAL;
  if (omega_num >= ((int64_t)1 << 31) || omega_den >= ((int64_t)1 << 31)) return ORC_EOVERFLOW;
  int32_t cm[MAX_SLICES * MAX_SLICES];
  for (int s = 0; s < T; s++)
    for (int r = 0; r < T; r++) {
      int32_t c = coupling ? coupling[s * T + r] : (s - r == 1 || r - s == 1);
      if (c < 0 || c >= (1 << 16) || (s == r && c != 0)) return ORC_EINVAL;
      cm[s * T + r] = c;
    }
  for (int s = 0; s < T; s++)
    for (int r = 0; r < T; r++) if (cm[s * T + r] != cm[r * T + s]) return ORC_EINVAL;
  int64_t gg = omega_num ? gcd64(omega_num, omega_den) : omega_den;
  int64_t a = omega_num / gg, b = omega_den / gg;
  int64_t E = off[T];
  int64_t n = (int64_t)N * T;
  if (n * 33 >= ((int64_t)1 << 32)) return ORC_EUNSUPPORTED;
  char *present = calloc(n ? n : 1, 1);
  for (int32_t s = 0; s < T; s++)
    for (int64_t k = off[s]; k < off[s + 1]; k++)
      if (src[k] >= 0 && src[k] < N && dst[k] >= 0 && dst[k] < N) {
        present[(int64_t)s * N + src[k]] = 1;
        present[(int64_t)s * N + dst[k]] = 1;
      }
  orc_graph tmp;
  tmp.N = N; tmp.T = T; tmp.present_only = present_only != 0; tmp.present = present;
  memcpy(tmp.cmat, cm, sizeof(cm));
  int64_t ninter = 0, ctot = 0;
  for (int32_t s = 0; s < T; s++)
    for (int32_t r = 0; r < T; r++)
      for (int32_t i = 0; i < N; i++) {
        int64_t c = coupled(&tmp, i, s, r);
        ctot += c;
        if (c && s < r && a > 0) ninter++;
      }
  int64_t cap = 2 * E + 2 * ninter;
  ent_t *e = malloc((cap ? cap : 1) * sizeof(ent_t));
  if (!e) { free(present); return ORC_ENOMEM; }
  int64_t m = 0;
  for (int32_t s = 0; s < T; s++) {
    if (off[s] > off[s + 1]) { free(e); return ORC_EINVAL; }
    for (int64_t k = off[s]; k < off[s + 1]; k++) {
      int32_t u = src[k], x = dst[k], ww = w ? w[k] : 1;
      if (u < 0 || u >= N || x < 0 || x >= N || u == x || ww < 1) { free(e); free(present); return ORC_EINVAL; }
      int64_t gu = (int64_t)s * N + u, gx = (int64_t)s * N + x;
      e[m++] = (ent_t){gu, (int32_t)gx, ww, 0};
      e[m++] = (ent_t){gx, (int32_t)gu, ww, 0};
    }
  }
  /* coupling entries: ent_t.raw holds the multiplier c_sr, ent_t.inter marks them */
  if (a > 0)
    for (int32_t s = 0; s < T; s++)
      for (int32_t r = s + 1; r < T; r++)
        for (int32_t i = 0; i < N; i++) {
          int64_t c = coupled(&tmp, i, s, r);
          if (!c) continue;
          int64_t v = (int64_t)s * N + i, x = (int64_t)r * N + i;
          e[m++] = (ent_t){v, (int32_t)x, (int32_t)c, 1};
          e[m++] = (ent_t){x, (int32_t)v, (int32_t)c, 1};
        }
  qsort(e, m, sizeof(ent_t), ent_cmp);
  /* merge repeated pairs (their weights add) */
  int64_t u = 0;
  for (int64_t k = 0; k < m; k++) {
    if (u > 0 && e[u - 1].row == e[k].row && e[u - 1].col == e[k].col) {
      int64_t s2 = (int64_t)e[u - 1].raw + e[k].raw;
      if (s2 >= ((int64_t)1 << 31)) { free(e); free(present); return ORC_EOVERFLOW; }
      e[u - 1].raw = (int32_t)s2;
    } else e[u++] = e[k];
  }
  m = u;
  orc_graph *g = calloc(1, sizeof(orc_graph));
  g->N = N; g->T = T; g->a = a; g->b = b;
  memcpy(g->cmat, cm, sizeof(cm));
  g->present_only = present_only != 0; g->present = present; g->ctot = ctot;
  level_t *L = &g->g0;
  L->n = n; L->nnz = m;
  L->rp = calloc(n + 1, sizeof(int64_t)); L->col = malloc((m ? m : 1) * sizeof(int32_t));
  L->w = malloc((m ? m : 1) * sizeof(int64_t)); g->raw = malloc((m ? m : 1) * sizeof(int32_t));
  int64_t *kdeg = calloc(n, sizeof(int64_t));
  for (int64_t k = 0; k < m; k++) {
    L->rp[e[k].row + 1]++;
    L->col[k] = e[k].col;
    L->w[k] = e[k].inter ? a * (int64_t)e[k].raw : b * (int64_t)e[k].raw;
    g->raw[k] = e[k].inter ? 0 : e[k].raw;
    if (!e[k].inter) kdeg[e[k].row] += e[k].raw;
  }
  free(e);
  for (int64_t v = 0; v < n; v++) L->rp[v + 1] += L->rp[v];
  for (int32_t s = 0; s < T; s++) {
    int64_t t2 = 0;
    for (int32_t i = 0; i < N; i++) t2 += kdeg[(int64_t)s * N + i];
    if (t2 >= ((int64_t)1 << 31)) { free(kdeg); orc_destroy(g); return ORC_EOVERFLOW; }
    g->twom[s] = t2;
  }
  int64_t np = 0;
  for (int64_t v = 0; v < n; v++) np += kdeg[v] > 0;
  L->pp = calloc(n + 1, sizeof(int64_t)); L->ps = malloc((np ? np : 1) * sizeof(int32_t));
  L->pk = malloc((np ? np : 1) * sizeof(int64_t));
  int64_t q = 0;
  for (int64_t v = 0; v < n; v++) {
    if (kdeg[v] > 0) { L->ps[q] = (int32_t)(v / N); L->pk[q] = kdeg[v]; q++; }
    L->pp[v + 1] = q;
  }
  free(kdeg);
  *out = g;
  return ORC_OK;
}

void orc_destroy(orc_graph *g) {
  if (!g) return;
  level_free(&g->g0); free(g->raw); free(g->present); free(g);
}

int64_t orc_nnz(const orc_graph *g) { return g->g0.nnz; }
/* sum over ordered coupled copy pairs of c_sr: 2mu = sum_s 2m_s + omega * this */
int64_t orc_coupling_total(const orc_graph *g) { return g->ctot; }
void orc_csr(const orc_graph *g, int64_t *rp, int32_t *col, int64_t *w, int32_t *raw, int64_t *twom) {
  memcpy(rp, g->g0.rp, (g->g0.n + 1) * sizeof(int64_t));
  memcpy(col, g->g0.col, g->g0.nnz * sizeof(int32_t));
  memcpy(w, g->g0.w, g->g0.nnz * sizeof(int64_t));
  memcpy(raw, g->raw, g->g0.nnz * sizeof(int32_t));
  memcpy(twom, g->twom, g->T * sizeof(int64_t));
}

/* ------------------------------------------------------------------ exact gains */
typedef struct {
  const int64_t *gp, *gq;      /* per slice: resolution gamma^(s) = gp[s]/gq[s], reduced */
  int64_t b;                   /* coupling denominator */
  const int64_t *S;            /* per-slice denominators: 2m_s, or 1 for an empty slice (and
                                  1 for every slice of the multislice CPM) */
} coef_t;

/* Exact value of  W*Pi - b*sum_j gp_j*k_j*y_j*(Pi/(gq_j*S_j))  with Pi = prod_j gq_j*S_j over
 * the unit's profile slices s_j.  For one fixed unit Pi is a common positive factor of every
 * target, so the ordering of these values is the ordering of the b-scaled gains
 *     W - b * sum_j gamma^(s_j) k_j y_j / S_j.
 * Single-slice units use int128; others the bignum path. */
typedef struct { int big; i128 small; bn_t v; } gval_t;

static void gain_value(const coef_t *cf, int64_t W, int m, const int32_t *ps, const int64_t *pk,
                       const int64_t *y, gval_t *out) {
  if (m <= 1) {
    out->big = 0;
    if (m == 0) { out->small = W; return; }
    int s = ps[0];
    out->small = (i128)cf->gq[s] * cf->S[s] * W - (i128)(cf->gp[s] * cf->b) * ((i128)pk[0] * y[0]);
    return;
  }
  /* sum_j gp_j k_j y_j / (gq_j S_j) as num/den, den = prod gq_j S_j */
  bn_t num, den, t1, t2;
  bn_zero(&num); bn_from_u64(&den, 1);
  for (int j = 0; j < m; j++) {
    int s = ps[j];
    uint64_t D = (uint64_t)cf->gq[s] * (uint64_t)cf->S[s];   /* < 2^62 */
    int64_t ky = pk[j] * y[j];          /* < 2^62 by the slice-size precondition */
    bn_mul_u64(&num, D);
    t1 = den; bn_mul_u64(&t1, (uint64_t)(ky < 0 ? -ky : ky)); bn_mul_u64(&t1, (uint64_t)cf->gp[s]);
    t1.neg = ky < 0 && t1.len;
    bn_add(&num, &num, &t1, 0);
    bn_mul_u64(&den, D);
  }
  /* W*den - b*num */
  t1 = den;
  uint64_t aw = (uint64_t)(W < 0 ? -W : W);
  bn_mul_u64(&t1, aw); t1.neg = W < 0 && t1.len;
  t2 = num; bn_mul_u64(&t2, (uint64_t)cf->b);
  if (t2.len == 0) t2.neg = 0;
  out->big = 1;
  bn_add(&out->v, &t1, &t2, 1);
}

static void bn_from_i128(bn_t *x, i128 s) {
  unsigned __int128 mg = s < 0 ? -(unsigned __int128)s : (unsigned __int128)s;
  x->len = 0;
  while (mg) { x->d[x->len++] = (uint32_t)mg; mg >>= 32; }
  x->neg = (s < 0) && x->len;
}
static int gval_cmp(const gval_t *x, const gval_t *y) {
  if (!x->big && !y->big) return x->small < y->small ? -1 : (x->small > y->small ? 1 : 0);
  bn_t a, b;
  if (x->big) a = x->v; else bn_from_i128(&a, x->small);
  if (y->big) b = y->v; else bn_from_i128(&b, y->small);
  return bn_cmp(&a, &b);
}
static int gval_sign(const gval_t *x) {
  if (!x->big) return x->small < 0 ? -1 : (x->small > 0 ? 1 : 0);
  return x->v.len == 0 ? 0 : (x->v.neg ? -1 : 1);
}

/* ------------------------------------------------------------------ canonical labels */
typedef struct { uint32_t lab; int64_t v; } lv_t;
static int lv_cmp(const void *x, const void *y) {
  const lv_t *a = x, *b = y;
  if (a->lab != b->lab) return a->lab < b->lab ? -1 : 1;
  return a->v < b->v ? -1 : (a->v > b->v);
}
/* out[v] = dense rank of label(v)'s community by its smallest member; returns #communities */
static int64_t canon(int64_t n, const uint32_t *lab, uint32_t *out) {
  lv_t *a = malloc((n ? n : 1) * sizeof(lv_t));
  for (int64_t v = 0; v < n; v++) { a[v].lab = lab[v]; a[v].v = v; }
  qsort(a, n, sizeof(lv_t), lv_cmp);
  char *ismin = calloc(n ? n : 1, 1);
  for (int64_t i = 0; i < n; i++) if (i == 0 || a[i].lab != a[i - 1].lab) ismin[a[i].v] = 1;
  uint32_t *rank = malloc((n ? n : 1) * sizeof(uint32_t));
  int64_t c = 0;
  for (int64_t v = 0; v < n; v++) if (ismin[v]) rank[v] = (uint32_t)c++;
  int64_t head = 0;
  for (int64_t i = 0; i < n; i++) {
    if (i == 0 || a[i].lab != a[i - 1].lab) head = a[i].v;
    out[a[i].v] = rank[head];
  }
  free(a); free(ismin); free(rank);
  return c;
}

/* ------------------------------------------------------------------ colouring */
typedef struct { uint64_t h; int64_t v; } pr_t;
static int pr_cmp_desc(const void *x, const void *y) {
  const pr_t *a = x, *b = y;
  if (a->h != b->h) return a->h > b->h ? -1 : 1;
  return a->v > b->v ? -1 : (a->v < b->v);
}
/* First-fit colouring in decreasing priority (hash, id): colour(v) is the smallest colour not
 * used by a neighbour of higher priority.  Returns the number of colours. */
static int32_t colour_units(const level_t *g, const uint32_t *local, uint64_t seed, int it, int lvl,
                            int32_t *col) {
  int64_t n = g->n;
  pr_t *o = malloc((n ? n : 1) * sizeof(pr_t));
  for (int64_t v = 0; v < n; v++) { o[v].h = orc_priority(seed, it, lvl, 0, local[v]); o[v].v = v; }
  qsort(o, n, sizeof(pr_t), pr_cmp_desc);
  for (int64_t v = 0; v < n; v++) col[v] = -1;
  int64_t maxdeg = 0;
  for (int64_t v = 0; v < n; v++) if (g->rp[v + 1] - g->rp[v] > maxdeg) maxdeg = g->rp[v + 1] - g->rp[v];
  int64_t *stamp = malloc((maxdeg + 2) * sizeof(int64_t));
  for (int64_t c = 0; c < maxdeg + 2; c++) stamp[c] = -1;
  int32_t ncol = 0;
  for (int64_t i = 0; i < n; i++) {
    int64_t v = o[i].v;
    for (int64_t e = g->rp[v]; e < g->rp[v + 1]; e++) {
      int32_t c = col[g->col[e]];
      if (c >= 0 && c <= maxdeg) stamp[c] = v;
    }
    int32_t c = 0;
    while (stamp[c] == v) c++;
    col[v] = c;
    if (c + 1 > ncol) ncol = c + 1;
  }
  free(o); free(stamp);
  return ncol;
}

/* ------------------------------------------------------------------ neighbour accumulation */
typedef struct { uint32_t lab; int64_t w; } acc_t;
static int acc_cmp(const void *x, const void *y) {
  const acc_t *a = x, *b = y;
  return a->lab < b->lab ? -1 : (a->lab > b->lab);
}
/* Weights from v to each label present among its neighbours (optionally only neighbours
 * whose filter label equals `only`), sorted by label.  Returns the number of labels. */
static int64_t gather(const level_t *g, int64_t v, const uint32_t *lab, const uint32_t *filt,
                      uint32_t only, acc_t *buf) {
  int64_t k = 0;
  for (int64_t e = g->rp[v]; e < g->rp[v + 1]; e++) {
    int32_t x = g->col[e];
    if (filt && filt[x] != only) continue;
    buf[k].lab = lab[x]; buf[k].w = g->w[e]; k++;
  }
  qsort(buf, k, sizeof(acc_t), acc_cmp);
  int64_t u = 0;
  for (int64_t i = 0; i < k; i++) {
    if (u > 0 && buf[u - 1].lab == buf[i].lab) buf[u - 1].w += buf[i].w;
    else buf[u++] = buf[i];
  }
  return u;
}

/* ------------------------------------------------------------------ statistics and trace */
typedef struct {
  int64_t sweeps, moves, sweep_cap_hits, refine_rounds, merges, splits;
  int32_t levels_run, iterations_run, n_communities, colours_first;
} orc_stats;

typedef struct {
  int it, lvl; int64_t n, nnz; int32_t ncol, sweeps;
  int64_t *rp; int32_t *col; int64_t *w; int64_t *pp; int32_t *ps; int64_t *pk;
  int32_t *colour; uint32_t *p_in, *p_lm, *r; int64_t *map0; int has_r;
  int64_t *ext; char *wc;     /* refinement bookkeeping at its end (valid for founders) */
} trace_level_t;

typedef struct { int on; int count, cap; trace_level_t *lv; } trace_t;
static trace_t g_trace;

void orc_trace_enable(int on) {
  for (int i = 0; i < g_trace.count; i++) {
    trace_level_t *t = &g_trace.lv[i];
    free(t->rp); free(t->col); free(t->w); free(t->pp); free(t->ps); free(t->pk);
    free(t->colour); free(t->p_in); free(t->p_lm); free(t->r); free(t->map0);
    free(t->ext); free(t->wc);
  }
  free(g_trace.lv);
  memset(&g_trace, 0, sizeof(g_trace));
  g_trace.on = on;
}
int orc_trace_count(void) { return g_trace.count; }
void orc_trace_info(int i, int64_t *info) {
  trace_level_t *t = &g_trace.lv[i];
  info[0] = t->it; info[1] = t->lvl; info[2] = t->n; info[3] = t->nnz; info[4] = t->ncol;
  info[5] = t->sweeps; info[6] = t->pp[t->n]; info[7] = t->has_r;
}
void orc_trace_get(int i, int64_t *rp, int32_t *col, int64_t *w, int64_t *pp, int32_t *ps, int64_t *pk,
                   int32_t *colour, uint32_t *p_in, uint32_t *p_lm, uint32_t *r, int64_t *map0, int64_t n0) {
  trace_level_t *t = &g_trace.lv[i];
  memcpy(rp, t->rp, (t->n + 1) * 8); memcpy(col, t->col, t->nnz * 4); memcpy(w, t->w, t->nnz * 8);
  memcpy(pp, t->pp, (t->n + 1) * 8); memcpy(ps, t->ps, t->pp[t->n] * 4); memcpy(pk, t->pk, t->pp[t->n] * 8);
  memcpy(colour, t->colour, t->n * 4); memcpy(p_in, t->p_in, t->n * 4); memcpy(p_lm, t->p_lm, t->n * 4);
  if (t->has_r) memcpy(r, t->r, t->n * 4);
  memcpy(map0, t->map0, n0 * 8);
}
/* the refinement's running edge weight to the rest of the community and its
 * well-connectedness flag, per founder of a refined sub-community (scaled weights) */
void orc_trace_refine(int i, int64_t *ext, char *wc) {
  trace_level_t *t = &g_trace.lv[i];
  if (!t->has_r) return;
  memcpy(ext, t->ext, t->n * 8); memcpy(wc, t->wc, t->n);
}
static void *dupmem(const void *p, size_t bytes) { void *q = malloc(bytes ? bytes : 1); memcpy(q, p, bytes); return q; }
static trace_level_t *trace_push(int it, int lvl, const level_t *g, const int64_t *map0, int64_t n0) {
  if (!g_trace.on) return NULL;
  if (g_trace.count == g_trace.cap) {
    g_trace.cap = g_trace.cap ? 2 * g_trace.cap : 8;
    g_trace.lv = realloc(g_trace.lv, g_trace.cap * sizeof(trace_level_t));
  }
  trace_level_t *t = &g_trace.lv[g_trace.count++];
  memset(t, 0, sizeof(*t));
  t->it = it; t->lvl = lvl; t->n = g->n; t->nnz = g->nnz;
  t->rp = dupmem(g->rp, (g->n + 1) * 8); t->col = dupmem(g->col, g->nnz * 4); t->w = dupmem(g->w, g->nnz * 8);
  t->pp = dupmem(g->pp, (g->n + 1) * 8); t->ps = dupmem(g->ps, g->pp[g->n] * 4); t->pk = dupmem(g->pk, g->pp[g->n] * 8);
  t->map0 = dupmem(map0, n0 * 8);
  return t;
}

/* ------------------------------------------------------------------ local moving */
typedef struct { const orc_graph *G; coef_t cf; int64_t n; } ctx_t;

static void profile_values(const level_t *g, int64_t v, const map_t *sig, uint32_t label,
                           int64_t *y, int subtract_own) {
  for (int64_t j = g->pp[v]; j < g->pp[v + 1]; j++) {
    y[j - g->pp[v]] = map_get(sig, label, g->ps[j]) - (subtract_own ? g->pk[j] : 0);
  }
}

/* Decide the move of unit v against the current state.  Returns the target label, or
 * NONE_LABEL to stay; *to_empty set when the target is a new empty community. */
static uint32_t decide_move(const ctx_t *cx, const level_t *g, int64_t v, const uint32_t *P,
                            const map_t *sig, acc_t *buf, int64_t *y, int *to_empty) {
  int64_t nc = gather(g, v, P, NULL, 0, buf);
  uint32_t D = P[v];
  int m = (int)(g->pp[v + 1] - g->pp[v]);
  const int32_t *ps = g->ps + g->pp[v];
  const int64_t *pk = g->pk + g->pp[v];
  int64_t wD = 0;
  for (int64_t i = 0; i < nc; i++) if (buf[i].lab == D) wD = buf[i].w;
  gval_t gD, best, cur;
  profile_values(g, v, sig, D, y, 1);
  gain_value(&cx->cf, wD, m, ps, pk, y, &gD);
  best.big = 0; best.small = 0;            /* empty community: gain 0, label +infinity */
  int best_empty = 1; uint32_t best_lab = NONE_LABEL;
  for (int64_t i = 0; i < nc; i++) {
    uint32_t C = buf[i].lab;
    if (C == D) continue;
    profile_values(g, v, sig, C, y, 0);
    gain_value(&cx->cf, buf[i].w, m, ps, pk, y, &cur);
    int c = gval_cmp(&cur, &best);
    if (c > 0 || (c == 0 && best_empty)) { best = cur; best_empty = 0; best_lab = C; }
  }
  *to_empty = 0;
  if (gval_cmp(&best, &gD) > 0) {
    if (best_empty) { *to_empty = 1; return NONE_LABEL - 1; }
    return best_lab;
  }
  return NONE_LABEL;
}

static int64_t max_degree(const level_t *g) {
  int64_t md = 0;
  for (int64_t v = 0; v < g->n; v++) if (g->rp[v + 1] - g->rp[v] > md) md = g->rp[v + 1] - g->rp[v];
  return md;
}
static int64_t max_profile(const level_t *g) {
  int64_t md = 0;
  for (int64_t v = 0; v < g->n; v++) if (g->pp[v + 1] - g->pp[v] > md) md = g->pp[v + 1] - g->pp[v];
  return md;
}

static void build_sigma(const level_t *g, const uint32_t *P, map_t *sig) {
  map_init(sig, g->pp[g->n]);
  for (int64_t v = 0; v < g->n; v++)
    for (int64_t j = g->pp[v]; j < g->pp[v + 1]; j++) map_add(sig, P[v], g->ps[j], g->pk[j]);
}

static int32_t local_move(const ctx_t *cx, const level_t *g, const int32_t *colour, int32_t ncol,
                          uint32_t *P, int max_sweeps, orc_stats *st, map_t *sig_out) {
  int64_t n = g->n;
  map_t sig; build_sigma(g, P, &sig);
  /* colour buckets, ids ascending inside each colour */
  int64_t *bp = calloc(ncol + 1, sizeof(int64_t)), *bn = malloc((n ? n : 1) * sizeof(int64_t));
  for (int64_t v = 0; v < n; v++) bp[colour[v] + 1]++;
  for (int32_t c = 0; c < ncol; c++) bp[c + 1] += bp[c];
  int64_t *fill = malloc((ncol + 1) * sizeof(int64_t));
  memcpy(fill, bp, (ncol + 1) * sizeof(int64_t));
  for (int64_t v = 0; v < n; v++) bn[fill[colour[v]]++] = v;
  free(fill);
  uint32_t *tgt = malloc((n ? n : 1) * sizeof(uint32_t));
  int64_t md = max_degree(g) + 1, mp = max_profile(g) + 1;
  int32_t sweeps = 0;
  for (int t = 0; t < max_sweeps; t++) {
    int64_t moved = 0;
    sweeps++;
    for (int32_t c = 0; c < ncol; c++) {
      int64_t lo = bp[c], hi = bp[c + 1];
#pragma omp parallel
      {
        acc_t *buf = malloc(md * sizeof(acc_t));
        int64_t *y = malloc(mp * sizeof(int64_t));
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = lo; i < hi; i++) {
          int64_t v = bn[i]; int te;
          uint32_t r = decide_move(cx, g, v, P, &sig, buf, y, &te);
          tgt[v] = te ? (uint32_t)((uint64_t)n * (1 + t) + (uint64_t)v) : r;
        }
        free(buf); free(y);
      }
      for (int64_t i = lo; i < hi; i++) {
        int64_t v = bn[i];
        if (tgt[v] == NONE_LABEL) continue;
        uint32_t D = P[v], C = tgt[v];
        for (int64_t j = g->pp[v]; j < g->pp[v + 1]; j++) {
          map_add(&sig, D, g->ps[j], -g->pk[j]);
          map_add(&sig, C, g->ps[j], g->pk[j]);
        }
        P[v] = C;
        moved++;
      }
    }
    st->sweeps++; st->moves += moved;
    if (moved == 0) break;
    if (t == max_sweeps - 1) st->sweep_cap_hits++;
  }
  free(bp); free(bn); free(tgt);
  if (sig_out) *sig_out = sig; else map_free(&sig);
  return sweeps;
}

/* ------------------------------------------------------------------ refinement */
/* Well-connectedness of a set X inside its community K (Section 3.2, after Traag et al.):
 *   ext(X) >= b * sum_s gamma^(s) Sigma_{X,s} (Sigma_{K,s} - Sigma_{X,s}) / S_s,
 * evaluated exactly as the sign of the gain form above with W = ext, k = x_s, y = K_s - x_s. */
static int well_connected(const coef_t *cf, int64_t ext, int m, const int32_t *sl, const int64_t *xs,
                          const int64_t *ks) {
  int64_t *prod = malloc((m ? m : 1) * sizeof(int64_t));
  for (int j = 0; j < m; j++) prod[j] = ks[j] - xs[j];
  gval_t g;
  gain_value(cf, ext, m, sl, xs, prod, &g);
  free(prod);
  return gval_sign(&g) >= 0;
}

static void set_profile(const map_t *sr, uint32_t T, uint64_t mask, int32_t *sl, int64_t *xs, int *m) {
  int k = 0;
  for (int s = 0; s < 64; s++) if (mask >> s & 1) {
    int64_t x = map_get(sr, T, s);
    if (x) { sl[k] = s; xs[k] = x; k++; }
  }
  *m = k;
}

static int64_t refine(const ctx_t *cx, const level_t *g, const uint32_t *P, const map_t *sigP,
                      const uint32_t *local, uint64_t seed, int it, int lvl, uint32_t *R, orc_stats *st,
                      int64_t *ext_out, char *wc_out) {
  int64_t n = g->n;
  map_t sr; map_init(&sr, g->pp[n]);
  int64_t *ext = calloc(n ? n : 1, sizeof(int64_t));
  uint64_t *mask = calloc(n ? n : 1, sizeof(uint64_t));
  char *single = malloc(n ? n : 1), *active = malloc(n ? n : 1), *wcT = malloc(n ? n : 1);
  char *elig = calloc(n ? n : 1, 1), *changed = calloc(n ? n : 1, 1);
  uint32_t *prop = malloc((n ? n : 1) * sizeof(uint32_t));
  int64_t *propw = calloc(n ? n : 1, sizeof(int64_t));
  uint64_t *pri = malloc((n ? n : 1) * sizeof(uint64_t));
  int32_t sl[MAX_SLICES]; int64_t xs[MAX_SLICES], ks[MAX_SLICES];
  for (int64_t v = 0; v < n; v++) {
    R[v] = (uint32_t)v;
    for (int64_t j = g->pp[v]; j < g->pp[v + 1]; j++) { map_add(&sr, (uint32_t)v, g->ps[j], g->pk[j]); mask[v] |= 1ULL << g->ps[j]; }
    for (int64_t e = g->rp[v]; e < g->rp[v + 1]; e++) if (P[g->col[e]] == P[v]) ext[v] += g->w[e];
    pri[v] = orc_priority(seed, it, lvl, 1, local[v]);
  }
  for (int64_t v = 0; v < n; v++) {
    int m; set_profile(&sr, (uint32_t)v, mask[v], sl, xs, &m);
    for (int j = 0; j < m; j++) ks[j] = map_get(sigP, P[v], sl[j]);
    wcT[v] = (char)well_connected(&cx->cf, ext[v], m, sl, xs, ks);
    single[v] = 1; active[v] = wcT[v];
  }
  int64_t md = max_degree(g) + 1, mp = max_profile(g) + 1;
  int64_t merges = 0;
  for (int round = 0; round < MAX_REFINE_ROUNDS; round++) {
    int any = 0;
#pragma omp parallel
    {
      acc_t *buf = malloc(md * sizeof(acc_t));
      int64_t *y = malloc(mp * sizeof(int64_t));
#pragma omp for schedule(dynamic, 256)
      for (int64_t v = 0; v < n; v++) {
        prop[v] = NONE_LABEL;
        if (!active[v]) continue;
        int64_t nc = gather(g, v, R, P, P[v], buf);
        int m = (int)(g->pp[v + 1] - g->pp[v]);
        gval_t best, cur; int have = 0; uint32_t bl = NONE_LABEL; int64_t bw = 0;
        for (int64_t i = 0; i < nc; i++) {
          uint32_t T = buf[i].lab;
          if (!wcT[T]) continue;
          for (int64_t j = g->pp[v]; j < g->pp[v + 1]; j++) y[j - g->pp[v]] = map_get(&sr, T, g->ps[j]);
          gain_value(&cx->cf, buf[i].w, m, g->ps + g->pp[v], g->pk + g->pp[v], y, &cur);
          if (gval_sign(&cur) <= 0) continue;
          if (!have || gval_cmp(&cur, &best) > 0) { best = cur; bl = T; bw = buf[i].w; have = 1; }
        }
        if (have) { prop[v] = bl; propw[v] = bw; }
      }
      free(buf); free(y);
    }
    for (int64_t v = 0; v < n; v++) if (active[v] && prop[v] == NONE_LABEL) active[v] = 0;
    /* A proposer merges when its target sub-community keeps all its members this round:
     *   (a) the target's founder does not propose (a larger sub-community never proposes), or
     *   (b) the proposer outranks every proposing neighbour of its community and the target's
     *       founder proposes to a target that is itself proposing (so the founder stays). */
    for (int64_t v = 0; v < n; v++) {
      elig[v] = 0;
      if (prop[v] == NONE_LABEL) continue;
      uint32_t T = prop[v];
      if (prop[T] == NONE_LABEL) { elig[v] = 1; any = 1; continue; }
      if (prop[prop[T]] == NONE_LABEL) continue;
      int ok = 1;
      for (int64_t e = g->rp[v]; e < g->rp[v + 1] && ok; e++) {
        int32_t u = g->col[e];
        if (P[u] != P[v] || prop[u] == NONE_LABEL) continue;
        if (pri[u] > pri[v] || (pri[u] == pri[v] && u > v)) ok = 0;
      }
      elig[v] = (char)ok;
      any |= ok;
    }
    st->refine_rounds++;
    if (!any) break;
    for (int64_t v = 0; v < n; v++) {
      if (!elig[v]) continue;
      uint32_t T = prop[v];
      /* edges to co-joiners of the same target become internal too */
      int64_t corr = 0;
      for (int64_t e = g->rp[v]; e < g->rp[v + 1]; e++) {
        int32_t x = g->col[e];
        if (elig[x] && prop[x] == T) corr += g->w[e];
      }
      R[v] = T;
      single[v] = 0; active[v] = 0; single[T] = 0; active[T] = 0;
      ext[T] += ext[v] - 2 * propw[v] - corr;
      for (int64_t j = g->pp[v]; j < g->pp[v + 1]; j++) map_add(&sr, T, g->ps[j], g->pk[j]);
      mask[T] |= mask[v];
      changed[T] = 1;
      merges++;
    }
    for (int64_t T = 0; T < n; T++) if (changed[T]) {
      changed[T] = 0;
      int m; set_profile(&sr, (uint32_t)T, mask[T], sl, xs, &m);
      for (int j = 0; j < m; j++) ks[j] = map_get(sigP, P[T], sl[j]);
      wcT[T] = (char)well_connected(&cx->cf, ext[T], m, sl, xs, ks);
    }
  }
  st->merges += merges;
  if (ext_out) memcpy(ext_out, ext, n * sizeof(int64_t));
  if (wc_out) memcpy(wc_out, wcT, n);
  map_free(&sr); free(ext); free(mask); free(single); free(active); free(wcT); free(elig); free(changed);
  free(prop); free(propw); free(pri);
  return merges;
}

/* ------------------------------------------------------------------ aggregation */
typedef struct { uint32_t a, b; int64_t w; } edge_t;
static int edge_cmp(const void *x, const void *y) {
  const edge_t *p = x, *q = y;
  if (p->a != q->a) return p->a < q->a ? -1 : 1;
  if (p->b != q->b) return p->b < q->b ? -1 : 1;
  return 0;
}

static void aggregate(const level_t *g, const uint32_t *R, const uint32_t *P, level_t *ng,
                      uint32_t *Pnext, int64_t *map0, int64_t n0) {
  int64_t n = g->n;
  uint32_t *r = malloc((n ? n : 1) * sizeof(uint32_t));
  int64_t n2 = canon(n, R, r);
  edge_t *e = malloc((g->nnz ? g->nnz : 1) * sizeof(edge_t));
  int64_t m = 0;
  for (int64_t v = 0; v < n; v++)
    for (int64_t k = g->rp[v]; k < g->rp[v + 1]; k++) {
      uint32_t a = r[v], b = r[g->col[k]];
      if (a != b) e[m++] = (edge_t){a, b, g->w[k]};
    }
  qsort(e, m, sizeof(edge_t), edge_cmp);
  int64_t u = 0;
  for (int64_t k = 0; k < m; k++) {
    if (u > 0 && e[u - 1].a == e[k].a && e[u - 1].b == e[k].b) e[u - 1].w += e[k].w;
    else e[u++] = e[k];
  }
  ng->n = n2; ng->nnz = u;
  ng->rp = calloc(n2 + 1, sizeof(int64_t)); ng->col = malloc((u ? u : 1) * 4); ng->w = malloc((u ? u : 1) * 8);
  for (int64_t k = 0; k < u; k++) { ng->rp[e[k].a + 1]++; ng->col[k] = (int32_t)e[k].b; ng->w[k] = e[k].w; }
  for (int64_t v = 0; v < n2; v++) ng->rp[v + 1] += ng->rp[v];
  free(e);
  /* profiles */
  int64_t np = g->pp[n];
  edge_t *pe = malloc((np ? np : 1) * sizeof(edge_t));
  m = 0;
  for (int64_t v = 0; v < n; v++)
    for (int64_t j = g->pp[v]; j < g->pp[v + 1]; j++) pe[m++] = (edge_t){r[v], (uint32_t)g->ps[j], g->pk[j]};
  qsort(pe, m, sizeof(edge_t), edge_cmp);
  u = 0;
  for (int64_t k = 0; k < m; k++) {
    if (u > 0 && pe[u - 1].a == pe[k].a && pe[u - 1].b == pe[k].b) pe[u - 1].w += pe[k].w;
    else pe[u++] = pe[k];
  }
  ng->pp = calloc(n2 + 1, sizeof(int64_t)); ng->ps = malloc((u ? u : 1) * 4); ng->pk = malloc((u ? u : 1) * 8);
  for (int64_t k = 0; k < u; k++) { ng->pp[pe[k].a + 1]++; ng->ps[k] = (int32_t)pe[k].b; ng->pk[k] = pe[k].w; }
  for (int64_t v = 0; v < n2; v++) ng->pp[v + 1] += ng->pp[v];
  free(pe);
  uint32_t *Pr = malloc((n2 ? n2 : 1) * sizeof(uint32_t));
  for (int64_t v = 0; v < n; v++) Pr[r[v]] = P[v];
  canon(n2, Pr, Pnext);
  free(Pr);
  for (int64_t i = 0; i < n0; i++) map0[i] = r[map0[i]];
  free(r);
}

/* ------------------------------------------------------------------ split and output labels */
/* Connected components of the level-0 supra-graph restricted to entries inside a community;
 * components numbered in order of their smallest supra-node.  Returns the count. */
static int64_t split_components(const level_t *g0, const uint32_t *Pf, int32_t *out) {
  int64_t n = g0->n;
  for (int64_t v = 0; v < n; v++) out[v] = -1;
  int64_t *stack = malloc((n ? n : 1) * sizeof(int64_t));
  int64_t c = 0;
  for (int64_t v = 0; v < n; v++) {
    if (out[v] >= 0) continue;
    int64_t top = 0; stack[top++] = v; out[v] = (int32_t)c;
    while (top) {
      int64_t x = stack[--top];
      for (int64_t e = g0->rp[x]; e < g0->rp[x + 1]; e++) {
        int32_t y = g0->col[e];
        if (out[y] < 0 && Pf[y] == Pf[x]) { out[y] = (int32_t)c; stack[top++] = y; }
      }
    }
    c++;
  }
  free(stack);
  return c;
}

/* ------------------------------------------------------------------ Q components */
/* comps[0..T-1] = W_s (intra weight inside communities, both directions, unscaled),
 * comps[T..2T-1] = SS_s = sum_C Sigma_{C,s}^2, comps[2T..3T-1] = 2m_s,
 * comps[3T] = I = sum of c_sr over the ordered coupled copy pairs sharing a community. */
int orc_q_components(const orc_graph *G, const int32_t *memb, int64_t *comps) {
  int32_t N = G->N, T = G->T;
  const level_t *g = &G->g0;
  for (int i = 0; i < 3 * T + 1; i++) comps[i] = 0;
  for (int64_t v = 0; v < g->n; v++) {
    int32_t s = (int32_t)(v / N);
    for (int64_t e = g->rp[v]; e < g->rp[v + 1]; e++)
      if (G->raw[e] && memb[g->col[e]] == memb[v]) comps[s] += G->raw[e];
  }
  map_t sig; map_init(&sig, g->n);
  for (int64_t v = 0; v < g->n; v++)
    for (int64_t j = g->pp[v]; j < g->pp[v + 1]; j++) map_add(&sig, (uint32_t)memb[v], g->ps[j], g->pk[j]);
  for (uint64_t h = 0; h < sig.cap; h++) if (sig.key[h] != MAP_EMPTY) {
    int32_t s = (int32_t)(sig.key[h] & 0xff);
    comps[T + s] += sig.val[h] * sig.val[h];
  }
  map_free(&sig);
  for (int32_t s = 0; s < T; s++) comps[2 * T + s] = G->twom[s];
  int64_t I = 0;
  for (int32_t s = 0; s < T; s++)
    for (int32_t r = 0; r < T; r++)
      for (int32_t i = 0; i < N; i++)
        if (memb[(int64_t)s * N + i] == memb[(int64_t)r * N + i]) I += coupled(G, i, s, r);
  comps[3 * T] = I;
  return ORC_OK;
}

/* Components of the global modularity: comps[0..T-1] = W_s as above, comps[T] = the sum over
 * communities of the squared scaled supra-degree sum (sum_C (sum_{v in C} kappa'_v)^2, with
 * kappa' = b * (intra degree) + a * (coupling count)), comps[T+1..2T-1] = 0, comps[2T..3T-1] =
 * 2m_s, comps[3T] = I. */
/* CPM node weight of supra-node v: 1, or 0 for a copy without edges when only present copies
 * are supra-nodes (they are then left out of the graph entirely). */
static int cpm_weight(const orc_graph *G, int64_t v) {
  return !G->present_only || G->present[v];
}

/* Components of the multislice CPM (node weight 1 per supra-node): as orc_q_components with
 * comps[T..2T-1] = sum over communities of the squared number of their supra-nodes in slice s. */
int orc_q_components_cpm(const orc_graph *G, const int32_t *memb, int64_t *comps) {
  int32_t N = G->N, T = G->T;
  const level_t *g = &G->g0;
  orc_q_components(G, memb, comps);
  map_t sig; map_init(&sig, g->n);
  for (int64_t v = 0; v < g->n; v++)
    if (cpm_weight(G, v)) map_add(&sig, (uint32_t)memb[v], (int32_t)(v / N), 1);
  for (int32_t s = T; s < 2 * T; s++) comps[s] = 0;
  for (uint64_t h = 0; h < sig.cap; h++) if (sig.key[h] != MAP_EMPTY) {
    int32_t s = (int32_t)(sig.key[h] & 0xff);
    comps[T + s] += sig.val[h] * sig.val[h];
  }
  map_free(&sig);
  return ORC_OK;
}

int orc_q_components_global(const orc_graph *G, const int32_t *memb, int64_t *comps) {
  int32_t T = G->T;
  const level_t *g = &G->g0;
  orc_q_components(G, memb, comps);
  map_t sig; map_init(&sig, g->n);
  for (int64_t v = 0; v < g->n; v++) {
    int64_t kap = 0;
    for (int64_t e = g->rp[v]; e < g->rp[v + 1]; e++) kap += g->w[e];
    if (kap) map_add(&sig, (uint32_t)memb[v], 0, kap);
  }
  i128 ss = 0;
  for (uint64_t h = 0; h < sig.cap; h++) if (sig.key[h] != MAP_EMPTY) ss += (i128)sig.val[h] * sig.val[h];
  map_free(&sig);
  for (int32_t s = T; s < 2 * T; s++) comps[s] = 0;
  comps[T] = (int64_t)ss;
  return ORC_OK;
}

/* ------------------------------------------------------------------ driver */
static int level_copy(const level_t *src, level_t *dst) {
  int64_t n = src->n, m = src->nnz, np = src->pp[n];
  dst->n = n; dst->nnz = m;
  dst->rp = dupmem(src->rp, (n + 1) * 8); dst->col = dupmem(src->col, m * 4); dst->w = dupmem(src->w, m * 8);
  dst->pp = dupmem(src->pp, (n + 1) * 8); dst->ps = dupmem(src->ps, np * 4); dst->pk = dupmem(src->pk, np * 8);
  return ORC_OK;
}

/* The global null model (Eq. 5 on the supra-graph): every unit's profile is the single
 * entry (slice 0, kappa'_v) with kappa'_v its scaled supra-degree (intra and coupling
 * weights), and the one denominator is 2mu' = sum of kappa'.  With the coupling denominator
 * b folded into kappa', the comparison value q*W*2mu' - p*kappa'*Sigma' orders targets as
 * the change of the global modularity does. */
static level_t global_level(const level_t *g0, int64_t *two_mu) {
  level_t g; level_copy(g0, &g);
  free(g.pp); free(g.ps); free(g.pk);
  int64_t n = g.n, np = 0;
  int64_t *kap = calloc(n ? n : 1, sizeof(int64_t));
  *two_mu = 0;
  for (int64_t v = 0; v < n; v++) {
    for (int64_t e = g.rp[v]; e < g.rp[v + 1]; e++) kap[v] += g.w[e];
    np += kap[v] > 0;
    *two_mu += kap[v];
  }
  g.pp = calloc(n + 1, sizeof(int64_t)); g.ps = malloc((np ? np : 1) * sizeof(int32_t));
  g.pk = malloc((np ? np : 1) * sizeof(int64_t));
  int64_t q = 0;
  for (int64_t v = 0; v < n; v++) {
    if (kap[v] > 0) { g.ps[q] = 0; g.pk[q] = kap[v]; q++; }
    g.pp[v + 1] = q;
  }
  free(kap);
  return g;
}

/* The multislice CPM (the Constant Potts Model of Traag et al. with the slices coupled as in
 * Eq. 6): the null term gamma^(s) k_i k_j / 2m_s of Eq. 6 becomes gamma^(s) n_i n_j with node
 * weight n = 1 per supra-node, so every supra-node's profile is the single entry (its slice, 1)
 * and every slice's denominator is 1. */
static level_t cpm_level(const orc_graph *G) {
  level_t g; level_copy(&G->g0, &g);
  free(g.pp); free(g.ps); free(g.pk);
  int64_t n = g.n, q = 0;
  g.pp = calloc(n + 1, sizeof(int64_t)); g.ps = malloc((n ? n : 1) * sizeof(int32_t));
  g.pk = malloc((n ? n : 1) * sizeof(int64_t));
  for (int64_t v = 0; v < n; v++) {
    if (cpm_weight(G, v)) { g.ps[q] = (int32_t)(v / G->N); g.pk[q] = 1; q++; }
    g.pp[v + 1] = q;
  }
  return g;
}

/* null_model: 0 Q_MS of Eq. 6, 1 the global modularity of the supra-graph, 2 the multislice
 * CPM.  gamma_slices (NULL: gamma_num/gamma_den in every slice) holds T pairs (num, den) of
 * positive per-slice resolutions gamma^(s) (not with the global null model).  initial (NULL:
 * singletons) is the start partition of the first iteration, labels in [0, N*T), taken in its
 * canonical form (labels by first appearance). */
int orc_leiden(const orc_graph *G, int64_t gamma_num, int64_t gamma_den,
               const int64_t *gamma_slices, const int32_t *initial, int32_t max_levels,
               int32_t max_iterations, int32_t max_sweeps, uint64_t seed, int32_t null_model,
               int32_t *membership, int64_t *comps, orc_stats *st) {
  if (max_levels < 1) return ORC_EINVAL;
  if (null_model < 0 || null_model > 2) return ORC_EINVAL;
  if (gamma_slices && null_model == 1) return ORC_EINVAL;
  const int64_t n0 = G->g0.n;
  if (initial)
    for (int64_t v = 0; v < n0; v++) if (initial[v] < 0 || initial[v] >= n0) return ORC_EINVAL;
  ctx_t cx; cx.G = G;
  int64_t S[MAX_SLICES], gp[MAX_SLICES], gq[MAX_SLICES];
  for (int s = 0; s < G->T; s++) {
    int64_t a = gamma_slices ? gamma_slices[2 * s] : gamma_num;
    int64_t d = gamma_slices ? gamma_slices[2 * s + 1] : gamma_den;
    if (a < 0 || d < 1 || (gamma_slices && a == 0)) return ORC_EINVAL;
    if (a >= ((int64_t)1 << 31) || d >= ((int64_t)1 << 31)) return ORC_EOVERFLOW;
    int64_t gg = a ? gcd64(a, d) : d;
    gp[s] = a / gg; gq[s] = d / gg;
    S[s] = null_model == 2 ? 1 : (G->twom[s] > 0 ? G->twom[s] : 1);
  }
  cx.cf.gp = gp; cx.cf.gq = gq; cx.cf.b = G->b; cx.cf.S = S;
  level_t gglob; memset(&gglob, 0, sizeof(gglob));
  const level_t *base = &G->g0;
  if (null_model == 1) {
    int64_t two_mu = 0;
    gglob = global_level(&G->g0, &two_mu);
    /* head-room of the exact values: 2mu' < 2^31 and max(p, q) * 2mu'^2 < 2^62 */
    int64_t pq = gp[0] > gq[0] ? gp[0] : gq[0];
    if (two_mu >= ((int64_t)1 << 31) || (i128)pq * two_mu * two_mu >= ((i128)1 << 62)) {
      level_free(&gglob);
      return ORC_EOVERFLOW;
    }
    S[0] = two_mu > 0 ? two_mu : 1;
    cx.cf.b = 1;
    base = &gglob;
  } else if (null_model == 2) {
    gglob = cpm_level(G);
    base = &gglob;
  }
  if (max_sweeps <= 0) max_sweeps = DEFAULT_SWEEPS;
  int iters = max_iterations > 0 ? max_iterations : MAX_ITER_CAP;
  if (iters > MAX_ITER_CAP) iters = MAX_ITER_CAP;
  memset(st, 0, sizeof(*st));
  int32_t *Pcur = malloc((n0 ? n0 : 1) * sizeof(int32_t));
  if (initial) {
    uint32_t *c0 = malloc((n0 ? n0 : 1) * sizeof(uint32_t));
    canon(n0, (const uint32_t *)initial, c0);
    for (int64_t v = 0; v < n0; v++) Pcur[v] = (int32_t)c0[v];
    free(c0);
  } else {
    for (int64_t v = 0; v < n0; v++) Pcur[v] = (int32_t)v;
  }
  int64_t *map0 = malloc(n0 * sizeof(int64_t));
  uint32_t *Pflat = malloc(n0 * sizeof(uint32_t));
  int32_t *Pnew = malloc(n0 * sizeof(int32_t));
  for (int it = 0; it < iters; it++) {
    level_t g; level_copy(base, &g);
    for (int64_t v = 0; v < n0; v++) map0[v] = v;
    uint32_t *P = malloc(n0 * sizeof(uint32_t));
    for (int64_t v = 0; v < n0; v++) P[v] = (uint32_t)Pcur[v];
    uint32_t *Pc = malloc(n0 * sizeof(uint32_t));
    canon(n0, P, Pc); free(P); P = Pc;
    int lvl;
    for (lvl = 0; lvl < max_levels; lvl++) {
      int64_t n = g.n;
      uint32_t *local = malloc((n ? n : 1) * sizeof(uint32_t));
      for (int64_t v = 0; v < n; v++) local[v] = (uint32_t)v;
      int32_t *colour = malloc((n ? n : 1) * sizeof(int32_t));
      int32_t ncol = colour_units(&g, local, seed, it, lvl, colour);
      if (it == 0 && lvl == 0) st->colours_first = ncol;
      trace_level_t *tr = trace_push(it, lvl, &g, map0, n0);
      if (tr) { tr->colour = dupmem(colour, n * 4); tr->p_in = dupmem(P, n * 4); tr->ncol = ncol; }
      map_t sig;
      int32_t sw = local_move(&cx, &g, colour, ncol, P, max_sweeps, st, &sig);
      if (tr) { tr->p_lm = dupmem(P, n * 4); tr->sweeps = sw; }
      uint32_t *tmp = malloc((n ? n : 1) * sizeof(uint32_t));
      int64_t ncomm = canon(n, P, tmp);
      free(tmp);
      free(colour);
      if (ncomm == n || lvl == max_levels - 1) { map_free(&sig); free(local); break; }
      uint32_t *R = malloc((n ? n : 1) * sizeof(uint32_t));
      int64_t *ext_t = tr ? malloc((n ? n : 1) * sizeof(int64_t)) : NULL;
      char *wc_t = tr ? malloc(n ? n : 1) : NULL;
      refine(&cx, &g, P, &sig, local, seed, it, lvl, R, st, ext_t, wc_t);
      map_free(&sig); free(local);
      if (tr) { tr->r = dupmem(R, n * 4); tr->has_r = 1; tr->ext = ext_t; tr->wc = wc_t; }
      uint32_t *tmp2 = malloc((n ? n : 1) * sizeof(uint32_t));
      int64_t nref = canon(n, R, tmp2);
      free(tmp2);
      if (nref == n) { free(R); break; }
      level_t ng; memset(&ng, 0, sizeof(ng));
      uint32_t *Pn = malloc((nref ? nref : 1) * sizeof(uint32_t));
      aggregate(&g, R, P, &ng, Pn, map0, n0);
      free(R); free(P); P = Pn;
      level_free(&g); g = ng;
    }
    if (lvl + 1 > st->levels_run) st->levels_run = lvl + 1;
    for (int64_t v = 0; v < n0; v++) Pflat[v] = P[map0[v]];
    free(P);
    level_free(&g);
    int64_t ncomp = split_components(&G->g0, Pflat, Pnew);
    uint32_t *tmp3 = malloc(n0 * sizeof(uint32_t));
    int64_t nflat = canon(n0, Pflat, tmp3);
    free(tmp3);
    st->splits += ncomp - nflat;
    st->iterations_run = it + 1;
    int same = memcmp(Pnew, Pcur, n0 * sizeof(int32_t)) == 0;
    memcpy(Pcur, Pnew, n0 * sizeof(int32_t));
    st->n_communities = (int32_t)ncomp;
    if (same) break;
  }
  memcpy(membership, Pcur, n0 * sizeof(int32_t));
  if (null_model == 1) orc_q_components_global(G, Pcur, comps);
  else if (null_model == 2) orc_q_components_cpm(G, Pcur, comps);
  else orc_q_components(G, Pcur, comps);
  free(Pcur); free(map0); free(Pflat); free(Pnew);
  if (null_model != 0) level_free(&gglob);
  return ORC_OK;
}

/* Exact comparison helper exposed for tests: sign of  q*W*Pi - p*b*sum_j k_j y_j Pi/S_j. */
int orc_gain_sign(int64_t p, int64_t q, int64_t b, const int64_t *S, int64_t W, int m,
                  const int32_t *ps, const int64_t *pk, const int64_t *y) {
  int64_t gp[MAX_SLICES], gq[MAX_SLICES];
  for (int s = 0; s < MAX_SLICES; s++) { gp[s] = p; gq[s] = q; }
  coef_t cf = {gp, gq, b, S};
  gval_t g; gain_value(&cf, W, m, ps, pk, y, &g);
  return gval_sign(&g);
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
