// Host-side checks and exact arithmetic of the C ABI: input validation, parameter reduction,
// the int64 head-room preconditions, the exact reduced fraction Q of Eq. 6 from its integer
// components, and the thread-local error text.  No HIP: this file also builds for the host
// alone (the sanitizer test compiles it with g++).
#include "host.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

using namespace mslm;

namespace {

thread_local std::string g_err;

mslm_status fail(mslm_status s, const std::string &m) {
  g_err = m;
  return s;
}

int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

constexpr int64_t kLim31 = (int64_t)1 << 31;

mslm_status check_fraction(int64_t num, int64_t den, const char *what) {
  if (num < 0 || den < 1) return fail(MSLM_EINVAL, std::string(what) + ": need numerator >= 0, denominator >= 1");
  if (num >= kLim31 || den >= kLim31) return fail(MSLM_EOVERFLOW, std::string(what) + ": numerator and denominator must be below 2^31");
  return MSLM_OK;
}

// Shape checks that need no device and no edge data.
mslm_status check_desc_shape(const mslm_graph_desc *d) {
  if (!d) return fail(MSLM_EINVAL, "desc is NULL");
  if (d->n_nodes < 1 || d->n_slices < 1) return fail(MSLM_EINVAL, "need n_nodes >= 1 and n_slices >= 1");
  if (d->n_slices > 64) return fail(MSLM_EUNSUPPORTED, "at most 64 snapshots are supported");
  if (!d->slice_offsets) return fail(MSLM_EINVAL, "slice_offsets is NULL");
  if (d->slice_offsets[0] != 0) return fail(MSLM_EINVAL, "slice_offsets[0] must be 0");
  for (int s = 0; s < d->n_slices; s++)
    if (d->slice_offsets[s + 1] < d->slice_offsets[s]) return fail(MSLM_EINVAL, "slice_offsets must be non-decreasing");
  const int64_t E = d->slice_offsets[d->n_slices];
  if (E > 0 && (!d->src || !d->dst)) return fail(MSLM_EINVAL, "src/dst are NULL");
  const int64_t n = (int64_t)d->n_nodes * d->n_slices;
  if ((uint64_t)n * 33u >= 0xffffffffull) return fail(MSLM_EUNSUPPORTED, "N*T*33 must stay below 2^32");
  if (2 * E + (int64_t)d->n_nodes * d->n_slices * (d->n_slices - 1) >= ((int64_t)1 << 40))
    return fail(MSLM_EUNSUPPORTED, "too many edges");
  mslm_status s = check_fraction(d->omega_num, d->omega_den, "omega");
  if (s != MSLM_OK) return s;
  if (d->coupling) {
    const int T = d->n_slices;
    for (int a = 0; a < T; a++)
      for (int b = 0; b < T; b++) {
        const int32_t c = d->coupling[a * T + b];
        if (c < 0 || c >= (1 << 16))
          return fail(MSLM_EINVAL, "coupling: entries must lie in [0, 2^16)");
        if (a == b && c != 0) return fail(MSLM_EINVAL, "coupling: the diagonal must be 0");
        if (c != d->coupling[b * T + a]) return fail(MSLM_EINVAL, "coupling: must be symmetric");
      }
  }
  return MSLM_OK;
}

// Edge checks on host inputs (device inputs are checked by a kernel during the build).
mslm_status check_desc_edges(const mslm_graph_desc *d) {
  if (d->flags & MSLM_INPUT_ON_DEVICE) return MSLM_OK;
  const int64_t E = d->slice_offsets[d->n_slices];
  for (int64_t e = 0; e < E; e++) {
    int32_t u = d->src[e], x = d->dst[e];
    if (u < 0 || u >= d->n_nodes || x < 0 || x >= d->n_nodes)
      return fail(MSLM_EINVAL, "edge " + std::to_string(e) + ": node id out of range");
    if (u == x) return fail(MSLM_EINVAL, "edge " + std::to_string(e) + ": self-loop");
    if (d->weight && d->weight[e] < 1) return fail(MSLM_EINVAL, "edge " + std::to_string(e) + ": weight < 1");
  }
  return MSLM_OK;
}

mslm_status make_spec(const mslm_params *p, int64_t def_on, int64_t def_od, SolveSpec &sp) {
  if (!p) return fail(MSLM_EINVAL, "params is NULL");
  mslm_status s = check_fraction(p->gamma_num, p->gamma_den, "gamma");
  if (s != MSLM_OK) return s;
  int64_t on = def_on, od = def_od;
  if (p->omega_den != 0) {
    s = check_fraction(p->omega_num, p->omega_den, "omega");
    if (s != MSLM_OK) return s;
    on = p->omega_num;
    od = p->omega_den;
  }
  if (p->max_levels < 1) return fail(MSLM_EINVAL, "max_levels must be >= 1");
  if (p->max_levels > 1024) return fail(MSLM_EINVAL, "max_levels must be <= 1024");
  int64_t gg = p->gamma_num ? gcd64(p->gamma_num, p->gamma_den) : p->gamma_den;
  sp.p = p->gamma_num / gg;
  sp.q = p->gamma_den / gg;
  int64_t go = on ? gcd64(on, od) : od;
  sp.a = on / go;
  sp.b = od / go;
  sp.max_levels = p->max_levels;
  sp.max_iterations = p->max_iterations > 0 ? std::min(p->max_iterations, 32) : 32;
  sp.max_sweeps = p->max_sweeps > 0 ? p->max_sweeps : 32;
  if (sp.max_sweeps > 32) return fail(MSLM_EINVAL, "max_sweeps must be <= 32");
  sp.seed = p->seed;
  if (p->null_model != MSLM_NULL_MULTISLICE && p->null_model != MSLM_NULL_GLOBAL &&
      p->null_model != MSLM_NULL_CPM)
    return fail(MSLM_EINVAL, "null_model must be MSLM_NULL_MULTISLICE, MSLM_NULL_GLOBAL or "
                             "MSLM_NULL_CPM");
  sp.null_model = p->null_model;
  sp.pe = sp.p;
  sp.qe = sp.q;
  sp.gn.clear();
  sp.gd.clear();
  sp.smul.clear();
  sp.init.clear();
  return MSLM_OK;
}

typedef __int128 i128h;

// lcm of two positive values, false when it reaches `limit`
bool lcm_below(int64_t x, int64_t y, int64_t limit, int64_t &out) {
  const i128h l = (i128h)(x / gcd64(x, y)) * y;
  if (l >= limit) return false;
  out = (int64_t)l;
  return true;
}

// Per-slice resolutions: reduce them and fold them into (pe, qe, smul) as SolveSpec states.
mslm_status slice_resolutions(const int64_t *gs, int32_t T, SolveSpec &sp) {
  if (sp.null_model == MSLM_NULL_GLOBAL)
    return fail(MSLM_EINVAL, "gamma_slices: the global null model has one resolution");
  sp.gn.assign(T, 0);
  sp.gd.assign(T, 1);
  for (int s = 0; s < T; s++) {
    mslm_status st = check_fraction(gs[2 * s], gs[2 * s + 1], "gamma_slices");
    if (st != MSLM_OK) return st;
    if (gs[2 * s] == 0) return fail(MSLM_EINVAL, "gamma_slices: every resolution must be > 0");
    const int64_t g = gcd64(gs[2 * s], gs[2 * s + 1]);
    sp.gn[s] = gs[2 * s] / g;
    sp.gd[s] = gs[2 * s + 1] / g;
  }
  int64_t Q = 1, C = 1;
  for (int s = 0; s < T; s++)
    if (!lcm_below(Q, sp.gd[s], kLim31, Q))
      return fail(MSLM_EOVERFLOW, "gamma_slices: the common denominator reaches 2^31");
  sp.smul.assign(T, 1);
  std::vector<int64_t> P(T);
  for (int s = 0; s < T; s++) {
    P[s] = sp.gn[s] * (Q / sp.gd[s]);   // < 2^62
    if (!lcm_below(C, P[s], (int64_t)1 << 62, C))
      return fail(MSLM_EOVERFLOW, "gamma_slices: the common multiple of the scaled resolutions "
                                  "reaches 2^62");
  }
  for (int s = 0; s < T; s++) sp.smul[s] = C / P[s];
  sp.pe = C;
  sp.qe = Q;
  return MSLM_OK;
}

// ------------------------------------------------------------------ exact rational Q
// Small arbitrary-precision integers for the host-side reduction of Q.
struct BigU {
  std::vector<uint32_t> d;   // little endian, no leading zeros
  void trim() {
    while (!d.empty() && d.back() == 0) d.pop_back();
  }
  bool zero() const { return d.empty(); }
  static BigU from(uint64_t v) {
    BigU r;
    while (v) {
      r.d.push_back((uint32_t)v);
      v >>= 32;
    }
    return r;
  }
  void mul(uint64_t m) {
    if (m == 0 || d.empty()) {
      d.clear();
      return;
    }
    unsigned __int128 c = 0;
    for (auto &x : d) {
      unsigned __int128 t = (unsigned __int128)x * m + c;
      x = (uint32_t)t;
      c = t >> 32;
    }
    while (c) {
      d.push_back((uint32_t)c);
      c >>= 32;
    }
  }
};
int cmpu(const BigU &a, const BigU &b) {
  if (a.d.size() != b.d.size()) return a.d.size() < b.d.size() ? -1 : 1;
  for (size_t i = a.d.size(); i-- > 0;)
    if (a.d[i] != b.d[i]) return a.d[i] < b.d[i] ? -1 : 1;
  return 0;
}
BigU addu(const BigU &a, const BigU &b) {
  BigU r;
  size_t n = std::max(a.d.size(), b.d.size());
  r.d.resize(n + 1);
  uint64_t c = 0;
  for (size_t i = 0; i < n; i++) {
    uint64_t t = c + (i < a.d.size() ? a.d[i] : 0) + (i < b.d.size() ? b.d[i] : 0);
    r.d[i] = (uint32_t)t;
    c = t >> 32;
  }
  r.d[n] = (uint32_t)c;
  r.trim();
  return r;
}
BigU subu(const BigU &a, const BigU &b) {   // a >= b
  BigU r;
  r.d.resize(a.d.size());
  int64_t br = 0;
  for (size_t i = 0; i < a.d.size(); i++) {
    int64_t t = (int64_t)a.d[i] - (i < b.d.size() ? b.d[i] : 0) - br;
    br = t < 0;
    if (t < 0) t += (int64_t)1 << 32;
    r.d[i] = (uint32_t)t;
  }
  r.trim();
  return r;
}
// quotient and remainder by shift-subtract long division
void divmodu(const BigU &a, const BigU &b, BigU &q, BigU &r) {
  q.d.assign(a.d.size(), 0);
  r.d.clear();
  for (size_t i = a.d.size() * 32; i-- > 0;) {
    // r = 2r + bit
    uint32_t carry = (a.d[i / 32] >> (i % 32)) & 1u;
    for (auto &x : r.d) {
      uint32_t nc = x >> 31;
      x = (x << 1) | carry;
      carry = nc;
    }
    if (carry) r.d.push_back(carry);
    if (cmpu(r, b) >= 0) {
      r = subu(r, b);
      q.d[i / 32] |= 1u << (i % 32);
    }
  }
  q.trim();
  r.trim();
}
BigU gcdu(BigU a, BigU b) {
  while (!b.zero()) {
    BigU q, r;
    divmodu(a, b, q, r);
    a = b;
    b = r;
  }
  return a;
}
std::string decimal(BigU a) {
  if (a.zero()) return "0";
  std::string s;
  while (!a.zero()) {
    uint64_t rem = 0;
    for (size_t i = a.d.size(); i-- > 0;) {
      uint64_t cur = (rem << 32) | a.d[i];
      a.d[i] = (uint32_t)(cur / 1000000000u);
      rem = cur % 1000000000u;
    }
    a.trim();
    char buf[16];
    snprintf(buf, sizeof buf, a.zero() ? "%llu" : "%09llu", (unsigned long long)rem);
    s = std::string(buf) + s;
  }
  return s;
}
struct BigS {   // signed
  bool neg = false;
  BigU m;
};
BigS adds(const BigS &a, const BigS &b) {
  BigS r;
  if (a.neg == b.neg) {
    r.m = addu(a.m, b.m);
    r.neg = a.neg;
  } else if (cmpu(a.m, b.m) >= 0) {
    r.m = subu(a.m, b.m);
    r.neg = a.neg;
  } else {
    r.m = subu(b.m, a.m);
    r.neg = b.neg;
  }
  if (r.m.zero()) r.neg = false;
  return r;
}
BigS mk(int64_t v) {
  BigS r;
  r.neg = v < 0;
  r.m = BigU::from(v < 0 ? (uint64_t)0 - (uint64_t)v : (uint64_t)v);
  return r;
}

// Q = (sum_s [W_s - gamma^(s) SS_s / D_s] + omega I) / (sum_s 2m_s + omega ctot) with
// D_s = 2m_s (Eq. 6; a slice without edges has no null term) or 1 (the multislice CPM),
// multiplied through by b * L, L = prod over the slices with a null term of gd_s * D_s, and
// reduced.
mslm_status q_exact_gen(const int64_t *c, int T, int64_t ctot, const int64_t *gn,
                        const int64_t *gd, bool cpm, int64_t oa, int64_t ob, std::string &num,
                        std::string &den, double &qd) {
  std::vector<uint64_t> dn(T, 0);   // gd_s * D_s (< 2^62), 0: no null term
  for (int s = 0; s < T; s++) {
    const int64_t D = cpm ? 1 : c[2 * T + s];
    if (D > 0) dn[s] = (uint64_t)gd[s] * (uint64_t)D;
  }
  BigU L = BigU::from(1);
  for (uint64_t m : dn)
    if (m) L.mul(m);
  BigS sumN;   // numerator
  int64_t sumW = 0, sum2m = 0;
  for (int s = 0; s < T; s++) {
    sumW += c[s];
    sum2m += c[2 * T + s];
  }
  BigS t = mk(sumW);
  t.m.mul((uint64_t)ob);
  t.m = [&] { BigU x = t.m; for (uint64_t m : dn) if (m) x.mul(m); return x; }();
  sumN = adds(sumN, t);
  for (int s = 0; s < T; s++) {
    if (!dn[s]) continue;
    BigS u = mk(c[T + s]);
    u.m.mul((uint64_t)ob);
    u.m.mul((uint64_t)gn[s]);
    for (int r = 0; r < T; r++)
      if (r != s && dn[r]) u.m.mul(dn[r]);
    u.neg = !u.m.zero();
    sumN = adds(sumN, u);
  }
  BigS iv = mk(c[3 * T]);
  iv.m.mul((uint64_t)oa);
  for (uint64_t m : dn)
    if (m) iv.m.mul(m);
  sumN = adds(sumN, iv);
  // denominator: b*L*sum 2m_s + a*L*ctot
  BigU d1 = BigU::from((uint64_t)sum2m);
  d1.mul((uint64_t)ob);
  for (uint64_t m : dn)
    if (m) d1.mul(m);
  BigU d2 = BigU::from((uint64_t)ctot);
  d2.mul((uint64_t)oa);
  for (uint64_t m : dn)
    if (m) d2.mul(m);
  BigU D = addu(d1, d2);
  if (D.zero()) {   // empty supra-graph: Q = 0 by convention
    num = "0";
    den = "1";
    qd = 0.0;
    return MSLM_OK;
  }
  BigU g = gcdu(sumN.m, D);
  BigU qn, rn, qdn, rdn;
  if (sumN.m.zero()) {
    num = "0";
    den = "1";
    qd = 0.0;
    return MSLM_OK;
  }
  divmodu(sumN.m, g, qn, rn);
  divmodu(D, g, qdn, rdn);
  num = (sumN.neg ? "-" : "") + decimal(qn);
  den = decimal(qdn);
  // double: each value as its top three limbs (96 bits, rounded to 53) times a power of two,
  // so the ratio keeps full double precision whatever the two sizes
  auto top = [](const BigU &x, int &e) {
    const size_t n = x.d.size(), k = std::min<size_t>(3, n);
    double t = 0;
    for (size_t i = n; i-- > n - k;) t = t * 4294967296.0 + x.d[i];
    e = 32 * (int)(n - k);
    return t;
  };
  int ea = 0, eb = 0;
  const double ta = top(qn, ea), tb = top(qdn, eb);
  qd = (sumN.neg ? -1.0 : 1.0) * std::ldexp(ta / tb, ea - eb);
  return MSLM_OK;
}

// Eq. 6 with one resolution gp/gq in every slice and the ordinal coupling of every copy.
mslm_status q_exact(const int64_t *c, int T, int N, int64_t gp, int64_t gq, int64_t oa, int64_t ob,
                    std::string &num, std::string &den, double &qd) {
  std::vector<int64_t> gn(T, gp), gd(T, gq);
  return q_exact_gen(c, T, 2 * (int64_t)N * (T - 1), gn.data(), gd.data(), false, oa, ob, num,
                     den, qd);
}

}  // namespace

namespace mslm {

mslm_status api_fail(mslm_status s, const std::string &m) { return fail(s, m); }
void api_clear_error() { g_err.clear(); }
const char *api_error_text() { return g_err.c_str(); }
size_t solve_scratch_estimate(int64_t n, int64_t nnz) {
  // aggregation keys and values double-buffered, sort scratch, two aggregated levels,
  // per-unit state, the Sigma tables and level 0 laid out in colour-batch order (with the
  // neighbour-label copy and reverse entries)
  return (size_t)(104 * nnz + 384 * n) + ((size_t)1 << 20);
}
size_t footprint_estimate(const mslm_graph_desc *d) {
  if (check_desc_shape(d) != MSLM_OK) return 0;
  const int64_t n = (int64_t)d->n_nodes * d->n_slices;
  const int64_t E = d->slice_offsets[d->n_slices];
  const int64_t P = api_coupled_pairs(api_coupling_matrix(d), d->n_slices);
  const int64_t nnz = 2 * E + 2 * (int64_t)d->n_nodes * P;
  // resident graph + peak of one solve
  return (size_t)(8 * (n + 1) + 12 * nnz + 4 * n) + solve_scratch_estimate(n, nnz) + (64u << 20);
}
mslm_status api_check_shape(const mslm_graph_desc *d) { return check_desc_shape(d); }
mslm_status api_check_desc(const mslm_graph_desc *d) {
  mslm_status s = check_desc_shape(d);
  return s != MSLM_OK ? s : check_desc_edges(d);
}
namespace {
typedef __int128 i128;
typedef unsigned __int128 u128;
u128 gcd128(u128 a, u128 b) {
  while (b) {
    u128 t = a % b;
    a = b;
    b = t;
  }
  return a;
}
std::string dec128(u128 x) {
  if (x == 0) return "0";
  std::string s;
  while (x) {
    s.push_back(char('0' + (int)(x % 10)));
    x /= 10;
  }
  return std::string(s.rbegin(), s.rend());
}
}  // namespace

int64_t global_two_mu(int64_t sum_two_m, int64_t ctot, const SolveSpec &sp) {
  const i128 v = (i128)sp.b * sum_two_m + (i128)sp.a * ctot;
  return v >= ((i128)1 << 62) ? ((int64_t)1 << 62) : (int64_t)v;
}

bool api_global_headroom(int64_t two_mu, const SolveSpec &sp) {
  const int64_t pq = sp.p > sp.q ? sp.p : sp.q;
  if (two_mu >= ((int64_t)1 << 31) || (i128)pq * two_mu * two_mu >= ((i128)1 << 62)) {
    fail(MSLM_EOVERFLOW, "global null model: 2mu' must stay below 2^31 and max(p,q)*2mu'^2 "
                         "below 2^62");
    return false;
  }
  return true;
}

mslm_status api_q_exact_global(const int64_t *c, int T, int N, int64_t ctot, int64_t gp, int64_t gq, int64_t oa,
                               int64_t ob, std::string &num, std::string &den, double &qd) {
  // every factor is below 2^31 or (SS') below 2^62, so the numerator and the denominator
  // stay below 2^94 and int128 holds them exactly
  int64_t W = 0, tm = 0;
  for (int s = 0; s < T; s++) {
    W += c[s];
    tm += c[2 * T + s];
  }
  (void)N;
  const i128 two_mu = (i128)ob * tm + (i128)oa * ctot;
  const i128 Wp = (i128)ob * W + (i128)oa * c[3 * T];
  if (two_mu == 0) {
    num = "0";
    den = "1";
    qd = 0.0;
    return MSLM_OK;
  }
  i128 nu = (i128)gq * two_mu * Wp - (i128)gp * c[T];
  const i128 de = (i128)gq * two_mu * two_mu;
  const bool neg = nu < 0;
  u128 a = neg ? (u128)(-nu) : (u128)nu, b = (u128)de;
  const u128 g = a ? gcd128(a, b) : b;
  a /= g;
  b /= g;
  num = (neg && a ? "-" : "") + dec128(a);
  den = dec128(b);
  qd = (neg ? -1.0 : 1.0) * ((double)a / (double)b);
  return MSLM_OK;
}

mslm_status api_tuning_from(const mslm_tuning *t, Tuning &out) {
  if (!t) return fail(MSLM_EINVAL, "tuning is NULL");
  if (t->graphs != 0 && t->graphs != 1) return fail(MSLM_EINVAL, "tuning.graphs must be 0 or 1");
  if (t->latency_units < 64 || t->latency_units > 65536)
    return fail(MSLM_EINVAL, "tuning.latency_units must be in 64..65536");
  if (t->split_group_units < 0 || t->split_group_units > (1 << 30))
    return fail(MSLM_EINVAL, "tuning.split_group_units must be in 0..2^30");
  if (t->copy_moves < 1 || t->copy_moves > (1 << 30))
    return fail(MSLM_EINVAL, "tuning.copy_moves must be in 1..2^30");
  if (t->lat_parts_max < 1 || t->lat_parts_max > 16)
    return fail(MSLM_EINVAL, "tuning.lat_parts_max must be in 1..16");
  if (t->batch_units < 1 || t->batch_units > 100)
    return fail(MSLM_EINVAL, "tuning.batch_units must be in 1..100");
  out.graphs = t->graphs;
  out.latency_units = t->latency_units;
  out.split_group_units = t->split_group_units;
  out.copy_moves = t->copy_moves;
  out.lat_parts_max = t->lat_parts_max;
  out.batch_units = (int64_t)t->batch_units << 20;
  return MSLM_OK;
}

void api_tuning_to(const Tuning &t, mslm_tuning *out) {
  std::memset(out, 0, sizeof(*out));
  out->graphs = t.graphs;
  out->latency_units = (int32_t)t.latency_units;
  out->split_group_units = (int32_t)t.split_group_units;
  out->copy_moves = (int32_t)t.copy_moves;
  out->lat_parts_max = t.lat_parts_max;
  out->batch_units = (int32_t)(t.batch_units >> 20);
}

mslm_status api_check_fraction(int64_t num, int64_t den, const char *what) {
  return check_fraction(num, den, what);
}
int64_t api_gcd(int64_t a, int64_t b) { return gcd64(a, b); }
mslm_status api_make_spec(const mslm_params *p, int64_t on, int64_t od, int32_t N, int32_t T,
                          SolveSpec &sp) {
  mslm_status s = make_spec(p, on, od, sp);
  if (s != MSLM_OK) return s;
  if (p->gamma_slices) {
    s = slice_resolutions(p->gamma_slices, T, sp);
    if (s != MSLM_OK) return s;
  }
  if (p->initial_membership) {
    const int64_t n = (int64_t)N * T;
    for (int64_t v = 0; v < n; v++)
      if (p->initial_membership[v] < 0 || p->initial_membership[v] >= n)
        return fail(MSLM_EINVAL, "initial_membership: label of supra-node " + std::to_string(v) +
                                     " outside [0, T*N)");
    sp.init.assign(p->initial_membership, p->initial_membership + n);
  }
  return MSLM_OK;
}

bool api_slice_denominator(const SolveSpec &sp, int s, int64_t two_m, int64_t N, int64_t crow_s,
                           int64_t &Sdev) {
  const bool cpm = sp.null_model == MSLM_NULL_CPM;
  const int64_t S = two_m > 0 ? two_m : 1;
  const i128h sd = (i128h)(cpm ? 1 : S) * (sp.smul.empty() ? 1 : sp.smul[s]);
  if (sd >= kLim31) {
    fail(MSLM_EOVERFLOW, "per-slice resolutions: a scaled slice denominator reaches 2^31");
    return false;
  }
  const i128h K = cpm ? N : S;
  const i128h a1 = (i128h)sp.qe * sd * ((i128h)sp.b * S + (i128h)sp.a * crow_s);
  const i128h a2 = (i128h)sp.pe * sp.b * K * K;
  if (a1 >= ((i128h)1 << 62) || a2 >= ((i128h)1 << 62)) {
    fail(MSLM_EOVERFLOW, "gain head-room: q*2m_s*w or p*b*k*Sigma reaches 2^62");
    return false;
  }
  Sdev = (int64_t)sd;
  return true;
}

mslm_status api_q_exact_spec(const int64_t *c, int T, int N, int64_t ctot, const SolveSpec &sp,
                             std::string &num, std::string &den, double &qd) {
  if (sp.null_model == MSLM_NULL_GLOBAL)
    return api_q_exact_global(c, T, N, ctot, sp.p, sp.q, sp.a, sp.b, num, den, qd);
  std::vector<int64_t> gn(sp.gn), gd(sp.gd);
  if (gn.empty()) {
    gn.assign(T, sp.p);
    gd.assign(T, sp.q);
  }
  (void)N;
  return q_exact_gen(c, T, ctot, gn.data(), gd.data(), sp.null_model == MSLM_NULL_CPM, sp.a,
                     sp.b, num, den, qd);
}

mslm_status api_q_exact_slices(const int64_t *c, int T, int N, int64_t ctot, const int64_t *gn,
                               const int64_t *gd, bool cpm, int64_t oa, int64_t ob,
                               std::string &num, std::string &den, double &qd) {
  (void)N;
  return q_exact_gen(c, T, ctot, gn, gd, cpm, oa, ob, num, den, qd);
}

std::vector<int32_t> api_coupling_matrix(const mslm_graph_desc *d) {
  const int T = d->n_slices;
  std::vector<int32_t> cm((size_t)T * T, 0);
  for (int a = 0; a < T; a++)
    for (int b = 0; b < T; b++)
      cm[(size_t)a * T + b] = d->coupling ? d->coupling[a * T + b] : (a - b == 1 || b - a == 1);
  return cm;
}

std::vector<int64_t> api_coupling_rows(const std::vector<int32_t> &cm, int T) {
  std::vector<int64_t> row(T, 0);
  for (int a = 0; a < T; a++)
    for (int b = 0; b < T; b++) row[a] += cm[(size_t)a * T + b];
  return row;
}

int64_t api_coupled_pairs(const std::vector<int32_t> &cm, int T) {
  int64_t P = 0;
  for (int a = 0; a < T; a++)
    for (int b = a + 1; b < T; b++) P += cm[(size_t)a * T + b] != 0;
  return P;
}

int64_t api_coupling_total_host(const mslm_graph_desc *d) {
  const int T = d->n_slices;
  const int64_t N = d->n_nodes;
  const std::vector<int32_t> cm = api_coupling_matrix(d);
  if (!(d->flags & MSLM_COUPLE_PRESENT)) {
    int64_t t = 0;
    for (int32_t c : cm) t += c;
    return t * N;
  }
  std::vector<uint8_t> pres((size_t)N * T, 0);
  for (int s = 0; s < T; s++)
    for (int64_t e = d->slice_offsets[s]; e < d->slice_offsets[s + 1]; e++) {
      pres[(size_t)s * N + d->src[e]] = 1;
      pres[(size_t)s * N + d->dst[e]] = 1;
    }
  int64_t t = 0;
  for (int a = 0; a < T; a++)
    for (int b = 0; b < T; b++) {
      const int32_t c = cm[(size_t)a * T + b];
      if (!c) continue;
      for (int64_t i = 0; i < N; i++)
        if (pres[(size_t)a * N + i] && pres[(size_t)b * N + i]) t += c;
    }
  return t;
}
mslm_status api_q_exact(const int64_t *c, int T, int N, int64_t gp, int64_t gq, int64_t oa,
                        int64_t ob, std::string &num, std::string &den, double &qd) {
  return q_exact(c, T, N, gp, gq, oa, ob, num, den, qd);
}
// The int64 head-room preconditions of a solve on host edge lists, taken before any device
// work: every slice's total degree 2m_s < 2^31 (build) and q*S*(b*S + 2a) < 2^62,
// p*b*S^2 < 2^62 with S = max(2m_s, 1) (level-0 gains); the same checks the device path
// makes, so a request that passes them cannot fail on them later.
mslm_status api_check_headroom(const mslm_graph_desc *d, const SolveSpec &sp) {
  const std::vector<int64_t> crow = api_coupling_rows(api_coupling_matrix(d), d->n_slices);
  int64_t sum_two_m = 0;
  for (int s = 0; s < d->n_slices; s++) {
    int64_t two_m = 0;
    for (int64_t e = d->slice_offsets[s]; e < d->slice_offsets[s + 1]; e++) {
      two_m += 2 * (int64_t)(d->weight ? d->weight[e] : 1);
      if (two_m >= kLim31) return fail(MSLM_EOVERFLOW, "a slice's total degree 2m_s reaches 2^31");
    }
    sum_two_m += two_m;
    if (sp.null_model == MSLM_NULL_GLOBAL) continue;
    int64_t Sdev = 0;
    if (!api_slice_denominator(sp, s, two_m, d->n_nodes, crow[s], Sdev)) return MSLM_EOVERFLOW;
  }
  if (sp.null_model == MSLM_NULL_GLOBAL &&
      !api_global_headroom(global_two_mu(sum_two_m, api_coupling_total_host(d), sp), sp))
    return MSLM_EOVERFLOW;
  return MSLM_OK;
}

}  // namespace mslm
