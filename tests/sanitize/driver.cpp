// Host code under AddressSanitizer and UndefinedBehaviorSanitizer (built and run by
// tests/test_sanitizers.py with g++/gcc, no GPU): the library's host-side validation, head-room
// checks and exact Q reduction (host.cpp), and the C oracle's whole schedule, its Q components,
// its exact comparator and its trace.  Any sanitizer report ends the run with an error.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mslm.h"
#include "../../paper_2608_03695_amd/csrc/host.hpp"

extern "C" {
struct orc_graph;
struct orc_stats {
  int64_t sweeps, moves, sweep_cap_hits, refine_rounds, merges, splits;
  int32_t levels_run, iterations_run, n_communities, colours_first;
};
int orc_create(int32_t N, int32_t T, const int64_t *off, const int32_t *src, const int32_t *dst,
               const int32_t *w, int64_t omega_num, int64_t omega_den, const int32_t *coupling,
               int32_t present_only, orc_graph **out);
int64_t orc_coupling_total(const orc_graph *g);
void orc_destroy(orc_graph *g);
int64_t orc_nnz(const orc_graph *g);
void orc_csr(const orc_graph *g, int64_t *rp, int32_t *col, int64_t *w, int32_t *raw, int64_t *twom);
int orc_leiden(const orc_graph *G, int64_t gamma_num, int64_t gamma_den,
               const int64_t *gamma_slices, const int32_t *initial, int32_t max_levels,
               int32_t max_iterations, int32_t max_sweeps, uint64_t seed, int32_t null_model,
               int32_t *membership, int64_t *comps, orc_stats *st);
int orc_q_components(const orc_graph *G, const int32_t *memb, int64_t *comps);
int orc_q_components_global(const orc_graph *G, const int32_t *memb, int64_t *comps);
int orc_q_components_cpm(const orc_graph *G, const int32_t *memb, int64_t *comps);
int orc_gain_sign(int64_t p, int64_t q, int64_t b, const int64_t *S, int64_t W, int m,
                  const int32_t *ps, const int64_t *pk, const int64_t *y);
void orc_trace_enable(int on);
int orc_trace_count(void);
void orc_trace_info(int i, int64_t *info);
void orc_trace_get(int i, int64_t *rp, int32_t *col, int64_t *w, int64_t *pp, int32_t *ps,
                   int64_t *pk, int32_t *colour, uint32_t *p_in, uint32_t *p_lm, uint32_t *r,
                   int64_t *map0, int64_t n0);
void orc_trace_refine(int i, int64_t *ext, char *wc);
}

namespace {

uint64_t g_state = 0x9e3779b97f4a7c15ull;
uint64_t next() {   // xorshift64*
  g_state ^= g_state >> 12;
  g_state ^= g_state << 25;
  g_state ^= g_state >> 27;
  return g_state * 0x2545f4914f6cdd1dull;
}
int64_t pick(int64_t lo, int64_t hi) { return lo + (int64_t)(next() % (uint64_t)(hi - lo + 1)); }

struct Graph {
  int32_t N = 0, T = 0;
  std::vector<int64_t> off;
  std::vector<int32_t> src, dst, w;
  mslm_graph_desc desc(bool weighted) const {
    mslm_graph_desc d{};
    d.n_nodes = N;
    d.n_slices = T;
    d.slice_offsets = off.data();
    d.src = src.data();
    d.dst = dst.data();
    d.weight = weighted ? w.data() : nullptr;
    d.omega_num = 1;
    d.omega_den = 1;
    return d;
  }
};

Graph random_graph(int32_t N, int32_t T, int per_slice) {
  Graph g;
  g.N = N;
  g.T = T;
  g.off.push_back(0);
  for (int s = 0; s < T; s++) {
    for (int e = 0; e < per_slice; e++) {
      int32_t u = (int32_t)pick(0, N - 1), x = (int32_t)pick(0, N - 1);
      if (u == x) continue;
      g.src.push_back(u);
      g.dst.push_back(x);
      g.w.push_back((int32_t)pick(1, 5));
    }
    g.off.push_back((int64_t)g.src.size());
  }
  return g;
}

int failures = 0;
void expect(bool ok, const char *what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (%s)\n", what, mslm::api_error_text());
    failures++;
  }
}

void host_checks() {
  using namespace mslm;
  Graph g = random_graph(20, 3, 30);
  mslm_graph_desc d = g.desc(true);
  expect(api_check_desc(&d) == MSLM_OK, "valid graph");
  expect(api_check_desc(nullptr) == MSLM_EINVAL, "NULL desc");
  Graph bad = g;
  bad.src[3] = 20;
  mslm_graph_desc db = bad.desc(true);
  expect(api_check_desc(&db) == MSLM_EINVAL, "id out of range");
  bad = g;
  bad.dst[2] = bad.src[2];
  db = bad.desc(true);
  expect(api_check_desc(&db) == MSLM_EINVAL, "self-loop");
  bad = g;
  bad.w[1] = 0;
  db = bad.desc(true);
  expect(api_check_desc(&db) == MSLM_EINVAL, "zero weight");
  db = g.desc(true);
  db.n_slices = 65;
  std::vector<int64_t> off65(66, 0);
  db.slice_offsets = off65.data();
  expect(api_check_desc(&db) == MSLM_EUNSUPPORTED, "65 slices");
  db = g.desc(true);
  db.omega_den = 0;
  expect(api_check_desc(&db) == MSLM_EINVAL, "omega denominator 0");
  db.omega_den = (int64_t)1 << 40;
  expect(api_check_desc(&db) == MSLM_EOVERFLOW, "omega too large");
  mslm_params p{};
  p.gamma_num = 3;
  p.gamma_den = 6;
  p.max_levels = 32;
  SolveSpec sp;
  expect(api_make_spec(&p, 2, 4, 10, 3, sp) == MSLM_OK && sp.p == 1 && sp.q == 2 && sp.a == 1 &&
             sp.b == 2 && sp.pe == 1 && sp.qe == 2 && sp.smul.empty(),
         "spec reduction");
  // per-slice resolutions over 64 slices and a start partition
  {
    mslm_params pv = p;
    std::vector<int64_t> gs(128);
    for (int s = 0; s < 64; s++) {
      gs[2 * s] = pick(1, 12);
      gs[2 * s + 1] = pick(1, 12);
    }
    std::vector<int32_t> init(64 * 5);
    for (auto &x : init) x = (int32_t)pick(0, 64 * 5 - 1);
    pv.gamma_slices = gs.data();
    pv.initial_membership = init.data();
    SolveSpec sv;
    const mslm_status rc = api_make_spec(&pv, 1, 1, 5, 64, sv);
    expect(rc == MSLM_OK || rc == MSLM_EOVERFLOW, "per-slice spec");
    if (rc == MSLM_OK) {
      bool ok = sv.smul.size() == 64 && sv.init.size() == 320;
      for (int s = 0; s < 64 && ok; s++)   // gamma^(s) = pe / (qe * smul_s)
        ok = (__int128)sv.gn[s] * sv.qe * sv.smul[s] == (__int128)sv.pe * sv.gd[s];
      expect(ok, "per-slice constants");
      int64_t Sd = 0;
      (void)api_slice_denominator(sv, 3, pick(0, 1 << 20), 5, pick(0, 1 << 20), Sd);
    }
    init[7] = 64 * 5;
    expect(api_make_spec(&pv, 1, 1, 5, 64, sv) == MSLM_EINVAL, "start label out of range");
    init[7] = 0;
    gs[10] = 0;
    expect(api_make_spec(&pv, 1, 1, 5, 64, sv) == MSLM_EINVAL, "zero per-slice resolution");
  }
  p.max_levels = 0;
  expect(api_make_spec(&p, 1, 1, 10, 3, sp) == MSLM_EINVAL, "zero levels");
  p.max_levels = 4;
  p.max_sweeps = 33;
  expect(api_make_spec(&p, 1, 1, 10, 3, sp) == MSLM_EINVAL, "33 sweeps");
  expect(api_make_spec(nullptr, 1, 1, 10, 3, sp) == MSLM_EINVAL, "NULL params");
  // head-room: a dense slice with gamma 2^30
  Graph dense = random_graph(400, 1, 40000);
  mslm_graph_desc dd = dense.desc(false);
  SolveSpec big;
  big.p = big.pe = (int64_t)1 << 30;
  expect(api_check_headroom(&dd, big) == MSLM_EOVERFLOW, "head-room overflow");
  SolveSpec one;
  expect(api_check_headroom(&dd, one) == MSLM_OK, "head-room ok");
  expect(footprint_estimate(&dd) > 0, "footprint");
  // general coupling: a random symmetric matrix, present-only copies, the global null model
  {
    Graph gc = random_graph(50, 5, 30);
    mslm_graph_desc dc = gc.desc(true);
    std::vector<int32_t> cm(25, 0);
    for (int s = 0; s < 5; s++)
      for (int r = s + 1; r < 5; r++) cm[s * 5 + r] = cm[r * 5 + s] = (int32_t)pick(0, 4);
    dc.coupling = cm.data();
    dc.flags = MSLM_COUPLE_PRESENT;
    expect(api_check_desc(&dc) == MSLM_OK, "coupling accepted");
    const int64_t ct = api_coupling_total_host(&dc);
    dc.flags = 0;
    const int64_t ct_all = api_coupling_total_host(&dc);
    expect(ct >= 0 && ct <= ct_all, "coupling totals");
    SolveSpec gs;
    gs.null_model = MSLM_NULL_GLOBAL;
    expect(api_check_headroom(&dc, gs) == MSLM_OK, "global head-room with coupling");
    expect(footprint_estimate(&dc) > 0, "footprint with coupling");
    cm[1] = 3;
    cm[5] = 2;   // not symmetric
    expect(api_check_desc(&dc) == MSLM_EINVAL, "asymmetric coupling");
    cm[5] = 3;
    cm[0] = 1;   // diagonal
    expect(api_check_desc(&dc) == MSLM_EINVAL, "coupling diagonal");
  }
  // exact Q from random components, all slice counts
  for (int rep = 0; rep < 200; rep++) {
    const int T = (int)pick(1, 64), N = (int)pick(1, 1 << 20);
    std::vector<int64_t> c(3 * T + 1);
    for (int s = 0; s < T; s++) {
      c[2 * T + s] = pick(0, 3) == 0 ? 0 : pick(1, ((int64_t)1 << 31) - 1);
      c[s] = pick(0, c[2 * T + s]);
      c[T + s] = pick(0, (int64_t)1 << 61);
    }
    c[3 * T] = pick(0, (int64_t)2 * N * (T - 1) + 1);
    std::string num, den;
    double q = 0;
    expect(api_q_exact(c.data(), T, N, pick(0, 1 << 30), pick(1, 1 << 30), pick(0, 1 << 30),
                       pick(1, 1 << 30), num, den, q) == MSLM_OK && !num.empty() && !den.empty() &&
               den != "0",
           "exact Q");
    std::vector<int64_t> gn(T), gd(T);
    for (int s = 0; s < T; s++) {
      gn[s] = pick(1, ((int64_t)1 << 31) - 1);
      gd[s] = pick(1, ((int64_t)1 << 31) - 1);
    }
    expect(api_q_exact_slices(c.data(), T, N, pick(0, (int64_t)1 << 40), gn.data(), gd.data(),
                              rep % 2 == 1,
                              pick(0, 1 << 30), pick(1, 1 << 30), num, den, q) == MSLM_OK &&
               !num.empty() && den != "0",
           "exact Q, per-slice resolutions");
  }
}

void oracle_runs() {
  for (int rep = 0; rep < 24; rep++) {
    const int32_t T = rep % 6 == 5 ? 64 : (int32_t)pick(1, 5);
    const int32_t N = (int32_t)pick(2, T == 64 ? 8 : 40);
    Graph g = random_graph(N, T, (int)pick(0, 3 * N));
    const bool weighted = rep % 2 == 0;
    orc_graph *og = nullptr;
    const int64_t on = pick(0, 3), od = pick(1, 4);
    // every third graph with a general coupling matrix, every other with present-only copies
    std::vector<int32_t> cm(T * T, 0);
    for (int s = 0; s < T; s++)
      for (int r = s + 1; r < T; r++) cm[s * T + r] = cm[r * T + s] = (int32_t)pick(0, 3);
    if (orc_create(N, T, g.off.data(), g.src.data(), g.dst.data(), weighted ? g.w.data() : nullptr,
                   on, od, rep % 3 == 1 ? cm.data() : nullptr, rep % 2, &og) != 0) {
      expect(false, "oracle create");
      continue;
    }
    const int64_t n = (int64_t)N * T, m = orc_nnz(og);
    expect(orc_coupling_total(og) >= 0, "coupling total");
    std::vector<int64_t> rp(n + 1), w(m > 0 ? m : 1), twom(T);
    std::vector<int32_t> col(m > 0 ? m : 1), raw(m > 0 ? m : 1);
    orc_csr(og, rp.data(), col.data(), w.data(), raw.data(), twom.data());
    const bool trace = rep % 4 == 0;
    orc_trace_enable(trace ? 1 : 0);
    std::vector<int32_t> memb(n);
    std::vector<int64_t> comps(3 * T + 1);
    orc_stats st{};
    // the three objectives in turn; per-slice resolutions and a start partition now and then
    const int model = rep % 3;
    std::vector<int64_t> gs(2 * T);
    for (int s = 0; s < T; s++) {
      gs[2 * s] = pick(1, 4);
      gs[2 * s + 1] = pick(1, 3);
    }
    std::vector<int32_t> init(n);
    for (int64_t v = 0; v < n; v++) init[v] = (int32_t)pick(0, n - 1);
    const bool per_slice = model != 1 && rep % 5 < 2, warm = rep % 7 < 3;
    expect(orc_leiden(og, pick(1, 4), pick(1, 3), per_slice ? gs.data() : nullptr,
                      warm ? init.data() : nullptr, (int32_t)pick(1, 32), (int32_t)pick(0, 3),
                      (int32_t)pick(0, 4), next(), model, memb.data(), comps.data(), &st) == 0,
           "oracle leiden");
    if (trace) {
      for (int i = 0; i < orc_trace_count(); i++) {
        int64_t info[8];
        orc_trace_info(i, info);
        const int64_t tn = info[2], tm = info[3], tp = info[6];
        std::vector<int64_t> trp(tn + 1), tw(tm + 1), tpp(tn + 1), tpk(tp + 1), map0(n);
        std::vector<int32_t> tcol(tm + 1), tps(tp + 1), colour(tn + 1);
        std::vector<uint32_t> pin(tn + 1), plm(tn + 1), r(tn + 1);
        orc_trace_get(i, trp.data(), tcol.data(), tw.data(), tpp.data(), tps.data(), tpk.data(),
                      colour.data(), pin.data(), plm.data(), info[7] ? r.data() : nullptr,
                      map0.data(), n);
        if (info[7]) {
          std::vector<int64_t> ext(tn + 1);
          std::vector<char> wc(tn + 1);
          orc_trace_refine(i, ext.data(), wc.data());
        }
      }
      orc_trace_enable(0);
    }
    std::vector<int64_t> comps2(3 * T + 1);
    if (model == 1) orc_q_components_global(og, memb.data(), comps2.data());
    else if (model == 2) orc_q_components_cpm(og, memb.data(), comps2.data());
    else orc_q_components(og, memb.data(), comps2.data());
    expect(comps == comps2, "Q components of the result");
    orc_destroy(og);
  }
  // the exact comparator on multi-slice profiles (the big-integer path)
  for (int rep = 0; rep < 500; rep++) {
    const int m = (int)pick(1, 64);
    std::vector<int64_t> S(64), pk(m), y(m);
    std::vector<int32_t> ps(m);
    for (int s = 0; s < 64; s++) S[s] = pick(1, ((int64_t)1 << 31) - 1);
    for (int j = 0; j < m; j++) {
      ps[j] = j;
      pk[j] = pick(1, 1 << 30);
      y[j] = pick(-(1 << 30), 1 << 30);
    }
    const int sgn = orc_gain_sign(pick(0, 1 << 20), pick(1, 1 << 20), pick(1, 1 << 10), S.data(),
                                  pick(-((int64_t)1 << 40), (int64_t)1 << 40), m, ps.data(),
                                  pk.data(), y.data());
    expect(sgn >= -1 && sgn <= 1, "gain sign");
  }
}

}  // namespace

int main() {
  host_checks();
  oracle_runs();
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("sanitized run ok\n");
  return 0;
}
