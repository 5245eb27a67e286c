// C ABI of the multislice Leiden library: argument checks, handles, exact Q, batching.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/mslm.h"
#include "engine.hpp"
#include "handles.hpp"
#include "host.hpp"
#include "server.hpp"

using namespace mslm;

namespace mslm {
void api_finish(const GraphDev &g, const SolveSpec &sp, SolveOut &o, mslm_result *res) {
  std::string a, b;
  double qd = 0;
  api_q_exact_spec(o.res.q_components, g.T, g.N, g.ctot, sp, a, b, qd);
  o.res.q = qd;
  o.res.coupling_total = g.ctot;
  if (res) *res = o.res;
}
}  // namespace mslm

namespace {
inline mslm_status fail(mslm_status s, const std::string &m) { return api_fail(s, m); }
}  // namespace

// ------------------------------------------------------------------ exported functions
extern "C" {

const char *mslm_last_error(void) { return api_error_text(); }

mslm_status mslm_set_allocator(void *(*alloc)(size_t, void *), void (*release)(void *, void *),
                               void *ctx) {
  if ((alloc == nullptr) != (release == nullptr))
    return fail(MSLM_EINVAL, "alloc and release must both be set or both be NULL");
  DevAlloc a;
  a.alloc = alloc;
  a.release = release;
  a.ctx = alloc ? ctx : nullptr;
  set_allocator(a);
  api_clear_error();
  return MSLM_OK;
}

mslm_status mslm_create(const mslm_graph_desc *desc, void *hip_stream, mslm_graph **out) {
  if (!out) return fail(MSLM_EINVAL, "out is NULL");
  *out = nullptr;
  mslm_status s = api_check_desc(desc);
  if (s != MSLM_OK) return s;
  std::unique_ptr<mslm_graph, void (*)(mslm_graph *)> h(new mslm_graph(), mslm_destroy);
  h->st = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&h->device) != hipSuccess) return fail(MSLM_EHIP, "no HIP device");
  try {
    h->ws = workspace_new();
    h->g.omega_num = desc->omega_num;
    h->g.omega_den = desc->omega_den;
    build_graph(h->g, *desc, h->st, h->ws);
    MSLM_HIP(hipStreamSynchronize(h->st));
    workspace_release_build(h->ws);
  } catch (const Error &e) {
    return fail(e.status, e.what());
  } catch (const std::exception &e) {
    return fail(MSLM_ENOMEM, e.what());
  }
  *out = h.release();
  api_clear_error();
  return MSLM_OK;
}

void mslm_destroy(mslm_graph *g) {
  if (!g) return;
  if (g->st) (void)hipStreamSynchronize(g->st);
  delete g;
}

mslm_status mslm_graph_info(const mslm_graph *g, int64_t *n_supra, int64_t *nnz, int64_t *two_m) {
  if (!g) return fail(MSLM_EINVAL, "graph is NULL");
  if (n_supra) *n_supra = g->g.n;
  if (nnz) *nnz = g->g.nnz;
  if (two_m) {
    int64_t t = 0;
    for (auto x : g->g.twom) t += x;
    *two_m = t;
  }
  return MSLM_OK;
}

mslm_status mslm_q_exact(const int64_t *qc, int32_t T, int32_t N, int64_t gamma_num,
                         int64_t gamma_den, int64_t omega_num, int64_t omega_den, char *num,
                         size_t num_cap, char *den, size_t den_cap) {
  if (!qc || !num || !den || T < 1 || T > 64 || N < 1) return fail(MSLM_EINVAL, "bad arguments");
  mslm_status s = api_check_fraction(gamma_num, gamma_den, "gamma");
  if (s != MSLM_OK) return s;
  s = api_check_fraction(omega_num, omega_den, "omega");
  if (s != MSLM_OK) return s;
  int64_t gg = gamma_num ? api_gcd(gamma_num, gamma_den) : gamma_den;
  int64_t go = omega_num ? api_gcd(omega_num, omega_den) : omega_den;
  std::string a, b;
  double qd;
  api_q_exact(qc, T, N, gamma_num / gg, gamma_den / gg, omega_num / go, omega_den / go, a, b, qd);
  if (a.size() + 1 > num_cap || b.size() + 1 > den_cap) return fail(MSLM_EINVAL, "buffer too small");
  memcpy(num, a.c_str(), a.size() + 1);
  memcpy(den, b.c_str(), b.size() + 1);
  return MSLM_OK;
}

mslm_status mslm_q_exact_global(const int64_t *qc, int32_t T, int32_t N, int64_t gamma_num,
                         int64_t gamma_den, int64_t omega_num, int64_t omega_den, char *num,
                         size_t num_cap, char *den, size_t den_cap) {
  if (!qc || !num || !den || T < 1 || T > 64 || N < 1) return fail(MSLM_EINVAL, "bad arguments");
  mslm_status s = api_check_fraction(gamma_num, gamma_den, "gamma");
  if (s != MSLM_OK) return s;
  s = api_check_fraction(omega_num, omega_den, "omega");
  if (s != MSLM_OK) return s;
  int64_t gg = gamma_num ? api_gcd(gamma_num, gamma_den) : gamma_den;
  int64_t go = omega_num ? api_gcd(omega_num, omega_den) : omega_den;
  std::string a, b;
  double qd;
  api_q_exact_global(qc, T, N, 2 * (int64_t)N * (T - 1), gamma_num / gg, gamma_den / gg,
                     omega_num / go, omega_den / go, a, b, qd);
  if (a.size() + 1 > num_cap || b.size() + 1 > den_cap) return fail(MSLM_EINVAL, "buffer too small");
  memcpy(num, a.c_str(), a.size() + 1);
  memcpy(den, b.c_str(), b.size() + 1);
  return MSLM_OK;
}

mslm_status mslm_q_exact_variant(const int64_t *qc, int32_t T, int32_t N, int32_t null_model,
                                 const int64_t *gamma_slices, int64_t gamma_num,
                                 int64_t gamma_den, int64_t omega_num, int64_t omega_den,
                                 int64_t coupling_total, char *num, size_t num_cap, char *den,
                                 size_t den_cap) {
  if (!qc || !num || !den || T < 1 || T > 64 || N < 1) return fail(MSLM_EINVAL, "bad arguments");
  const int64_t ctot = coupling_total < 0 ? 2 * (int64_t)N * (T - 1) : coupling_total;
  if (null_model == MSLM_NULL_GLOBAL && !gamma_slices) {
    mslm_status s = api_check_fraction(gamma_num, gamma_den, "gamma");
    if (s != MSLM_OK) return s;
    s = api_check_fraction(omega_num, omega_den, "omega");
    if (s != MSLM_OK) return s;
    int64_t gg = gamma_num ? api_gcd(gamma_num, gamma_den) : gamma_den;
    int64_t go = omega_num ? api_gcd(omega_num, omega_den) : omega_den;
    std::string a, b;
    double qd;
    api_q_exact_global(qc, T, N, ctot, gamma_num / gg, gamma_den / gg, omega_num / go,
                       omega_den / go, a, b, qd);
    if (a.size() + 1 > num_cap || b.size() + 1 > den_cap)
      return fail(MSLM_EINVAL, "buffer too small");
    memcpy(num, a.c_str(), a.size() + 1);
    memcpy(den, b.c_str(), b.size() + 1);
    return MSLM_OK;
  }
  if (null_model != MSLM_NULL_MULTISLICE && null_model != MSLM_NULL_CPM)
    return fail(MSLM_EINVAL, "null_model: one resolution for the global null model, else "
                             "MSLM_NULL_MULTISLICE or MSLM_NULL_CPM");
  mslm_status s = api_check_fraction(omega_num, omega_den, "omega");
  if (s != MSLM_OK) return s;
  std::vector<int64_t> gn(T), gd(T);
  for (int t = 0; t < T; t++) {
    const int64_t a = gamma_slices ? gamma_slices[2 * t] : gamma_num;
    const int64_t d = gamma_slices ? gamma_slices[2 * t + 1] : gamma_den;
    s = api_check_fraction(a, d, "gamma");
    if (s != MSLM_OK) return s;
    const int64_t g = a ? api_gcd(a, d) : d;
    gn[t] = a / g;
    gd[t] = d / g;
  }
  int64_t go = omega_num ? api_gcd(omega_num, omega_den) : omega_den;
  std::string a, b;
  double qd;
  api_q_exact_slices(qc, T, N, ctot, gn.data(), gd.data(), null_model == MSLM_NULL_CPM,
                     omega_num / go, omega_den / go, a, b, qd);
  if (a.size() + 1 > num_cap || b.size() + 1 > den_cap) return fail(MSLM_EINVAL, "buffer too small");
  memcpy(num, a.c_str(), a.size() + 1);
  memcpy(den, b.c_str(), b.size() + 1);
  return MSLM_OK;
}

mslm_status mslm_leiden_windowed(const mslm_graph_desc *desc, const mslm_params *params,
                                 int32_t window, int32_t overlap, void *hip_stream,
                                 int32_t *membership, mslm_window_result *res) {
  if (!desc || !params || !membership) return fail(MSLM_EINVAL, "desc, params or membership is NULL");
  if (window < 1 || window > 64 || overlap < 0 || overlap >= window)
    return fail(MSLM_EINVAL, "windowed: need 1 <= window <= 64 and 0 <= overlap < window");
  if (desc->flags & MSLM_INPUT_ON_DEVICE) return fail(MSLM_EINVAL, "windowed: host edge lists only");
  if (desc->coupling) return fail(MSLM_EINVAL, "windowed: ordinal coupling only (coupling NULL)");
  if (params->initial_membership) return fail(MSLM_EINVAL, "windowed: no start partition");
  const int32_t T = desc->n_slices, N = desc->n_nodes;
  if (T < 1 || N < 1 || !desc->slice_offsets || desc->slice_offsets[0] != 0)
    return fail(MSLM_EINVAL, "windowed: need n_nodes >= 1, n_slices >= 1, slice_offsets[0] = 0");
  for (int s = 0; s < T; s++)
    if (desc->slice_offsets[s + 1] < desc->slice_offsets[s])
      return fail(MSLM_EINVAL, "slice_offsets must be non-decreasing");
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t n = (int64_t)N * T;
  // global labels are dense ids 0..fresh-1 (at most n); window labels are canonical ids
  // below the window's size: the stitching maps are plain arrays, reset after each window
  std::vector<int64_t> glob(n, -1);
  std::vector<int32_t> first_copy(n, -1);   // global label -> first overlap copy of a window
  int64_t fresh = 0;
  int windows = 0;
  int32_t prev_end = 0;
  // one handle for every window: its graph is rebuilt in place and its workspace kept, so
  // device buffers are allocated once for the largest window rather than once per window
  std::unique_ptr<mslm_graph, void (*)(mslm_graph *)> h(new mslm_graph(), mslm_destroy);
  h->st = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&h->device) != hipSuccess) return fail(MSLM_EHIP, "no HIP device");
  try {
    h->ws = workspace_new();
  } catch (const std::exception &e) {
    return fail(MSLM_ENOMEM, e.what());
  }
  for (int32_t s0 = 0;;) {
    const int32_t s1 = std::min(T, s0 + window);
    const int32_t ov = windows == 0 ? 0 : prev_end - s0;   // overlapping snapshots
    const int64_t nw = (int64_t)(s1 - s0) * N;
    std::vector<int64_t> off(s1 - s0 + 1);
    for (int s = s0; s <= s1; s++) off[s - s0] = desc->slice_offsets[s] - desc->slice_offsets[s0];
    mslm_graph_desc sub = *desc;
    sub.n_slices = s1 - s0;
    sub.slice_offsets = off.data();
    const int64_t e0 = desc->slice_offsets[s0];
    sub.src = desc->src ? desc->src + e0 : nullptr;
    sub.dst = desc->dst ? desc->dst + e0 : nullptr;
    sub.weight = desc->weight ? desc->weight + e0 : nullptr;
    std::vector<int32_t> init;
    if (ov > 0) {   // the overlapping copies' labels so far, as labels of this window
      init.resize(nw);
      for (int64_t v = 0; v < nw; v++) init[v] = (int32_t)v;
      const int64_t *gl = glob.data() + (int64_t)s0 * N;
      for (int64_t v = 0; v < (int64_t)ov * N; v++) {
        int32_t &f = first_copy[gl[v]];
        if (f < 0) f = (int32_t)v;
        init[v] = f;
      }
      for (int64_t v = 0; v < (int64_t)ov * N; v++) first_copy[gl[v]] = -1;
    }
    mslm_params p = *params;
    p.gamma_slices = params->gamma_slices ? params->gamma_slices + 2 * (int64_t)s0 : nullptr;
    p.initial_membership = ov > 0 ? init.data() : nullptr;
    p.flags &= ~(uint32_t)(MSLM_OUTPUT_ON_DEVICE | MSLM_PROFILE | MSLM_COUNT);
    mslm_status st = api_check_desc(&sub);
    if (st != MSLM_OK) return st;
    try {
      h->g.omega_num = sub.omega_num;
      h->g.omega_den = sub.omega_den;
      build_graph(h->g, sub, h->st, h->ws);
      MSLM_HIP(hipStreamSynchronize(h->st));
    } catch (const Error &e) {
      return fail(e.status, e.what());
    } catch (const std::exception &e) {
      return fail(MSLM_ENOMEM, e.what());
    }
    std::vector<int32_t> m(nw);
    st = mslm_leiden(h.get(), &p, m.data(), nullptr);
    if (st != MSLM_OK) return st;
    std::vector<int64_t> label_of(nw, -1);   // window label -> global label
    for (int64_t v = 0; v < (int64_t)ov * N; v++) {   // communities holding overlapping copies
      int64_t &l = label_of[m[v]];
      if (l < 0) l = glob[(int64_t)s0 * N + v];
    }
    for (int64_t v = (int64_t)ov * N; v < nw; v++) {
      int64_t &l = label_of[m[v]];
      if (l < 0) l = fresh++;
      glob[(int64_t)s0 * N + v] = l;
    }
    windows++;
    prev_end = s1;
    if (s1 == T) break;
    s0 = s1 - overlap;
  }
  std::vector<int32_t> first(fresh, -1);   // labels by first appearance
  int32_t ncomm = 0;
  for (int64_t v = 0; v < n; v++) {
    int32_t &f = first[glob[v]];
    if (f < 0) f = ncomm++;
    membership[v] = f;
  }
  if (res) {
    res->windows = windows;
    res->n_communities = ncomm;
    res->ms_total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  api_clear_error();
  return MSLM_OK;
}

mslm_status mslm_get_tuning(const mslm_graph *g, mslm_tuning *out) {
  if (!g || !out) return fail(MSLM_EINVAL, "graph or tuning is NULL");
  api_tuning_to(g->tune, out);
  api_clear_error();
  return MSLM_OK;
}

mslm_status mslm_set_tuning(mslm_graph *g, const mslm_tuning *t) {
  if (!g) return fail(MSLM_EINVAL, "graph is NULL");
  Tuning tu;
  mslm_status s = api_tuning_from(t, tu);
  if (s != MSLM_OK) return s;
  g->tune = tu;
  api_clear_error();
  return MSLM_OK;
}

// One timed solve of the autotuner under tuning `tu`: its wall time (ms; the call returns once
// its outputs are on the host) and outputs.
static mslm_status tune_trial(mslm_graph *g, const SolveSpec &sp, const Tuning &tu, double &ms,
                              SolveOut &out) {
  std::vector<SolveOut> outs(1);
  try {
    const auto t0 = std::chrono::steady_clock::now();
    run_solves({&g->g}, {sp}, outs, g->st, g->ws, false, false, false, tu);
    ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  } catch (const Error &e) {
    return fail(e.status, e.what());
  } catch (const std::exception &e) {
    return fail(MSLM_ENOMEM, e.what());
  }
  out = std::move(outs[0]);
  return MSLM_OK;
}

mslm_status mslm_autotune(mslm_graph *g, const mslm_params *params, int32_t rounds,
                          mslm_tuning *out, double *ms_start, double *ms_best) {
  if (!g || !out) return fail(MSLM_EINVAL, "graph or tuning is NULL");
  if (rounds < 1 || rounds > 4) return fail(MSLM_EINVAL, "rounds must be in 1..4");
  SolveSpec sp;
  mslm_status s = api_make_spec(params, g->g.omega_num, g->g.omega_den, g->g.N, g->g.T, sp);
  if (s != MSLM_OK) return s;
  Tuning best = g->tune;
  SolveOut ref;
  double t_ref = 0, t_best = 0;
  if ((s = tune_trial(g, sp, best, t_ref, ref)) != MSLM_OK) return s;   // warm-up, reference
  if ((s = tune_trial(g, sp, best, t_best, ref)) != MSLM_OK) return s;
  const double t_start = t_best;
  auto same = [&](const SolveOut &o) {
    return o.membership == ref.membership &&
           std::memcmp(o.res.q_components, ref.res.q_components,
                       sizeof(int64_t) * (3 * g->g.T + 1)) == 0;
  };
  for (int r = 0; r < rounds; r++) {
    for (int knob = 0; knob < 5; knob++) {
      static const int64_t kCand[5][3] = {{0, 1, -1},
                                          {256, 1024, 4096},
                                          {4096, 16384, 65536},
                                          {64, 1024, 16384},
                                          {1, 4, 16}};
      for (int ci = 0; ci < 3 && kCand[knob][ci] >= 0; ci++) {
        Tuning tr = best;
        const int64_t v = kCand[knob][ci];
        int64_t *field[5] = {nullptr, &tr.latency_units, &tr.split_group_units, &tr.copy_moves,
                             nullptr};
        if (knob == 0) {
          if (tr.graphs == v) continue;
          tr.graphs = (int)v;
        } else if (knob == 4) {
          if (tr.lat_parts_max == v) continue;
          tr.lat_parts_max = (int)v;
        } else {
          if (*field[knob] == v) continue;
          *field[knob] = v;
        }
        double ms = 0;
        SolveOut o;
        if ((s = tune_trial(g, sp, tr, ms, o)) != MSLM_OK) return s;
        if (!same(o))
          return fail(MSLM_EHIP, "autotune: a tuning changed a solve's result (library bug)");
        if (ms < 0.98 * t_best) {
          best = tr;
          t_best = ms;
        }
      }
    }
  }
  g->tune = best;
  api_tuning_to(best, out);
  if (ms_start) *ms_start = t_start;
  if (ms_best) *ms_best = t_best;
  api_clear_error();
  return MSLM_OK;
}

size_t mslm_footprint_bytes(const mslm_graph_desc *d) { return footprint_estimate(d); }

static mslm_status finish_result(const GraphDev &g, const SolveSpec &sp, SolveOut &o,
                                 mslm_result *res) {
  api_finish(g, sp, o, res);
  return MSLM_OK;
}

mslm_status mslm_leiden(mslm_graph *g, const mslm_params *params, int32_t *membership,
                        mslm_result *res) {
  if (!g) return fail(MSLM_EINVAL, "graph is NULL");
  if (!membership) return fail(MSLM_EINVAL, "membership is NULL");
  SolveSpec sp;
  mslm_status s = api_make_spec(params, g->g.omega_num, g->g.omega_den, g->g.N, g->g.T, sp);
  if (s != MSLM_OK) return s;
  std::vector<SolveOut> outs(1);
  if (params->flags & MSLM_OUTPUT_ON_DEVICE) outs[0].dev_membership = membership;
  try {
    run_solves({&g->g}, {sp}, outs, g->st, g->ws, (params->flags & MSLM_PROFILE) != 0,
               (params->flags & MSLM_COUNT) != 0, false, g->tune);
  } catch (const Error &e) {
    return fail(e.status, e.what());
  } catch (const std::exception &e) {
    return fail(MSLM_ENOMEM, e.what());
  }
  if (!(params->flags & MSLM_OUTPUT_ON_DEVICE))
    memcpy(membership, outs[0].membership.data(), sizeof(int32_t) * g->g.n);
  finish_result(g->g, sp, outs[0], res);
  api_clear_error();
  return MSLM_OK;
}

mslm_status mslm_batch_leiden(mslm_graph *const *graphs, int32_t n_graphs, const mslm_solve *solves,
                              int32_t n_solves, void *hip_stream) {
  if (n_solves < 0 || n_graphs < 0 || (n_solves > 0 && (!graphs || !solves)))
    return fail(MSLM_EINVAL, "bad batch arguments");
  std::vector<SolveSpec> specs(n_solves);
  std::vector<const GraphDev *> gs(n_solves);
  for (int i = 0; i < n_solves; i++) {
    int gi = solves[i].graph;
    if (gi < 0 || gi >= n_graphs || !graphs[gi]) return fail(MSLM_EINVAL, "solve names an invalid graph");
    if (!solves[i].membership) return fail(MSLM_EINVAL, "solve has no membership buffer");
    mslm_status s = api_make_spec(&solves[i].params, graphs[gi]->g.omega_num, graphs[gi]->g.omega_den,
                                  graphs[gi]->g.N, graphs[gi]->g.T, specs[i]);
    if (s != MSLM_OK) return s;
    gs[i] = &graphs[gi]->g;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // the tuning of the graph the first solve names
  const Tuning tune = n_solves > 0 ? graphs[solves[0].graph]->tune : Tuning();
  Workspace *ws = workspace_new();
  try {
    // chunks bounded in units and entries (32-bit labels, device memory)
    const int64_t kUnits = tune.batch_units, kEntries = 400ll << 20;
    int i = 0;
    while (i < n_solves) {
      int j = i;
      int64_t un = 0, en = 0;
      while (j < n_solves && (j == i || (un + gs[j]->n <= kUnits && en + gs[j]->nnz <= kEntries))) {
        un += gs[j]->n;
        en += gs[j]->nnz;
        j++;
      }
      std::vector<const GraphDev *> cg(gs.begin() + i, gs.begin() + j);
      std::vector<SolveSpec> cs(specs.begin() + i, specs.begin() + j);
      std::vector<SolveOut> outs(j - i);
      run_solves(cg, cs, outs, st, ws, false, false, false, tune);
      for (int k = i; k < j; k++) {
        SolveOut &o = outs[k - i];
        memcpy(solves[k].membership, o.membership.data(), sizeof(int32_t) * gs[k]->n);
        finish_result(*gs[k], specs[k], o, solves[k].result);
      }
      i = j;
    }
  } catch (const Error &e) {
    workspace_free(ws);
    return fail(e.status, e.what());
  } catch (const std::exception &e) {
    workspace_free(ws);
    return fail(MSLM_ENOMEM, e.what());
  }
  workspace_free(ws);
  api_clear_error();
  return MSLM_OK;
}

}  // extern "C"
