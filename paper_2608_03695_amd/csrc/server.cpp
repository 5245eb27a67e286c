// Continuous-batching request loop.
//
// Requests (a temporal graph plus solve parameters) are queued by mslm_server_submit and
// admitted in arrival order while the device-memory footprint of everything admitted stays
// within the budget.  A pool of worker slots, each with its own HIP stream and workspace,
// takes every admitted request waiting at the moment it becomes free and runs the group as
// one disjoint-union solve (per-solve constants, local ids and stopping rules keep every
// result identical to a plain mslm_create + mslm_leiden).  Requests arriving while other
// groups are on the device join the next free slot, so their work overlaps on the GPU.
// Every request pays its own upload and supra-CSR build: nothing is cached across requests.
#include "server.hpp"

#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.hpp"

using namespace mslm;

namespace mslm {
mslm_status api_check_desc(const mslm_graph_desc *d);
mslm_status api_make_spec(const mslm_params *p, int64_t on, int64_t od, SolveSpec &sp);
void api_finish(const GraphDev &g, const SolveSpec &sp, SolveOut &o, mslm_result *res);
mslm_status api_fail(mslm_status s, const std::string &m);
}  // namespace mslm

namespace {

using Clock = std::chrono::steady_clock;

// Requests grouped into one run: bounded so that a group's latency stays that of a few solves.
constexpr int kMaxGroup = 64;
constexpr int64_t kMaxGroupUnits = 8ll << 20;

struct Request {
  uint64_t ticket = 0;
  int32_t N = 0, T = 0;
  std::vector<int64_t> off;
  std::vector<int32_t> src, dst, w;
  bool weighted = false;
  int64_t omega_num = 1, omega_den = 1;
  SolveSpec spec;
  size_t footprint = 0;
  Clock::time_point t_submit;
  // result
  bool done = false;
  mslm_status status = MSLM_OK;
  std::string err;
  std::vector<int32_t> membership;
  mslm_result res{};
  double latency = 0.0;
};

}  // namespace

struct mslm_server {
  size_t budget = 0;
  int device = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;
  size_t admitted_bytes = 0;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::vector<std::thread> workers;
};

namespace {

void finish_group(mslm_server *s, std::vector<std::shared_ptr<Request>> &grp, mslm_status st,
                  const std::string &err) {
  const Clock::time_point now = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  for (auto &r : grp) {
    r->done = true;
    r->status = st;
    r->err = err;
    r->latency = std::chrono::duration<double>(now - r->t_submit).count();
    s->admitted_bytes -= r->footprint;
  }
  s->cv_done.notify_all();
  s->cv_work.notify_all();
}

// graphs: the slot's pool of device graphs, reused across groups so that steady-state
// serving allocates and frees no device memory (each build overwrites its graph)
void run_group(mslm_server *s, std::vector<std::shared_ptr<Request>> &grp, hipStream_t st,
               Workspace *ws, std::vector<std::unique_ptr<GraphDev>> &graphs) {
  const size_t G = grp.size();
  while (graphs.size() < G) graphs.emplace_back(new GraphDev());
  try {
    for (size_t i = 0; i < G; i++) {
      Request &r = *grp[i];
      mslm_graph_desc d{};
      d.n_nodes = r.N;
      d.n_slices = r.T;
      d.slice_offsets = r.off.data();
      d.src = r.src.data();
      d.dst = r.dst.data();
      d.weight = r.weighted ? r.w.data() : nullptr;
      d.omega_num = r.omega_num;
      d.omega_den = r.omega_den;
      d.flags = 0;
      graphs[i]->omega_num = r.omega_num;
      graphs[i]->omega_den = r.omega_den;
      build_graph(*graphs[i], d, st, ws);
    }
    std::vector<const GraphDev *> gp(G);
    std::vector<SolveSpec> specs(G);
    for (size_t i = 0; i < G; i++) {
      gp[i] = graphs[i].get();
      specs[i] = grp[i]->spec;
    }
    std::vector<SolveOut> outs(G);
    run_solves(gp, specs, outs, st, ws, false);
    for (size_t i = 0; i < G; i++) {
      grp[i]->membership.swap(outs[i].membership);
      api_finish(*graphs[i], specs[i], outs[i], &grp[i]->res);
    }
    finish_group(s, grp, MSLM_OK, "");
  } catch (const Error &e) {
    (void)hipStreamSynchronize(st);
    finish_group(s, grp, e.status, e.what());
  } catch (const std::exception &e) {
    (void)hipStreamSynchronize(st);
    finish_group(s, grp, MSLM_ENOMEM, e.what());
  }
}

void worker_main(mslm_server *s) {
  (void)hipSetDevice(s->device);
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
  Workspace *ws = workspace_new();
  std::vector<std::unique_ptr<GraphDev>> graphs;
  for (;;) {
    std::vector<std::shared_ptr<Request>> grp;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      // admit in arrival order while the head fits next to what is already admitted
      s->cv_work.wait(lk, [&] {
        return s->stop || (!s->queue.empty() &&
                           s->admitted_bytes + s->queue.front()->footprint <= s->budget);
      });
      if (s->stop) break;
      int64_t units = 0;
      while (!s->queue.empty() && (int)grp.size() < kMaxGroup) {
        auto &r = s->queue.front();
        const int64_t n = (int64_t)r->N * r->T;
        if (!grp.empty() && (units + n > kMaxGroupUnits ||
                             s->admitted_bytes + r->footprint > s->budget))
          break;
        units += n;
        s->admitted_bytes += r->footprint;
        grp.push_back(r);
        s->queue.pop_front();
      }
    }
    if (st == nullptr) {
      finish_group(s, grp, MSLM_EHIP, "server stream could not be created");
      continue;
    }
    run_group(s, grp, st, ws, graphs);
  }
  graphs.clear();
  workspace_free(ws);
  if (st) (void)hipStreamDestroy(st);
}

}  // namespace

extern "C" {

mslm_status mslm_server_create(size_t hbm_budget_bytes, int32_t max_slots, mslm_server **out) {
  if (!out) return api_fail(MSLM_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 16) return api_fail(MSLM_EINVAL, "max_slots must be in 1..16");
  if (hbm_budget_bytes == 0) return api_fail(MSLM_EINVAL, "hbm_budget_bytes must be > 0");
  std::unique_ptr<mslm_server> s(new mslm_server());
  s->budget = hbm_budget_bytes;
  if (hipGetDevice(&s->device) != hipSuccess) return api_fail(MSLM_EHIP, "no HIP device");
  try {
    for (int i = 0; i < max_slots; i++) s->workers.emplace_back(worker_main, s.get());
  } catch (const std::exception &e) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    return api_fail(MSLM_ENOMEM, e.what());
  }
  *out = s.release();
  return MSLM_OK;
}

mslm_status mslm_server_submit(mslm_server *s, const mslm_graph_desc *d, const mslm_params *p,
                               uint64_t *ticket) {
  if (!s || !ticket) return api_fail(MSLM_EINVAL, "server or ticket is NULL");
  mslm_status rc = api_check_desc(d);
  if (rc != MSLM_OK) return rc;
  if (d->flags & MSLM_INPUT_ON_DEVICE)
    return api_fail(MSLM_EINVAL, "the server takes host edge lists only");
  auto r = std::make_shared<Request>();
  rc = api_make_spec(p, d->omega_num, d->omega_den, r->spec);
  if (rc != MSLM_OK) return rc;
  r->footprint = mslm_footprint_bytes(d);
  if (r->footprint > s->budget)
    return api_fail(MSLM_EINVAL, "request footprint exceeds the server's memory budget");
  r->N = d->n_nodes;
  r->T = d->n_slices;
  r->off.assign(d->slice_offsets, d->slice_offsets + d->n_slices + 1);
  const int64_t E = r->off[d->n_slices];
  r->src.assign(d->src, d->src + E);
  r->dst.assign(d->dst, d->dst + E);
  r->weighted = d->weight != nullptr;
  if (r->weighted) r->w.assign(d->weight, d->weight + E);
  r->omega_num = d->omega_num;
  r->omega_den = d->omega_den;
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    s->tickets[r->ticket] = r;
    s->queue.push_back(r);
  }
  s->cv_work.notify_one();
  *ticket = r->ticket;
  return MSLM_OK;
}

mslm_status mslm_server_wait(mslm_server *s, uint64_t ticket, int32_t timeout_ms,
                             int32_t *membership, mslm_result *res, double *latency_s) {
  if (!s) return api_fail(MSLM_EINVAL, "server is NULL");
  std::shared_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return api_fail(MSLM_EINVAL, "unknown ticket");
    r = it->second;
    auto ready = [&] { return r->done; };
    if (timeout_ms < 0) {
      s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
      return api_fail(MSLM_EBUSY, "result not ready");
    }
    s->tickets.erase(it);
  }
  if (r->status != MSLM_OK) return api_fail(r->status, r->err);
  if (membership) memcpy(membership, r->membership.data(), sizeof(int32_t) * r->membership.size());
  if (res) *res = r->res;
  if (latency_s) *latency_s = r->latency;
  return MSLM_OK;
}

void mslm_server_destroy(mslm_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto &t : s->workers) t.join();
  delete s;
}

}  // extern "C"
