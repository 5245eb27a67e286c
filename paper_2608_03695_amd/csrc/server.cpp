// Continuous-batching request loop.
//
// Requests (a temporal graph plus solve parameters) are queued by mslm_server_submit and
// admitted in arrival order.  A pool of worker slots, each with its own workspace (and its own
// HIP stream unless the caller gave one), takes every admitted request waiting at the moment it
// becomes free and runs the group as one disjoint-union solve (per-solve constants, local ids
// and stopping rules keep every result identical to a plain mslm_create + mslm_leiden).
// Requests arriving while other groups are on the device join the next free slot, so their
// work overlaps on the GPU.  Every request pays its own upload and supra-CSR build: nothing is
// cached across requests.
//
// Memory: a slot keeps its device buffers between groups (so steady serving allocates
// nothing), and those bytes count against the budget.  The budget covers, for every slot, the
// larger of what it holds and the footprint estimate of the group it runs; an idle slot whose
// holdings keep the queue's head out gives its buffers back.
#include "server.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
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
#include "handles.hpp"

using namespace mslm;

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
  std::vector<int32_t> coupling;   // T*T, empty: ordinal
  uint32_t couple_flags = 0;       // MSLM_COUPLE_PRESENT
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

namespace {
struct Slot {
  std::atomic<int64_t> held{0};   // device bytes its buffers hold (its thread's account)
  size_t charge = 0;              // what it counts against the budget (under the server lock)
};
}  // namespace

struct mslm_server {
  size_t budget = 0;
  int device = 0;
  hipStream_t user_stream = nullptr;   // the caller's stream for every slot, or null
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;
  std::vector<std::unique_ptr<Slot>> slots;
  size_t charged = 0;        // sum of the slots' charges (never above the budget)
  size_t peak_charged = 0;
  size_t peak_held = 0;      // largest sum of the slots' held bytes seen at a group's start or end
  int waiters = 0;           // threads inside mslm_server_wait
  uint64_t next_ticket = 1;
  bool stop = false;
  std::vector<std::thread> workers;
};

namespace {

void set_charge(mslm_server *s, Slot &slot, size_t c) {
  s->charged = s->charged - slot.charge + c;
  slot.charge = c;
  s->peak_charged = std::max(s->peak_charged, s->charged);
}

void sample_held(mslm_server *s) {
  size_t h = 0;
  for (auto &sl : s->slots) h += (size_t)std::max<int64_t>(0, sl->held.load());
  s->peak_held = std::max(s->peak_held, h);
}

void finish_one(mslm_server *s, Request &r, mslm_status st, const std::string &err,
                Clock::time_point now) {
  r.done = true;
  r.status = st;
  r.err = err;
  r.latency = std::chrono::duration<double>(now - r.t_submit).count();
  (void)s;
}

// graphs: the slot's pool of device graphs, reused across groups so that steady-state
// serving allocates and frees no device memory (each build overwrites its graph)
void solve_group(std::vector<std::shared_ptr<Request>> &grp, hipStream_t st, Workspace *ws,
                 std::vector<std::unique_ptr<GraphDev>> &graphs) {
  const size_t G = grp.size();
  while (graphs.size() < G) graphs.emplace_back(new GraphDev());
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
    d.flags = r.couple_flags;
    d.coupling = r.coupling.empty() ? nullptr : r.coupling.data();
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
}

// Run a group; if the union fails, run its requests one at a time so that a request's own
// error never becomes another request's result.
void run_group(mslm_server *s, std::vector<std::shared_ptr<Request>> &grp, hipStream_t st,
               Workspace *ws, std::vector<std::unique_ptr<GraphDev>> &graphs) {
  std::vector<mslm_status> status(grp.size(), MSLM_OK);
  std::vector<std::string> errs(grp.size());
  auto attempt = [&](std::vector<std::shared_ptr<Request>> &g, mslm_status &rc, std::string &msg) {
    try {
      solve_group(g, st, ws, graphs);
      rc = MSLM_OK;
    } catch (const Error &e) {
      (void)hipStreamSynchronize(st);
      rc = e.status;
      msg = e.what();
    } catch (const std::exception &e) {
      (void)hipStreamSynchronize(st);
      rc = MSLM_ENOMEM;
      msg = e.what();
    }
  };
  mslm_status rc;
  std::string msg;
  attempt(grp, rc, msg);
  if (rc != MSLM_OK && grp.size() > 1) {
    for (size_t i = 0; i < grp.size(); i++) {
      std::vector<std::shared_ptr<Request>> one{grp[i]};
      attempt(one, status[i], errs[i]);
    }
  } else {
    for (size_t i = 0; i < grp.size(); i++) {
      status[i] = rc;
      errs[i] = msg;
    }
  }
  const Clock::time_point now = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  for (size_t i = 0; i < grp.size(); i++) finish_one(s, *grp[i], status[i], errs[i], now);
  s->cv_done.notify_all();
}

void worker_main(mslm_server *s, Slot *slot) {
  (void)hipSetDevice(s->device);
  thread_account() = &slot->held;
  hipStream_t own = nullptr, st = s->user_stream;
  if (!st) {
    if (hipStreamCreateWithFlags(&own, hipStreamNonBlocking) != hipSuccess) own = nullptr;
    st = own;
  }
  Workspace *ws = workspace_new();
  std::vector<std::unique_ptr<GraphDev>> graphs;
  auto trim = [&] {   // give every device buffer back (called without the lock)
    graphs.clear();
    workspace_free(ws);
    ws = workspace_new();
  };
  for (;;) {
    std::vector<std::shared_ptr<Request>> grp;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        if (s->stop) break;
        if (s->queue.empty()) {
          s->cv_work.wait(lk);
          continue;
        }
        const size_t held = (size_t)std::max<int64_t>(0, slot->held.load());
        const size_t others = s->charged - slot->charge;
        size_t need = 0;
        int64_t units = 0;
        while (!s->queue.empty() && (int)grp.size() < kMaxGroup) {
          auto &r = s->queue.front();
          const int64_t n = (int64_t)r->N * r->T;
          const size_t need2 = need + r->footprint;
          if (others + std::max(held, need2) > s->budget) break;
          if (!grp.empty() && units + n > kMaxGroupUnits) break;
          need = need2;
          units += n;
          grp.push_back(r);
          s->queue.pop_front();
        }
        if (!grp.empty()) {
          set_charge(s, *slot, std::max(held, need));
          sample_held(s);
          break;
        }
        if (held > 0) {   // this slot's idle buffers keep the head out: give them back
          lk.unlock();
          trim();
          lk.lock();
          set_charge(s, *slot, (size_t)std::max<int64_t>(0, slot->held.load()));
          s->cv_work.notify_all();
          continue;
        }
        s->cv_work.wait(lk);
      }
      if (s->stop && grp.empty()) break;
    }
    if (st == nullptr) {
      std::lock_guard<std::mutex> lk(s->mu);
      for (auto &r : grp) finish_one(s, *r, MSLM_EHIP, "server stream could not be created", Clock::now());
      s->cv_done.notify_all();
      continue;
    }
    run_group(s, grp, st, ws, graphs);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      sample_held(s);
      set_charge(s, *slot, (size_t)std::max<int64_t>(0, slot->held.load()));
    }
    s->cv_work.notify_all();
  }
  graphs.clear();
  workspace_free(ws);
  thread_account() = nullptr;
  if (own) (void)hipStreamDestroy(own);
}

}  // namespace

extern "C" {

mslm_status mslm_server_create(size_t hbm_budget_bytes, int32_t max_slots, void *hip_stream,
                               mslm_server **out) {
  if (!out) return api_fail(MSLM_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 16) return api_fail(MSLM_EINVAL, "max_slots must be in 1..16");
  if (hbm_budget_bytes == 0) return api_fail(MSLM_EINVAL, "hbm_budget_bytes must be > 0");
  std::unique_ptr<mslm_server> s(new mslm_server());
  s->budget = hbm_budget_bytes;
  s->user_stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&s->device) != hipSuccess) return api_fail(MSLM_EHIP, "no HIP device");
  for (int i = 0; i < max_slots; i++) s->slots.emplace_back(new Slot());
  try {
    for (int i = 0; i < max_slots; i++) s->workers.emplace_back(worker_main, s.get(), s->slots[i].get());
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
  rc = api_make_spec(p, d->omega_num, d->omega_den, d->n_nodes, d->n_slices, r->spec);
  if (rc != MSLM_OK) return rc;
  rc = api_check_headroom(d, r->spec);   // a request that passes cannot fail on head-room later
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
  if (d->coupling) r->coupling.assign(d->coupling, d->coupling + (size_t)d->n_slices * d->n_slices);
  r->couple_flags = d->flags & MSLM_COUPLE_PRESENT;
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
    s->waiters++;
    bool got = true;
    if (timeout_ms < 0) s->cv_done.wait(lk, ready);
    else got = s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    s->waiters--;
    s->cv_done.notify_all();   // a destroy may be waiting for the last waiter to leave
    if (!got) return api_fail(MSLM_EBUSY, "result not ready");
    s->tickets.erase(r->ticket);
  }
  if (r->status != MSLM_OK) return api_fail(r->status, r->err);
  if (membership) memcpy(membership, r->membership.data(), sizeof(int32_t) * r->membership.size());
  if (res) *res = r->res;
  if (latency_s) *latency_s = r->latency;
  return MSLM_OK;
}

mslm_status mslm_server_memory(mslm_server *s, size_t *held_bytes, size_t *peak_held_bytes,
                               size_t *peak_charged_bytes) {
  if (!s) return api_fail(MSLM_EINVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  size_t h = 0;
  for (auto &sl : s->slots) h += (size_t)std::max<int64_t>(0, sl->held.load());
  if (held_bytes) *held_bytes = h;
  if (peak_held_bytes) *peak_held_bytes = std::max(s->peak_held, h);
  if (peak_charged_bytes) *peak_charged_bytes = s->peak_charged;
  return MSLM_OK;
}

void mslm_server_destroy(mslm_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    // requests still queued end with an error; groups already running finish normally
    const Clock::time_point now = Clock::now();
    for (auto &r : s->queue) finish_one(s, *r, MSLM_EINVAL, "server destroyed before the request ran", now);
    s->queue.clear();
  }
  s->cv_work.notify_all();
  s->cv_done.notify_all();
  for (auto &t : s->workers) t.join();
  {
    // threads already inside mslm_server_wait leave before the server goes away
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.notify_all();
    s->cv_done.wait(lk, [&] { return s->waiters == 0; });
  }
  delete s;
}

}  // extern "C"
