// Host-side driver of the multislice Leiden schedule on one device stream.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include <stdexcept>
#include <utility>
#include <string>
#include <vector>

#include "../../include/mslm.h"
#include "host.hpp"

namespace mslm {

struct Error : std::runtime_error {
  mslm_status status;
  Error(mslm_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

#define MSLM_HIP(call)                                                                     \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      throw ::mslm::Error(e_ == hipErrorOutOfMemory ? MSLM_ENOMEM : MSLM_EHIP,             \
                          std::string(#call) + ": " + hipGetErrorString(e_));              \
  } while (0)

// Where device buffers come from.  By default hipMalloc/hipFree; mslm_set_allocator installs a
// caller's pair (for example a caching allocator).  A buffer remembers the pair that made it.
struct DevAlloc {
  void *(*alloc)(size_t, void *) = nullptr;   // null: hipMalloc / hipFree
  void (*release)(void *, void *) = nullptr;
  void *ctx = nullptr;
};
DevAlloc current_allocator();
void set_allocator(const DevAlloc &a);

// A fixed span of device memory that buffers are carved from while it is bound to the calling
// thread (the allocation-free entry point binds its static scratch array).  Carved buffers are
// never released; growing one abandons its old span.
struct Arena {
  char *base = nullptr;
  size_t cap = 0, used = 0, high = 0;
};
Arena *&thread_arena();

// Device bytes held by the buffers a thread allocates while an account is bound to it (the
// request loop's worker slots each keep one); a buffer settles with the account that paid.
std::atomic<int64_t> *&thread_account();

// Growable device buffer (contents are not preserved on growth).
struct Buf {
  void *p = nullptr;
  size_t cap = 0;
  DevAlloc src;        // the allocator that made p (unused for arena spans)
  bool carved = false; // p lies in an arena
  std::atomic<int64_t> *acct = nullptr;   // account charged for p
  Buf() = default;
  Buf(const Buf &) = delete;
  Buf &operator=(const Buf &) = delete;
  ~Buf() { release(); }
  void release() {
    if (p && !carved) {
      if (src.release) {
        // a caller's allocator may hand the block to other work at once: let queued kernels
        // that use it finish first
        (void)hipDeviceSynchronize();
        src.release(p, src.ctx);
      } else {
        (void)hipFree(p);
      }
      if (acct) *acct -= (int64_t)cap;
    }
    p = nullptr;
    acct = nullptr;
    cap = 0;
    carved = false;
  }
  void *ensure(size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (bytes > cap) {
      release();
      if (Arena *a = thread_arena()) {
        const size_t off = (a->used + 255) & ~(size_t)255;
        if (off > a->cap || bytes > a->cap - off)
          throw Error(MSLM_EUNSUPPORTED, "the static scratch of " + std::to_string(a->cap) +
                                             " bytes cannot hold this solve's work buffers");
        p = a->base + off;
        cap = bytes;
        carved = true;
        a->used = off + bytes;
        if (a->used > a->high) a->high = a->used;
        return p;
      }
      size_t want = bytes + bytes / 8 + 256;
      src = current_allocator();
      if (src.alloc) {
        p = src.alloc(want, src.ctx);
        if (!p) throw Error(MSLM_ENOMEM, "the installed device allocator returned NULL");
      } else {
        MSLM_HIP(hipMalloc(&p, want));
      }
      cap = want;
      acct = thread_account();
      if (acct) *acct += (int64_t)want;
    }
    return p;
  }
  template <class T>
  T *as() const { return static_cast<T *>(p); }
  void swap_with(Buf &o) {
    std::swap(p, o.p);
    std::swap(cap, o.cap);
    std::swap(src, o.src);
    std::swap(carved, o.carved);
    std::swap(acct, o.acct);
  }
  template <class T>
  T *get(int64_t n) { return static_cast<T *>(ensure(sizeof(T) * (size_t)(n > 0 ? n : 1))); }
};

// Level-0 supra-CSR of one temporal graph, resident on the device (owned by mslm_graph).
struct GraphDev {
  int32_t N = 0, T = 0;
  int64_t n = 0, nnz = 0;
  int64_t omega_num = 1, omega_den = 1;
  bool unit = true;
  int32_t maxdeg = 0;
  std::vector<int64_t> twom;     // per slice, host copy
  std::vector<int64_t> nzslice;  // per slice: units of nonzero degree
  // coupling omega^(sr) = omega * c_sr: per slice the sum over r of c_sr (bounds a copy's
  // coupling weight), and the coupling total C = sum of c_sr over ordered coupled copy pairs
  // (2mu = sum_s 2m_s + omega * C)
  std::vector<int64_t> crow;
  int64_t ctot = 0;
  bool present_only = false;   // only copies with an intra edge are coupled (CPM weight 0 else)
  Buf rp, col, w, k;
  Buf rev;   // per entry (u, x): offset of the entry (x, u) within x's row
};

struct SolveOut {
  std::vector<int32_t> membership;     // host copy (empty when written to device)
  int32_t *dev_membership = nullptr;   // optional device destination
  mslm_result res{};
};

struct Workspace;   // opaque, cached per graph or per batch

Workspace *workspace_new();
void workspace_free(Workspace *ws);
// Return the graph-build scratch (edge lists, sort keys) of a workspace to the device.
void workspace_release_build(Workspace *ws);

// Build the level-0 CSR of a graph from (host or device) edge lists.
void build_graph(GraphDev &g, const mslm_graph_desc &d, hipStream_t st, Workspace *ws);

// Run the schedule for one or more solves (each solve names a graph); results are
// bit-identical to running every solve alone.
// no_events: record no HIP events (the allocation-free entry point; phase times stay 0).
void run_solves(const std::vector<const GraphDev *> &graphs, const std::vector<SolveSpec> &specs,
                std::vector<SolveOut> &outs, hipStream_t st, Workspace *ws, bool profile,
                bool count = false, bool no_events = false, const Tuning &tune = Tuning());

}  // namespace mslm
