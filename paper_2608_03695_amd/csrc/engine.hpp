// Host-side driver of the multislice Leiden schedule on one device stream.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <stdexcept>
#include <utility>
#include <string>
#include <vector>

#include "../../include/mslm.h"

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

// Growable device buffer (contents are not preserved on growth).
struct Buf {
  void *p = nullptr;
  size_t cap = 0;
  Buf() = default;
  Buf(const Buf &) = delete;
  Buf &operator=(const Buf &) = delete;
  ~Buf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  void *ensure(size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (bytes > cap) {
      release();
      size_t want = bytes + bytes / 8 + 256;
      MSLM_HIP(hipMalloc(&p, want));
      cap = want;
    }
    return p;
  }
  template <class T>
  T *as() const { return static_cast<T *>(p); }
  void swap_with(Buf &o) {
    std::swap(p, o.p);
    std::swap(cap, o.cap);
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
  Buf rp, col, w, k;
};

struct SolveSpec {
  int64_t p = 1, q = 1, a = 1, b = 1;   // reduced gamma = p/q, omega = a/b
  int32_t max_levels = 32, max_iterations = 2, max_sweeps = 32;
  uint64_t seed = 0;
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
void run_solves(const std::vector<const GraphDev *> &graphs, const std::vector<SolveSpec> &specs,
                std::vector<SolveOut> &outs, hipStream_t st, Workspace *ws, bool profile,
                bool count = false);

}  // namespace mslm
