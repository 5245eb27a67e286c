// Allocation-free solve: mslm_leiden whose work buffers live in a static device array.
//
// For callers that cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid allocation).  The array below is the only device memory the
// call touches besides the resident graph and the caller's outputs; each GPU the library runs
// on holds its own copy from module load until the process ends.  Host code never passes the
// array's name as an address: on the first call on a device (with that device current) the
// device address is taken with hipGetSymbolAddress and kept per device.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mslm.h"
#include "engine.hpp"
#include "handles.hpp"

using namespace mslm;

namespace {

constexpr size_t kScratchBytes = (size_t)MSLM_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_dev_mu[kMaxDevices];       // one allocation-free call at a time per device
void *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per device

// Device address of this device's scratch array (the device must be current).
mslm_status scratch_address(int dev, void **out) {
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return api_fail(MSLM_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                     hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MSLM_OK;
}

}  // namespace

extern "C" mslm_status mslm_leiden_static(mslm_graph *g, const mslm_params *params,
                                          int32_t *membership, mslm_result *res) {
  if (!g) return api_fail(MSLM_EINVAL, "graph is NULL");
  if (!membership) return api_fail(MSLM_EINVAL, "membership is NULL");
  if (params && (params->flags & MSLM_PROFILE))
    return api_fail(MSLM_EINVAL, "MSLM_PROFILE records HIP events, which this entry point does not create");
  SolveSpec sp;
  mslm_status s = api_make_spec(params, g->g.omega_num, g->g.omega_den, g->g.N, g->g.T, sp);
  if (s != MSLM_OK) return s;
  const size_t need = solve_scratch_estimate(g->g.n, g->g.nnz);
  if (need > kScratchBytes)
    return api_fail(MSLM_EUNSUPPORTED, "this graph's solve needs about " + std::to_string(need) +
                                           " bytes of work buffers; the static scratch holds " +
                                           std::to_string(kScratchBytes));
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return api_fail(MSLM_EHIP, "no usable HIP device");
  if (dev != g->device)
    return api_fail(MSLM_EINVAL, "the graph's device must be current");
  std::lock_guard<std::mutex> lk(g_dev_mu[dev]);
  void *base = nullptr;
  s = scratch_address(dev, &base);
  if (s != MSLM_OK) return s;
  Arena arena;
  arena.base = static_cast<char *>(base);
  arena.cap = kScratchBytes;
  Arena *&bound = thread_arena();
  bound = &arena;
  Workspace *ws = workspace_new();   // a host object; its buffers are carved from the arena
  std::vector<SolveOut> outs(1);
  if (params->flags & MSLM_OUTPUT_ON_DEVICE) outs[0].dev_membership = membership;
  mslm_status rc = MSLM_OK;
  std::string msg;
  try {
    run_solves({&g->g}, {sp}, outs, g->st, ws, false, (params->flags & MSLM_COUNT) != 0,
               /*no_events=*/true, g->tune);
  } catch (const Error &e) {
    rc = e.status;
    msg = e.what();
  } catch (const std::exception &e) {
    rc = MSLM_ENOMEM;
    msg = e.what();
  }
  // work queued before an error may still use the array: let it end before the next call
  if (rc != MSLM_OK) (void)hipStreamSynchronize(g->st);
  workspace_free(ws);   // carved buffers: nothing to release
  bound = nullptr;
  if (rc != MSLM_OK) return api_fail(rc, msg);
  if (!(params->flags & MSLM_OUTPUT_ON_DEVICE))
    std::memcpy(membership, outs[0].membership.data(), sizeof(int32_t) * g->g.n);
  api_finish(g->g, sp, outs[0], res);
  api_clear_error();
  return MSLM_OK;
}
