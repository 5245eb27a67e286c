// The opaque graph handle of the C ABI and the host-side helpers the entry points share.
#pragma once
#include <string>

#include "../../include/mslm.h"
#include "engine.hpp"
#include "host.hpp"

struct mslm_graph {
  mslm::GraphDev g;
  hipStream_t st = nullptr;
  int device = 0;                     // the device current when the graph was created
  mslm::Workspace *ws = nullptr;
  mslm::Tuning tune;                  // result-invariant execution choices (mslm_set_tuning)
  ~mslm_graph() { mslm::workspace_free(ws); }
};

namespace mslm {
// Q and the nearest double into a solve's result, then a copy to the caller's (may be NULL).
void api_finish(const GraphDev &g, const SolveSpec &sp, SolveOut &o, mslm_result *res);
}  // namespace mslm
