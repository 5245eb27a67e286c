// Continuous-batching request loop.
#include "server.hpp"

extern "C" {
mslm_status mslm_server_create(size_t, int32_t, mslm_server **out) {
  if (out) *out = nullptr;
  return MSLM_EUNSUPPORTED;
}
mslm_status mslm_server_submit(mslm_server *, const mslm_graph_desc *, const mslm_params *,
                               uint64_t *) {
  return MSLM_EUNSUPPORTED;
}
mslm_status mslm_server_wait(mslm_server *, uint64_t, int32_t, int32_t *, mslm_result *, double *) {
  return MSLM_EUNSUPPORTED;
}
void mslm_server_destroy(mslm_server *) {}
}
