// Serving layer: continuous batching of forward / gradient queries against
// device-resident designs.
#include "dp_internal.h"

using dp::fail;

struct dp_server {
  dp_ctx *ctx = nullptr;
};

extern "C" {

dp_status dp_server_create(dp_ctx *ctx, size_t, dp_server **out) {
  if (!ctx || !out) return fail(DP_E_INVALID, "dp_server_create: NULL argument");
  return fail(DP_E_UNSUPPORTED, "dp_server_create: serving is not built yet");
}
dp_status dp_server_add_design(dp_server *, dp_design *, const float *, const dp_params *, int32_t *) {
  return fail(DP_E_UNSUPPORTED, "serving is not built yet");
}
dp_status dp_submit(dp_server *, const dp_query *, uint64_t *) {
  return fail(DP_E_UNSUPPORTED, "serving is not built yet");
}
dp_status dp_poll(dp_server *, uint64_t, int32_t *) {
  return fail(DP_E_UNSUPPORTED, "serving is not built yet");
}
dp_status dp_wait(dp_server *, uint64_t, double *) {
  return fail(DP_E_UNSUPPORTED, "serving is not built yet");
}
dp_status dp_server_get_stats(dp_server *, dp_server_stats *) {
  return fail(DP_E_UNSUPPORTED, "serving is not built yet");
}
void dp_server_destroy(dp_server *srv) { delete srv; }

}  // extern "C"
