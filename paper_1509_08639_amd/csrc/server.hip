// Serving loop (continuous batching) of the C ABI.
#include <hip/hip_runtime.h>

#include "../../include/ymine.h"
#include "ym_runtime.h"

using namespace ym;

extern "C" {

ym_status ym_server_start(ym_ctx *, const ym_lexicon *, const ym_params *, const ym_server_opts *, ym_server **out) {
  if (out) *out = nullptr;
  return fail(YM_EINVAL, "serving loop not available in this build");
}
ym_status ym_submit(ym_server *, const ym_batch *, uint64_t *) { return fail(YM_EINVAL, "no server"); }
ym_status ym_poll(ym_server *, uint64_t, int64_t, ym_result **) { return fail(YM_EINVAL, "no server"); }
ym_status ym_cancel(ym_server *, uint64_t) { return fail(YM_EINVAL, "no server"); }
ym_status ym_server_stop(ym_server *) { return fail(YM_EINVAL, "no server"); }
ym_status ym_server_stats(const ym_server *, int64_t *, int64_t *, int64_t *) { return fail(YM_EINVAL, "no server"); }

}  // extern "C"
