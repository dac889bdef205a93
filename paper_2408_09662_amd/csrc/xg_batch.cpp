// Persistent multi-program launch, HIP graph capture and autotuning.
#include <cstring>

#include "xg_internal.h"
#include "xg_program.h"

using namespace xg;

extern "C" {

xg_status xg_batch_create(xg_program* const*, int32_t, const xg_options*, xg_batch** out) {
  if (out) *out = nullptr;
  set_error("batch: not implemented yet");
  return XG_EUNSUPPORTED;
}
void xg_batch_free(xg_batch*) {}
xg_status xg_batch_workspace_bytes(xg_batch*, const int64_t*, size_t*) { return XG_EUNSUPPORTED; }
xg_status xg_batch_eval(xg_batch*, const xg_batch_args*, void*, void*) { return XG_EUNSUPPORTED; }
xg_status xg_graph_capture_eval(xg_program*, int64_t, const void* const*, const int64_t*,
                                void* const*, const int64_t*, void*, void*, xg_graph** out) {
  if (out) *out = nullptr;
  return XG_EUNSUPPORTED;
}
xg_status xg_graph_capture_batch(xg_batch*, const xg_batch_args*, void*, void*, xg_graph** out) {
  if (out) *out = nullptr;
  return XG_EUNSUPPORTED;
}
xg_status xg_graph_launch(xg_graph*, void*) { return XG_EUNSUPPORTED; }
void xg_graph_free(xg_graph*) {}
xg_status xg_autotune(xg_program*, int64_t, const void* const*, const int64_t*, void* const*,
                      const int64_t*, void*, size_t, void*, xg_options*) {
  return XG_EUNSUPPORTED;
}

}  // extern "C"
