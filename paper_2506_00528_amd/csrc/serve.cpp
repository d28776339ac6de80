// serve.cpp -- continuous-batching server (placeholder until it lands).
#include "tq_runtime.h"

using namespace tqr;

extern "C" {

int tq_serve_create(const tq_db *, const tq_serve_cfg *, tq_server **out) {
  clear_error();
  if (out) *out = nullptr;
  return fail(TQ_ERR_STATE, "serving is not available in this build");
}
int tq_serve_submit(tq_server *, const uint32_t *, int, int, uint64_t *) {
  return fail(TQ_ERR_STATE, "serving is not available in this build");
}
int tq_serve_poll(tq_server *, uint64_t, int32_t *, int32_t *, tq_req_stats *) {
  return fail(TQ_ERR_STATE, "serving is not available in this build");
}
int tq_serve_wait(tq_server *, uint64_t, int, int32_t *, int32_t *, tq_req_stats *) {
  return fail(TQ_ERR_STATE, "serving is not available in this build");
}
int tq_serve_cancel(tq_server *, uint64_t) { return fail(TQ_ERR_STATE, "serving is not available in this build"); }
int tq_serve_stats(tq_server *, uint64_t *, uint64_t *, uint64_t *, uint64_t *) {
  return fail(TQ_ERR_STATE, "serving is not available in this build");
}
int tq_serve_destroy(tq_server *) { return TQ_OK; }

}  // extern "C"
