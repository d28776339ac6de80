// batched.cpp -- the batched search path (placeholder until its kernel lands).
#include "tq_runtime.h"

namespace tqr {

struct BatchedState {};

int choose_path(tq_db *, int requested, int, int) {
  return requested == TQ_PATH_BATCHED ? TQ_PATH_BATCHED : TQ_PATH_PLAIN;
}

int search_batched(tq_db *, const uint32_t *, int, int, int32_t *, int32_t *, const tq_search_opts *,
                   hipStream_t) {
  return fail(TQ_ERR_STATE, "the batched path is not available in this build");
}

void batched_release(tq_db *db) {
  delete db->batched;
  db->batched = nullptr;
}

}  // namespace tqr
