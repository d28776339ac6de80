// tq_runtime.h -- host-side runtime internals of the library (not public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <mutex>
#include <unordered_map>

#include "tq.h"
#include "tq_internal.h"

namespace tqr {

// --- errors --------------------------------------------------------------
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char *what);
void clear_error();
int log_level();

// --- devices ---------------------------------------------------------------
struct DevCtx {
  bool ready = false;
  int num_cu = 0;
  int *flags = nullptr;  // sticky device error flags (bit 0: non-finite encode input)
};
int current_device(int *dev);
int device_ctx(int dev, DevCtx **out);

class DeviceGuard {
 public:
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
  DeviceGuard(const DeviceGuard &) = delete;
  DeviceGuard &operator=(const DeviceGuard &) = delete;

 private:
  int prev_ = -1;
  bool switched_ = false;
};

// --- kernel timing ----------------------------------------------------------
enum TimingFamily { kTimePlain = 0, kTimeBatched = 1, kTimeMasked = 2, kTimeSparse = 3, kTimeFamilies = 4 };

bool timing_enabled();

// Brackets one kernel launch with HIP events on stream `s` when timing is on.
class TimedLaunch {
 public:
  // `allow` = false leaves the launch untimed whatever tq_timing_enable says.
  TimedLaunch(int family, hipStream_t s, bool allow = true);
  ~TimedLaunch();
  TimedLaunch(const TimedLaunch &) = delete;
  TimedLaunch &operator=(const TimedLaunch &) = delete;

 private:
  int family_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};

// --- device memory ------------------------------------------------------------
// Every device allocation of the library goes through these: the bytes held
// are counted, and an allocation that would take them past the limit set by
// tq_set_device_limit fails with hipErrorOutOfMemory before hipMalloc runs.
hipError_t dev_malloc_raw(void **p, size_t bytes);
void dev_free(void *p);
template <class T>
hipError_t dev_malloc(T **p, size_t bytes) {
  return dev_malloc_raw(reinterpret_cast<void **>(p), bytes);
}

// --- scratch -----------------------------------------------------------------
struct Scratch {
  void *p = nullptr;
  size_t bytes = 0;
};
using ScratchMap = std::unordered_map<hipStream_t, Scratch>;
// A caller-provided device buffer used in place of scratch_get().
struct ScratchSpan {
  void *p = nullptr;
  size_t bytes = 0;
};
// Buffer of at least `bytes` private to (owner, stream); growing it waits for
// the stream first.  The owner's mutex must be held.
int scratch_get(ScratchMap &map, hipStream_t s, size_t bytes, void **out);
void scratch_free_all(ScratchMap &map);

int count_bad_codes(const uint32_t *codes, int64_t n, int d, int x, hipStream_t s, unsigned long long *bad);

struct BatchedState;  // batched.cpp

}  // namespace tqr

// The database handle of the public ABI.
struct tq_db {
  int device = 0;
  int num_cu = 0;
  tqi::DbDev dev{};
  size_t bytes = 0;
  std::mutex mu;  // guards scratch and batched state during enqueue
  tqr::ScratchMap scratch;
  tqr::BatchedState *batched = nullptr;
};

namespace tqr {

// search.cpp
int default_plain_grid(const tq_db *db);
// engine: TQ_ENGINE_SPARSE takes the index-list scan, TQ_ENGINE_AUTO takes it
// where sparse_preferred(), anything else the bit-plane scan.
// With `ext` the scratch comes from that buffer (nothing is allocated and no
// launch is timed); TQ_ERR_INVALID if one query's need does not fit in it.
// metric: TQ_METRIC_DELTA or TQ_METRIC_L2 (not with the index-list engine).
int search_plain(tq_db *db, const uint32_t *qcodes, int nq, int k, int32_t *ids, int32_t *scores, int grid,
                 int engine, hipStream_t s, const ScratchSpan *ext = nullptr, int metric = TQ_METRIC_DELTA);
int search_masked(tq_db *db, const float *Q, int nq, int k, int32_t *ids, float *scores, int grid, hipStream_t s);

// batched.cpp
int choose_path(tq_db *db, int requested, int nq, int k);
int search_batched(tq_db *db, const uint32_t *qcodes, int nq, int k, int32_t *ids, int32_t *scores,
                   const tq_search_opts *opts, hipStream_t s);
void batched_release(tq_db *db);
int autotune(tq_db *db, int nq_max, const int *ks, int nks, hipStream_t s, int verbose);
int default_engine(int k, int nq);

}  // namespace tqr
