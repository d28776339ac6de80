// api.cpp -- the C ABI of include/tq.h: argument checks, device contexts,
// database lifetime, search dispatch and kernel timing.  All GPU work is done
// by the kernels in the .hip files; this file only validates and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "tq.h"
#include "tq_internal.h"
#include "tq_runtime.h"

// ---------------------------------------------------------------------------
// errors and logging
// ---------------------------------------------------------------------------

namespace tqr {

static thread_local std::string t_last_error;

int log_level() {
  static int level = [] {
    const char *e = std::getenv("TQ_LOG");
    return e ? std::atoi(e) : 0;
  }();
  return level;
}

int fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_last_error = buf;
  if (log_level() >= 1) std::fprintf(stderr, "[tq] %s: %s\n", tq_status_str(code), buf);
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(e == hipErrorOutOfMemory ? TQ_ERR_NOMEM : TQ_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { t_last_error.clear(); }

// ---------------------------------------------------------------------------
// per-device context
// ---------------------------------------------------------------------------

namespace {
constexpr int kMaxDevices = 64;
DevCtx g_dev[kMaxDevices];
std::mutex g_dev_mu;
}  // namespace

int current_device(int *dev) {
  hipError_t e = hipGetDevice(dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (*dev < 0 || *dev >= kMaxDevices) return fail(TQ_ERR_DEVICE, "device index %d out of range", *dev);
  return TQ_OK;
}

int device_ctx(int dev, DevCtx **out) {
  std::lock_guard<std::mutex> g(g_dev_mu);
  DevCtx &c = g_dev[dev];
  if (!c.ready) {
    int cu = 0;
    hipError_t e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    e = dev_malloc(&c.flags, 256);
    if (e != hipSuccess) return hip_fail(e, "device allocation (flags)");
    e = hipMemset(c.flags, 0, 256);
    if (e != hipSuccess) return hip_fail(e, "hipMemset(flags)");
    c.num_cu = cu;
    c.ready = true;
  }
  *out = &c;
  return TQ_OK;
}

DeviceGuard::DeviceGuard(int dev) {
  if (hipGetDevice(&prev_) == hipSuccess && prev_ != dev) {
    if (hipSetDevice(dev) == hipSuccess) switched_ = true;
  }
}
DeviceGuard::~DeviceGuard() {
  if (switched_) (void)hipSetDevice(prev_);
}

// ---------------------------------------------------------------------------
// kernel timing (HIP events around scan launches, on the launch stream)
// ---------------------------------------------------------------------------

namespace {
struct Timing {
  std::mutex mu;
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[kTimeFamilies];
  double total_ms[kTimeFamilies] = {};
  int64_t launches[kTimeFamilies] = {};
};
Timing g_timing;
std::atomic<int> g_timing_on{0};

hipEvent_t pooled_event() {
  if (!g_timing.pool.empty()) {
    hipEvent_t e = g_timing.pool.back();
    g_timing.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool timing_enabled() { return g_timing_on.load(std::memory_order_relaxed) != 0; }

// Timing is best effort: a pair whose events could not be had or recorded
// is not timed, and its events go back to the pool.
TimedLaunch::TimedLaunch(int family, hipStream_t s, bool allow) : family_(family), s_(s) {
  if (!allow || !g_timing_on.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> g(g_timing.mu);
  hipEvent_t a = pooled_event(), b = pooled_event();
  if (a && b && hipEventRecord(a, s_) == hipSuccess) {
    a_ = a;
    b_ = b;
    return;
  }
  if (a) g_timing.pool.push_back(a);
  if (b) g_timing.pool.push_back(b);
}

TimedLaunch::~TimedLaunch() {
  if (!a_ || !b_) return;
  std::lock_guard<std::mutex> g(g_timing.mu);
  if (hipEventRecord(b_, s_) == hipSuccess) {
    g_timing.pending[family_].emplace_back(a_, b_);
  } else {
    g_timing.pool.push_back(a_);
    g_timing.pool.push_back(b_);
  }
}

// ---------------------------------------------------------------------------
// counted device allocations
// ---------------------------------------------------------------------------

namespace {
struct DevMem {
  std::mutex mu;
  std::unordered_map<void *, size_t> sizes;
  uint64_t held = 0;
  uint64_t limit = 0;  // 0: none
};
DevMem g_mem;
}  // namespace

hipError_t dev_malloc_raw(void **p, size_t bytes) {
  *p = nullptr;
  std::lock_guard<std::mutex> g(g_mem.mu);
  if (g_mem.limit && g_mem.held + bytes > g_mem.limit) return hipErrorOutOfMemory;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    return e;
  }
  g_mem.sizes[*p] = bytes;
  g_mem.held += bytes;
  return hipSuccess;
}

void dev_free(void *p) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> g(g_mem.mu);
    auto it = g_mem.sizes.find(p);
    if (it != g_mem.sizes.end()) {
      g_mem.held -= it->second;
      g_mem.sizes.erase(it);
    }
  }
  (void)hipFree(p);
}

// ---------------------------------------------------------------------------
// scratch buffers
// ---------------------------------------------------------------------------

int scratch_get(ScratchMap &map, hipStream_t s, size_t bytes, void **out) {
  Scratch &sc = map[s];
  if (sc.bytes < bytes) {
    if (sc.p) {
      (void)hipStreamSynchronize(s);
      dev_free(sc.p);
      sc.p = nullptr;
      sc.bytes = 0;
    }
    hipError_t e = dev_malloc(&sc.p, bytes);
    if (e != hipSuccess) {
      sc.p = nullptr;
      return hip_fail(e, "device allocation (scratch)");
    }
    sc.bytes = bytes;
  }
  *out = sc.p;
  return TQ_OK;
}

void scratch_free_all(ScratchMap &map) {
  for (auto &kv : map)
    if (kv.second.p) dev_free(kv.second.p);
  map.clear();
}

// ---------------------------------------------------------------------------
// code validation (exactly x non-zeros, disjoint planes, zero padding)
// ---------------------------------------------------------------------------

int count_bad_codes(const uint32_t *codes, int64_t n, int d, int x, hipStream_t s, unsigned long long *bad) {
  unsigned long long *dcount = nullptr;
  hipError_t e = dev_malloc(&dcount, sizeof *dcount);
  if (e != hipSuccess) return hip_fail(e, "device allocation (counter)");
  unsigned long long h = 0;
  e = hipMemcpyAsync(dcount, &h, sizeof h, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = tqi::validate_launch(codes, n, d, x, dcount, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&h, dcount, sizeof h, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(dcount);
  if (e != hipSuccess) return hip_fail(e, "code validation");
  *bad = h;
  return TQ_OK;
}

}  // namespace tqr

using namespace tqr;

// ---------------------------------------------------------------------------
// public ABI
// ---------------------------------------------------------------------------

extern "C" {

const char *tq_status_str(int status) {
  switch (status) {
    case TQ_OK: return "TQ_OK";
    case TQ_ERR_INVALID: return "TQ_ERR_INVALID";
    case TQ_ERR_NOMEM: return "TQ_ERR_NOMEM";
    case TQ_ERR_DEVICE: return "TQ_ERR_DEVICE";
    case TQ_ERR_AGAIN: return "TQ_ERR_AGAIN";
    case TQ_ERR_NOTFOUND: return "TQ_ERR_NOTFOUND";
    case TQ_ERR_STATE: return "TQ_ERR_STATE";
    default: return "TQ_ERR_UNKNOWN";
  }
}

const char *tq_last_error(void) { return t_last_error.c_str(); }

int tq_version(void) { return 10000; }

int tq_code_words(int d) {
  if (d < 1 || d > TQ_MAX_D) return fail(TQ_ERR_INVALID, "d=%d outside [1, %d]", d, TQ_MAX_D);
  return (d + 31) / 32;
}

int tq_default_x(int d) {
  if (d < 1 || d > TQ_MAX_D) return fail(TQ_ERR_INVALID, "d=%d outside [1, %d]", d, TQ_MAX_D);
  return (2 * d + 1) / 3;  // ceil((2d - 1) / 3)
}

int tq_encode(const float *X, int64_t n, int d, int x, uint32_t *codes, void *stream) {
  clear_error();
  if (n < 0) return fail(TQ_ERR_INVALID, "n=%lld < 0", (long long)n);
  if (d < 1 || d > TQ_MAX_D) return fail(TQ_ERR_INVALID, "d=%d outside [1, %d]", d, TQ_MAX_D);
  if (x < 1 || x > d) return fail(TQ_ERR_INVALID, "x=%d outside [1, d=%d]", x, d);
  if (n == 0) return TQ_OK;
  if (!X || !codes) return fail(TQ_ERR_INVALID, "null X or codes");
  int dev;
  int rc = current_device(&dev);
  if (rc) return rc;
  DevCtx *ctx;
  if ((rc = device_ctx(dev, &ctx))) return rc;
  hipError_t e = tqi::encode_launch(X, n, d, x, codes, ctx->flags, ctx->num_cu, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "encode launch");
  return TQ_OK;
}

int tq_encode_b158(const float *X, int64_t n, int d, uint32_t *codes, void *stream) {
  clear_error();
  if (n < 0) return fail(TQ_ERR_INVALID, "n=%lld < 0", (long long)n);
  if (d < 1 || d > TQ_MAX_D) return fail(TQ_ERR_INVALID, "d=%d outside [1, %d]", d, TQ_MAX_D);
  if (n == 0) return TQ_OK;
  if (!X || !codes) return fail(TQ_ERR_INVALID, "null X or codes");
  int dev;
  int rc = current_device(&dev);
  if (rc) return rc;
  DevCtx *ctx;
  if ((rc = device_ctx(dev, &ctx))) return rc;
  hipError_t e = tqi::b158_launch(X, n, d, codes, ctx->flags, ctx->num_cu, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "b1.58 encode launch");
  return TQ_OK;
}

int tq_sync(void *stream) {
  clear_error();
  int dev;
  int rc = current_device(&dev);
  if (rc) return rc;
  DevCtx *ctx;
  if ((rc = device_ctx(dev, &ctx))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  int flag = 0;
  e = hipMemcpy(&flag, ctx->flags, sizeof flag, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "reading device flags");
  if (flag) {
    int zero = 0;
    e = hipMemcpy(ctx->flags, &zero, sizeof zero, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "clearing device flags");
    if (flag & 1) return fail(TQ_ERR_INVALID, "tq_encode saw a NaN or infinite input (row code set to zero)");
  }
  return TQ_OK;
}

int tq_db_create(const uint32_t *codes, int64_t n, int d, int x, void *stream, tq_db **out) {
  clear_error();
  if (!out) return fail(TQ_ERR_INVALID, "null out");
  *out = nullptr;
  if (!codes) return fail(TQ_ERR_INVALID, "null codes");
  if (n < 1 || n > INT32_MAX) return fail(TQ_ERR_INVALID, "n=%lld outside [1, 2^31)", (long long)n);
  if (d < 1 || d > TQ_MAX_D) return fail(TQ_ERR_INVALID, "d=%d outside [1, %d]", d, TQ_MAX_D);
  if (x < 0 || x > d) return fail(TQ_ERR_INVALID, "x=%d outside [0, d=%d]", x, d);
  int dev;
  int rc = current_device(&dev);
  if (rc) return rc;
  DevCtx *ctx;
  if ((rc = device_ctx(dev, &ctx))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);

  unsigned long long bad = 0;
  if ((rc = count_bad_codes(codes, n, d, x, s, &bad))) return rc;
  if (bad) return fail(TQ_ERR_INVALID, "%llu of %lld code rows are not {%d,%d} EVP vertices", bad, (long long)n, x, d);

  tq_db *db = new (std::nothrow) tq_db();
  if (!db) return fail(TQ_ERR_NOMEM, "host allocation");
  db->device = dev;
  db->num_cu = ctx->num_cu;
  const int W = (d + 31) / 32;
  const int nc = (W + 3) / 4;
  const int64_t ntiles = (n + tqi::kTileVecs - 1) / tqi::kTileVecs;
  db->bytes = static_cast<size_t>(ntiles) * 2 * nc * 64 * sizeof(uint4);
  uint4 *tiles = nullptr;
  hipError_t e = dev_malloc(&tiles, db->bytes);
  if (e != hipSuccess) {
    delete db;
    return hip_fail(e, "device allocation (database)");
  }
  e = tqi::repack_launch(codes, n, d, tiles, ntiles, nc, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    dev_free(tiles);
    delete db;
    return hip_fail(e, "database repack");
  }
  db->dev = tqi::DbDev{tiles, n, ntiles, d, x, W, nc};
  const int sc = tqi::sparse_chunks(d, x);
  if (sc > 0) {
    const size_t sbytes = static_cast<size_t>(ntiles) * sc * 64 * sizeof(uint4);
    uint4 *sp = nullptr;
    e = dev_malloc(&sp, sbytes);
    if (e == hipSuccess) {
      e = tqi::sparse_repack_launch(db->dev, sp, sc, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) dev_free(sp);
    }
    if (e != hipSuccess) {
      dev_free(tiles);
      delete db;
      return hip_fail(e, "index-list copy of the database");
    }
    db->dev.sparse = sp;
    db->dev.sc = sc;
    db->bytes += sbytes;
  }
  *out = db;
  return TQ_OK;
}

int tq_db_export(const tq_db *db, uint32_t *codes, void *stream) {
  clear_error();
  if (!db || !codes) return fail(TQ_ERR_INVALID, "null db or codes");
  DeviceGuard g(db->device);
  hipError_t e = tqi::export_launch(db->dev, codes, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "export launch");
  return TQ_OK;
}

int tq_db_info(const tq_db *db, int64_t *n, int *d, int *x, size_t *device_bytes) {
  clear_error();
  if (!db) return fail(TQ_ERR_INVALID, "null db");
  if (n) *n = db->dev.n;
  if (d) *d = db->dev.d;
  if (x) *x = db->dev.x;
  if (device_bytes) *device_bytes = db->bytes;
  return TQ_OK;
}

int tq_db_destroy(tq_db *db) {
  clear_error();
  if (!db) return TQ_OK;
  {
    DeviceGuard g(db->device);
    std::lock_guard<std::mutex> l(db->mu);
    scratch_free_all(db->scratch);
    batched_release(db);
    if (db->dev.tiles) dev_free(const_cast<uint4 *>(db->dev.tiles));
    if (db->dev.sparse) dev_free(const_cast<uint4 *>(db->dev.sparse));
  }
  delete db;
  return TQ_OK;
}

int tq_search_knn(const tq_db *cdb, const uint32_t *qcodes, int nq, int k, int32_t *ids, int32_t *scores,
                  const tq_search_opts *opts, void *stream) {
  clear_error();
  tq_db *db = const_cast<tq_db *>(cdb);
  if (!db) return fail(TQ_ERR_INVALID, "null db");
  if (!qcodes || !ids || !scores) return fail(TQ_ERR_INVALID, "null qcodes, ids or scores");
  if (nq < 1) return fail(TQ_ERR_INVALID, "nq=%d < 1", nq);
  if (k < 1 || k > TQ_MAX_K || k > db->dev.n)
    return fail(TQ_ERR_INVALID, "k=%d outside [1, min(n=%lld, %d)]", k, (long long)db->dev.n, TQ_MAX_K);
  const int path = opts ? opts->path : TQ_PATH_AUTO;
  if (path < TQ_PATH_AUTO || path > TQ_PATH_BATCHED) return fail(TQ_ERR_INVALID, "unknown path %d", path);
  if (opts && (opts->grid < 0 || opts->qtile < 0)) return fail(TQ_ERR_INVALID, "negative grid or qtile");
  const int engine = opts ? opts->engine : TQ_ENGINE_AUTO;
  if (engine < TQ_ENGINE_AUTO || engine > TQ_ENGINE_SPARSE) return fail(TQ_ERR_INVALID, "unknown engine %d", engine);
  const int metric = opts ? opts->metric : TQ_METRIC_DELTA;
  if (metric != TQ_METRIC_DELTA && metric != TQ_METRIC_L2) return fail(TQ_ERR_INVALID, "unknown metric %d", metric);
  if (metric == TQ_METRIC_L2 && (engine == TQ_ENGINE_MATRIX || engine == TQ_ENGINE_SPARSE))
    return fail(TQ_ERR_INVALID, "metric L2 runs on the bit planes: engine AUTO or POPCOUNT (engine %d given)", engine);
  if (engine == TQ_ENGINE_SPARSE) {
    if (path == TQ_PATH_BATCHED) return fail(TQ_ERR_INVALID, "the index-list engine serves the plain path only");
    if (!db->dev.sparse)
      return fail(TQ_ERR_INVALID, "no index-list copy: kept only for 8x <= d (x=%d, d=%d)", db->dev.x, db->dev.d);
  }
  DeviceGuard g(db->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc;
  if (opts && opts->check_queries) {
    unsigned long long bad = 0;
    if ((rc = count_bad_codes(qcodes, nq, db->dev.d, db->dev.x, s, &bad))) return rc;
    if (bad)
      return fail(TQ_ERR_INVALID, "%llu of %d query codes are not {%d,%d} EVP vertices", bad, nq, db->dev.x,
                  db->dev.d);
  }
  std::lock_guard<std::mutex> l(db->mu);
  const int use = engine == TQ_ENGINE_SPARSE ? TQ_PATH_PLAIN : choose_path(db, path, nq, k);
  if (use == TQ_PATH_BATCHED) return search_batched(db, qcodes, nq, k, ids, scores, opts, s);
  return search_plain(db, qcodes, nq, k, ids, scores, opts ? opts->grid : 0, engine, s, nullptr, metric);
}

int tq_search_masked(const tq_db *cdb, const float *Q, int nq, int k, int32_t *ids, float *scores,
                     const tq_search_opts *opts, void *stream) {
  clear_error();
  tq_db *db = const_cast<tq_db *>(cdb);
  if (!db) return fail(TQ_ERR_INVALID, "null db");
  if (!Q || !ids || !scores) return fail(TQ_ERR_INVALID, "null Q, ids or scores");
  if (nq < 1) return fail(TQ_ERR_INVALID, "nq=%d < 1", nq);
  if (k < 1 || k > TQ_MAX_K || k > db->dev.n)
    return fail(TQ_ERR_INVALID, "k=%d outside [1, min(n=%lld, %d)]", k, (long long)db->dev.n, TQ_MAX_K);
  DeviceGuard g(db->device);
  std::lock_guard<std::mutex> l(db->mu);
  return search_masked(db, Q, nq, k, ids, scores, opts ? opts->grid : 0, static_cast<hipStream_t>(stream));
}

int tq_rerank(const float *X, int64_t n, int d, const float *Q, int nq, const int32_t *cand, int ncand, int k,
              int32_t *ids, double *scores, void *stream) {
  clear_error();
  if (!X || !Q || !cand || !ids || !scores) return fail(TQ_ERR_INVALID, "null pointer argument");
  if (n < 1) return fail(TQ_ERR_INVALID, "n=%lld < 1", (long long)n);
  if (d < 1 || d > TQ_MAX_D) return fail(TQ_ERR_INVALID, "d=%d outside [1, %d]", d, TQ_MAX_D);
  if (nq < 0) return fail(TQ_ERR_INVALID, "nq=%d < 0", nq);
  if (ncand < 1 || ncand > TQ_MAX_RERANK)
    return fail(TQ_ERR_INVALID, "ncand=%d outside [1, %d]", ncand, TQ_MAX_RERANK);
  if (k < 1 || k > ncand) return fail(TQ_ERR_INVALID, "k=%d outside [1, ncand=%d]", k, ncand);
  static_assert(TQ_MAX_RERANK == tqi::kMaxRerank, "candidate limit");
  if (nq == 0) return TQ_OK;
  hipError_t e = tqi::rerank_launch(X, n, d, Q, nq, cand, ncand, k, ids, scores, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "rerank launch");
  return TQ_OK;
}

int tq_delta_dump(const tq_db *db, const uint32_t *qcodes, int nq, int32_t *delta, void *stream) {
  clear_error();
  if (!db || !qcodes || !delta) return fail(TQ_ERR_INVALID, "null db, qcodes or delta");
  if (nq < 1 || nq > 65535) return fail(TQ_ERR_INVALID, "nq=%d outside [1, 65535]", nq);
  DeviceGuard g(db->device);
  hipError_t e = tqi::delta_dump_launch(db->dev, qcodes, nq, delta, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "delta dump launch");
  return TQ_OK;
}

int tq_autotune(const tq_db *cdb, int nq_max, const int *ks, int nks, void *stream) {
  clear_error();
  tq_db *db = const_cast<tq_db *>(cdb);
  if (!db) return fail(TQ_ERR_INVALID, "null db");
  if (nq_max < 1) return fail(TQ_ERR_INVALID, "nq_max=%d < 1", nq_max);
  if (!ks || nks < 1) return fail(TQ_ERR_INVALID, "no k values");
  DeviceGuard g(db->device);
  std::lock_guard<std::mutex> l(db->mu);
  return autotune(db, nq_max, ks, nks, static_cast<hipStream_t>(stream), log_level() >= 2);
}

int tq_set_device_limit(uint64_t bytes) {
  clear_error();
  std::lock_guard<std::mutex> g(g_mem.mu);
  g_mem.limit = bytes;
  return TQ_OK;
}

int tq_device_bytes(uint64_t *held) {
  clear_error();
  if (!held) return fail(TQ_ERR_INVALID, "null held");
  std::lock_guard<std::mutex> g(g_mem.mu);
  *held = g_mem.held;
  return TQ_OK;
}

int tq_timing_enable(int enable) {
  clear_error();
  g_timing_on.store(enable ? 1 : 0);
  return TQ_OK;
}

int tq_timing_read(int which, double *total_ms, int64_t *launches, int reset) {
  clear_error();
  if (which < 0 || which >= kTimeFamilies) return fail(TQ_ERR_INVALID, "timing family %d", which);
  std::lock_guard<std::mutex> g(g_timing.mu);
  for (auto &pr : g_timing.pending[which]) {
    float ms = 0.f;
    if (hipEventSynchronize(pr.second) == hipSuccess && hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
      g_timing.total_ms[which] += ms;
      g_timing.launches[which] += 1;
    }
    g_timing.pool.push_back(pr.first);
    g_timing.pool.push_back(pr.second);
  }
  g_timing.pending[which].clear();
  if (total_ms) *total_ms = g_timing.total_ms[which];
  if (launches) *launches = g_timing.launches[which];
  if (reset) {
    g_timing.total_ms[which] = 0;
    g_timing.launches[which] = 0;
  }
  return TQ_OK;
}

}  // extern "C"
