// noalloc.hip -- tq_search_knn_noalloc: the plain search path (one full
// database pass per query, then the per-query merge) with its scratch in a
// fixed device array of this file instead of memory allocated on demand.
//
// The scratch holds, per merge round, every workgroup's sorted list of k keys
// for each query of the round, the merge's intermediate keys and, where the
// plain path takes a sample pass first, the sample's result rows.  Rounds are
// sized to fit the array, so any nq fits; one query's need (grid x k keys plus
// its share of the rest) must fit, else the call fails before any launch.
//
// The array lives as long as the process, one copy per GPU the library runs
// on.  Its device address is looked up once per device, with that device
// current; host code passes that address, never the array's name (which in
// host code is only a stand-in for the symbol).  Nothing here needs the array
// to start at zero: every word a call reads was written earlier in that call.
#include <mutex>

#include "tq_runtime.h"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint64_t scratch[kScratchBytes / sizeof(uint64_t)];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (the device is current).
int scratch_address(int dev, void **out) {
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return tqr::hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return TQ_OK;
}

}  // namespace

extern "C" int tq_search_knn_noalloc(const tq_db *cdb, const uint32_t *qcodes, int nq, int k, int32_t *ids,
                                     int32_t *scores, const tq_search_opts *opts, void *stream) {
  using namespace tqr;
  clear_error();
  tq_db *db = const_cast<tq_db *>(cdb);
  if (!db) return fail(TQ_ERR_INVALID, "null db");
  if (!qcodes || !ids || !scores) return fail(TQ_ERR_INVALID, "null qcodes, ids or scores");
  if (nq < 1) return fail(TQ_ERR_INVALID, "nq=%d < 1", nq);
  if (k < 1 || k > TQ_MAX_K || k > db->dev.n)
    return fail(TQ_ERR_INVALID, "k=%d outside [1, min(n=%lld, %d)]", k, (long long)db->dev.n, TQ_MAX_K);
  const int path = opts ? opts->path : TQ_PATH_AUTO;
  if (path != TQ_PATH_AUTO && path != TQ_PATH_PLAIN)
    return fail(TQ_ERR_INVALID, "path %d: only the plain path runs without allocating", path);
  if (opts && opts->check_queries)
    return fail(TQ_ERR_INVALID, "check_queries allocates a counter; not available without allocation");
  if (opts && opts->grid < 0) return fail(TQ_ERR_INVALID, "negative grid");
  const int engine = opts ? opts->engine : TQ_ENGINE_AUTO;
  if (engine != TQ_ENGINE_AUTO && engine != TQ_ENGINE_POPCOUNT && engine != TQ_ENGINE_SPARSE)
    return fail(TQ_ERR_INVALID, "engine %d: the plain path takes AUTO, POPCOUNT or SPARSE", engine);
  const int metric = opts ? opts->metric : TQ_METRIC_DELTA;
  if (metric != TQ_METRIC_DELTA && metric != TQ_METRIC_L2) return fail(TQ_ERR_INVALID, "unknown metric %d", metric);
  if (engine == TQ_ENGINE_SPARSE && !db->dev.sparse)
    return fail(TQ_ERR_INVALID, "no index-list copy: kept only for 8x <= d (x=%d, d=%d)", db->dev.x, db->dev.d);
  if (db->device < 0 || db->device >= kMaxDevices) return fail(TQ_ERR_DEVICE, "device index %d", db->device);
  DeviceGuard g(db->device);
  ScratchSpan span;
  span.bytes = kScratchBytes;
  int rc = scratch_address(db->device, &span.p);
  if (rc) return rc;
  // Serialises the host-side enqueue of such calls; calls whose GPU work
  // overlaps (other streams of the same device) still share the one array.
  std::lock_guard<std::mutex> l(g_mu);
  return search_plain(db, qcodes, nq, k, ids, scores, opts ? opts->grid : 0, engine,
                      static_cast<hipStream_t>(stream), &span, metric);
}
