// batched.cpp -- host runtime of the batched search path: per-bucket device
// resources and hipGraphs, the shape autotuner and its cache, and the choice
// between the plain and the batched path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "tq_batched.h"
#include "tq_runtime.h"

namespace tqr {

namespace {

constexpr int kMaxBucket = 1024;

int bucket_of(int nq) {
  int b = 1;
  while (b < nq) b <<= 1;
  return b;
}

struct Shape {
  int qtile = 0;
  int grid = 0;
  bool plain = false;  // the plain path was faster for this bucket
  int engine = TQ_ENGINE_POPCOUNT;
  float ms = 0.f;      // tuned time of a full bucket (0: not timed)
};

// ---------------------------------------------------------------------------
// tuning cache: key "nc<nc>/kc<k class>/b<bucket>/t<log2 tiles>" -> Shape
// (the database's size class is part of the key: the best grid and the
// plain / batched split depend on it), and the same key + "/q<qtile>" -> the
// best matrix-engine shape with that query tile and its time; optional JSON
// file.  The k class
// separates every set of k that has its own kernels and valid query tiles:
// k <= kGroupMaxK (the matrix engine's grouped lists, 256-query tiles), then
// one class per list depth R = rows_for_k(k) above that.
// ---------------------------------------------------------------------------
struct TuneCache {
  std::mutex mu;
  bool loaded = false;
  std::map<std::string, Shape> map;
};
TuneCache g_tune;

int size_class(int64_t ntiles) {
  int c = 0;
  while ((int64_t(1) << c) < ntiles) ++c;
  return c;
}

int k_class(int k) { return k <= tqi::kGroupMaxK ? 0 : tqi::rows_for_k(k); }

std::string tune_key(const tqi::DbDev &db, int k, int bucket, int qtile = 0) {
  char b[80];
  if (qtile)
    std::snprintf(b, sizeof b, "nc%d/kc%d/b%d/t%d/q%d", db.nc, k_class(k), bucket, size_class(db.ntiles), qtile);
  else
    std::snprintf(b, sizeof b, "nc%d/kc%d/b%d/t%d", db.nc, k_class(k), bucket, size_class(db.ntiles));
  return b;
}

const char *tune_file() { return std::getenv("TQ_TUNE_CACHE"); }

void tune_load_locked() {
  if (g_tune.loaded) return;
  g_tune.loaded = true;
  const char *f = tune_file();
  if (!f) return;
  FILE *fp = std::fopen(f, "r");
  if (!fp) return;
  char line[256];
  while (std::fgets(line, sizeof line, fp)) {
    char key[64];
    Shape s;
    int plain = 0;
    const int got = std::sscanf(line,
                                " \"%63[^\"]\": {\"qtile\": %d, \"grid\": %d, \"plain\": %d, \"engine\": %d, "
                                "\"ms\": %f}",
                                key, &s.qtile, &s.grid, &plain, &s.engine, &s.ms);
    if (got >= 5) {  // files written before the time was stored have none
      if (got == 5) s.ms = 0.f;
      s.plain = plain != 0;
      g_tune.map[key] = s;
    }
  }
  std::fclose(fp);
}

void tune_save_locked() {
  const char *f = tune_file();
  if (!f) return;
  std::string tmp = std::string(f) + ".tmp";
  FILE *fp = std::fopen(tmp.c_str(), "w");
  if (!fp) return;
  std::fprintf(fp, "{\n");
  size_t i = 0;
  for (auto &kv : g_tune.map) {
    std::fprintf(fp, " \"%s\": {\"qtile\": %d, \"grid\": %d, \"plain\": %d, \"engine\": %d, \"ms\": %.4f}%s\n",
                 kv.first.c_str(), kv.second.qtile, kv.second.grid, kv.second.plain ? 1 : 0, kv.second.engine,
                 kv.second.ms, ++i < g_tune.map.size() ? "," : "");
  }
  std::fprintf(fp, "}\n");
  std::fclose(fp);
  std::rename(tmp.c_str(), f);
}

bool tune_lookup(const tqi::DbDev &db, int k, int bucket, Shape *out, int qtile = 0) {
  std::lock_guard<std::mutex> g(g_tune.mu);
  tune_load_locked();
  auto it = g_tune.map.find(tune_key(db, k, bucket, qtile));
  if (it == g_tune.map.end()) return false;
  *out = it->second;
  return true;
}

void tune_store(const tqi::DbDev &db, int k, int bucket, const Shape &s, int qtile = 0) {
  std::lock_guard<std::mutex> g(g_tune.mu);
  tune_load_locked();
  g_tune.map[tune_key(db, k, bucket, qtile)] = s;
  tune_save_locked();
}

}  // namespace

// Untuned choice, from measurements on MI355X: the matrix engine wins from
// about 10 queries for k <= 128 (N = 1e7, d = 1024, k = 10: 0.58 against
// 0.71 ms at 10 queries, 0.56 against 0.57 at 8; N = 5e6, d = 768: 0.36
// against 0.42 ms at 12, 0.33 against 0.30 at 8); the popcount engine below
// that and for larger k.  (The batched path passes its power-of-two bucket,
// serving ticks their query count.)
int default_engine(int k, int nq) {
  if (tqi::rows_for_k(k) <= 2 && nq >= 10) return TQ_ENGINE_MATRIX;
  return TQ_ENGINE_POPCOUNT;
}

namespace {

// Workgroups per CU of the matrix engine's default grid: two for 64-query
// tiles (four waves) and for the eight-wave 128-query tiles of k <= 16 (124
// VGPRs; measured best at two per CU), one for the eight-wave 128-query tiles
// of k > 16 and for 256-query tiles.
int mfma_resident_per_cu(int k, int qtile) {
  return (qtile == 256 || (qtile == 128 && k > tqi::kGroupMaxK)) ? 1 : 2;
}

int default_matrix_qtile(int k, int bucket) {
  if (k <= tqi::kGroupMaxK) return bucket >= 512 ? 256 : bucket >= 128 ? 128 : 64;
  return bucket >= 256 ? 256 : bucket >= 128 ? 128 : 64;
}

Shape default_shape(const tq_db *db, int k, int bucket) {
  Shape s;
  const int cu = db->num_cu > 0 ? db->num_cu : 256;
  s.grid = cu * 2;
  s.plain = bucket == 1;
  s.engine = default_engine(k, bucket);
  if (s.engine == TQ_ENGINE_MATRIX) {
    // (N = 1e7, d = 1024, k = 10: 1 024 queries 5.2 / 5.3 / 7.4 ms on 256 /
    // 128 / 64-query tiles, 256 queries 1.8 / 1.6 / 2.2 ms; k = 100, 1 024
    // queries: 6.6 / 8.8 ms on 256 / 128, 512 queries 3.5 / 4.8 ms, 160
    // queries 1.7 / 2.4 / 2.2 ms on 256 / 128 / 64, 100 queries 1.5 / 1.2 /
    // 1.4 ms, 64 queries 1.4 / 1.1 / 0.8 ms)
    s.qtile = default_matrix_qtile(k, bucket);
    s.grid = cu * mfma_resident_per_cu(k, s.qtile);
  } else {
    const int qmax = tqi::batched_max_qtile(k);
    s.qtile = std::min(qmax, bucket <= 2 ? 2 : bucket <= 4 ? 4 : bucket <= 8 ? 8 : 16);
  }
  return s;
}

}  // namespace

// ---------------------------------------------------------------------------
// per-database state: buffers and graphs per (stream, bucket, k, shape)
// ---------------------------------------------------------------------------

struct BatchEntry {
  uint32_t *qprep = nullptr;
  tqi::BatchParams *prm = nullptr;
  uint64_t *partial = nullptr;
  uint64_t *mid = nullptr;  // first-stage merge results
  uint64_t *bound = nullptr;  // per (query, part) published keys (BatchParams::bound)
  uint64_t *floor = nullptr;  // per query: the matrix scan's sample floor (k > 16)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;  // recorded after the entry's latest use
  uint64_t last_use = 0;
};

// Entries kept per database; beyond this the least recently used one is freed
// (after its latest use has finished), so that many distinct k, buckets or
// streams do not hold device memory without bound.
constexpr size_t kMaxEntries = 96;

struct BatchedState {
  hipStream_t capture = nullptr;
  uint64_t clock = 0;
  std::map<std::tuple<hipStream_t, int, int, int, int, int>, BatchEntry> entries;
};

namespace {

void free_entry(BatchEntry &e) {
  if (e.done) {
    (void)hipEventSynchronize(e.done);
    (void)hipEventDestroy(e.done);
  }
  if (e.exec) (void)hipGraphExecDestroy(e.exec);
  if (e.graph) (void)hipGraphDestroy(e.graph);
  if (e.qprep) dev_free(e.qprep);
  if (e.prm) dev_free(e.prm);
  if (e.partial) dev_free(e.partial);
  if (e.mid) dev_free(e.mid);
  if (e.bound) dev_free(e.bound);
  if (e.floor) dev_free(e.floor);
  e = BatchEntry{};
}

int get_entry(tq_db *db, hipStream_t s, int bucket, int k, const Shape &sh, BatchEntry **out) {
  if (!db->batched) db->batched = new BatchedState();
  BatchedState &st = *db->batched;
  auto key = std::make_tuple(s, bucket, k, sh.qtile, sh.grid, sh.engine);
  auto it = st.entries.find(key);
  if (it != st.entries.end()) {
    *out = &it->second;
    return TQ_OK;
  }
  if (st.entries.size() >= kMaxEntries) {
    auto victim = st.entries.begin();
    for (auto v = st.entries.begin(); v != st.entries.end(); ++v)
      if (v->second.last_use < victim->second.last_use) victim = v;
    free_entry(victim->second);  // waits for its latest use
    st.entries.erase(victim);
  }
  BatchEntry e;
  const size_t qbytes = static_cast<size_t>(bucket) * 8 * db->dev.nc * sizeof(uint32_t);
  // (query, part) lists of any split of up to `bucket` queries
  const size_t lists = tqi::batch_max_lists(sh.qtile, sh.grid, bucket);
  hipError_t err = dev_malloc(&e.qprep, qbytes);
  if (err == hipSuccess) err = dev_malloc(&e.prm, sizeof(tqi::BatchParams));
  if (err == hipSuccess) err = dev_malloc(&e.partial, lists * k * sizeof(uint64_t));
  if (err == hipSuccess) err = dev_malloc(&e.bound, lists * tqi::kBoundSlotsPerPart * sizeof(uint64_t));
  if (err == hipSuccess) err = dev_malloc(&e.floor, static_cast<size_t>(bucket) * sizeof(uint64_t));
  if (err == hipSuccess) err = hipEventCreateWithFlags(&e.done, hipEventDisableTiming);
  if (err == hipSuccess)
    err = dev_malloc(&e.mid, static_cast<size_t>(tqi::merge_batched_mid_keys(bucket, tqi::batch_max_parts(sh.grid),
                                                                              k)) * sizeof(uint64_t));
  if (err != hipSuccess) {
    free_entry(e);
    return hip_fail(err, "device allocation (batched buffers)");
  }
  *out = &(st.entries[key] = e);
  return TQ_OK;
}

// The matrix engine's k > 16 scan starts from a sample floor (every 16th
// tile scored first, scan_mfma_launch) on databases of at least 2 048 tiles,
// where the sample holds >= 128 tiles: each (query, part) list then takes
// only the keys above the floor instead of k keys at its start and the keys
// that outrank them later.  (N = 1e7, d = 1024, 1 024 queries at k = 100 on
// 256-query tiles: 7.5 / 6.8 / 6.6 ms with every 32nd / 16th / 8th tile; 128-
// query tiles, which also exchange bounds between parts: 8.7 / 8.8 / 9.1 ms.)
constexpr int kMfmaSampleStride = 16;
constexpr int64_t kMfmaSampleMinTiles = 2048;

hipError_t launch_scan(tq_db *db, BatchEntry &e, int bucket, int k, const Shape &sh, hipStream_t s) {
  if (sh.engine == TQ_ENGINE_MATRIX) {
    // the longest part of any split the entry's graph may replay (up to
    // `bucket` queries): one split per query-tile count
    int64_t widest = 0;
    for (int nqt = 1; (nqt - 1) * sh.qtile < bucket; ++nqt) {
      tqi::BatchParams b;
      tqi::batch_split(b, std::min(nqt * sh.qtile, bucket), sh.qtile, sh.grid, 0, db->dev.ntiles);
      widest = std::max(widest, b.tiles_per_part);
    }
    tqi::MfmaSample smp;
    if (k > tqi::kGroupMaxK && db->dev.ntiles >= kMfmaSampleMinTiles) {
      smp.stride = kMfmaSampleStride;
      smp.bucket = bucket;
      smp.floor = e.floor;
    }
    return tqi::scan_mfma_launch(db->dev, e.qprep, e.prm, k, sh.qtile, sh.grid, widest, e.partial, s, smp);
  }
  return tqi::scan_batched_launch(db->dev, e.qprep, e.prm, k, sh.qtile, sh.grid, e.partial, s);
}

int enqueue_scan_merge(tq_db *db, BatchEntry &e, int bucket, int k, const Shape &sh, hipStream_t s) {
  hipError_t err = launch_scan(db, e, bucket, k, sh, s);
  if (err != hipSuccess) return hip_fail(err, "batched scan launch");
  err = tqi::merge_batched_launch(e.partial, e.prm, bucket, k, tqi::batch_max_parts(sh.grid), e.mid, s);
  if (err != hipSuccess) return hip_fail(err, "batched merge launch");
  return TQ_OK;
}

int ensure_graph(tq_db *db, BatchEntry &e, int bucket, int k, const Shape &sh) {
  if (e.exec) return TQ_OK;
  BatchedState &st = *db->batched;
  hipError_t err = hipSuccess;
  if (!st.capture) {
    err = hipStreamCreateWithFlags(&st.capture, hipStreamNonBlocking);
    if (err != hipSuccess) return hip_fail(err, "hipStreamCreate(capture)");
  }
  err = hipStreamBeginCapture(st.capture, hipStreamCaptureModeThreadLocal);
  if (err != hipSuccess) return hip_fail(err, "hipStreamBeginCapture");
  int rc = enqueue_scan_merge(db, e, bucket, k, sh, st.capture);
  hipGraph_t g = nullptr;
  err = hipStreamEndCapture(st.capture, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (err != hipSuccess) return hip_fail(err, "hipStreamEndCapture");
  hipGraphExec_t x = nullptr;
  err = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (err != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(err, "hipGraphInstantiate");
  }
  e.graph = g;
  e.exec = x;
  return TQ_OK;
}

// One chunk of <= kMaxBucket queries; l2 != 0 scores 2 Delta - nnz(v).
int run_chunk_on(tq_db *db, BatchEntry *e, const uint32_t *qcodes, int nq, int k, int32_t *ids, int32_t *scores,
                 const Shape &sh, bool use_graph, hipStream_t s, int l2);

int run_chunk(tq_db *db, const uint32_t *qcodes, int nq, int k, int32_t *ids, int32_t *scores, const Shape &sh,
              bool use_graph, hipStream_t s, int l2 = 0) {
  BatchEntry *e = nullptr;
  int rc = get_entry(db, s, bucket_of(nq), k, sh, &e);
  if (rc) return rc;
  rc = run_chunk_on(db, e, qcodes, nq, k, ids, scores, sh, use_graph, s, l2);
  // the entry's latest use, for a later eviction
  e->last_use = ++db->batched->clock;
  if (hipEventRecord(e->done, s) != hipSuccess && rc == TQ_OK) rc = fail(TQ_ERR_DEVICE, "hipEventRecord");
  return rc;
}

int run_chunk_on(tq_db *db, BatchEntry *e, const uint32_t *qcodes, int nq, int k, int32_t *ids, int32_t *scores,
                 const Shape &sh, bool use_graph, hipStream_t s, int l2) {
  const int bucket = bucket_of(nq);
  int rc = TQ_OK;
  hipError_t err = tqi::batch_prep_launch(qcodes, nq, bucket, db->dev, sh.qtile, sh.grid, ids, scores, e->qprep,
                                          e->prm, e->bound, l2, s);
  if (err != hipSuccess) return hip_fail(err, "batch prep launch");
  if (timing_enabled()) {
    // timed runs launch directly so the events bracket the scan kernel alone
    {
      TimedLaunch t(kTimeBatched, s);
      err = launch_scan(db, *e, bucket, k, sh, s);
    }
    if (err != hipSuccess) return hip_fail(err, "batched scan launch");
    err = tqi::merge_batched_launch(e->partial, e->prm, bucket, k, tqi::batch_max_parts(sh.grid), e->mid, s);
    if (err != hipSuccess) return hip_fail(err, "batched merge launch");
    return TQ_OK;
  }
  if (use_graph) {
    if ((rc = ensure_graph(db, *e, bucket, k, sh))) return rc;
    err = hipGraphLaunch(e->exec, s);
    if (err != hipSuccess) return hip_fail(err, "hipGraphLaunch");
    return TQ_OK;
  }
  return enqueue_scan_merge(db, *e, bucket, k, sh, s);
}

// Engine and query tile of a call: explicit options first, then the tuning
// cache, then the default.  An explicit query tile implies its engine (2..16:
// popcount, 64 / 128: matrix).
// A shape the kernels accept for this k (a cache file written by another
// build, or edited by hand, may hold one they do not).
bool shape_valid(const Shape &sh, int k) {
  if (sh.grid < 1) return false;
  if (sh.engine == TQ_ENGINE_MATRIX) return tqi::rows_for_k(k) <= 2 && tqi::mfma_supported(k, sh.qtile);
  if (sh.engine != TQ_ENGINE_POPCOUNT) return false;
  return (sh.qtile == 2 || sh.qtile == 4 || sh.qtile == 8 || sh.qtile == 16) && sh.qtile <= tqi::batched_max_qtile(k);
}

// The tuned matrix shape whose time at a full bucket, scaled by the query
// tiles `nq` queries fill against the tiles of the full bucket, is least:
// a bucket's queries fill its tiles, a smaller batch may fill fewer of a
// smaller tile (600 queries: three 256-query tiles out of four, or five
// 128-query tiles out of eight).  `sh` when no alternative was timed.
Shape tile_for(const tq_db *db, int k, int bucket, int nq, const Shape &sh) {
  Shape best = sh;
  double best_est = 1e300;
  for (int qt : {64, 128, 256}) {
    Shape c;
    if (!tqi::mfma_supported(k, qt) || !tune_lookup(db->dev, k, bucket, &c, qt) || c.ms <= 0.f) continue;
    const double est = static_cast<double>(c.ms) * ((nq + qt - 1) / qt) / ((bucket + qt - 1) / qt);
    if (est < best_est) {
      best_est = est;
      best = c;
    }
  }
  return best;
}

Shape shape_for(tq_db *db, int k, int bucket, int nq, const tq_search_opts *opts) {
  Shape sh;
  if (!tune_lookup(db->dev, k, bucket, &sh) || !shape_valid(sh, k)) sh = default_shape(db, k, bucket);
  int engine = opts ? opts->engine : TQ_ENGINE_AUTO;
  const int qtile = opts ? opts->qtile : 0;
  const bool any_matrix = engine == TQ_ENGINE_AUTO || engine == TQ_ENGINE_MATRIX;
  if (sh.engine == TQ_ENGINE_MATRIX && !sh.plain && qtile == 0 && any_matrix) sh = tile_for(db, k, bucket, nq, sh);
  if (engine == TQ_ENGINE_AUTO && qtile > 0) engine = qtile >= 64 ? TQ_ENGINE_MATRIX : TQ_ENGINE_POPCOUNT;
  // the l2 order (2 Delta - nnz(v)) is scored by the popcount engine only
  if (engine == TQ_ENGINE_AUTO && opts && opts->metric == TQ_METRIC_L2) engine = TQ_ENGINE_POPCOUNT;
  bool changed = false;
  if (engine != TQ_ENGINE_AUTO && engine != sh.engine) {
    sh.engine = engine;
    changed = true;
    if (engine == TQ_ENGINE_MATRIX) {
      sh.qtile = default_matrix_qtile(k, bucket);
    } else {
      const int qmax = tqi::batched_max_qtile(k);
      sh.qtile = std::min(qmax, bucket <= 2 ? 2 : bucket <= 4 ? 4 : bucket <= 8 ? 8 : 16);
    }
  }
  if (qtile > 0 && qtile != sh.qtile) {
    sh.qtile = qtile;
    changed = true;
  }
  if (changed) {
    const int cu = db->num_cu > 0 ? db->num_cu : 256;
    sh.grid = sh.engine == TQ_ENGINE_MATRIX ? cu * mfma_resident_per_cu(k, sh.qtile) : cu * 2;
  }
  if (opts && opts->grid > 0) sh.grid = opts->grid;
  return sh;
}

}  // namespace

int choose_path(tq_db *db, int requested, int nq, int k) {
  if (requested != TQ_PATH_AUTO) return requested;
  const int bucket = bucket_of(std::min(nq, kMaxBucket));
  Shape sh;
  if (!tune_lookup(db->dev, k, bucket, &sh) || !shape_valid(sh, k)) sh = default_shape(db, k, bucket);
  return sh.plain ? TQ_PATH_PLAIN : TQ_PATH_BATCHED;
}

int search_batched(tq_db *db, const uint32_t *qcodes, int nq, int k, int32_t *ids, int32_t *scores,
                   const tq_search_opts *opts, hipStream_t s) {
  const bool use_graph = opts ? opts->use_graph != 0 : true;
  const int engine = opts ? opts->engine : TQ_ENGINE_AUTO;
  const int q = opts ? opts->qtile : 0;
  if (engine < TQ_ENGINE_AUTO || engine > TQ_ENGINE_MATRIX)
    return fail(TQ_ERR_INVALID, "engine %d does not serve the batched path", engine);
  const bool matrix = engine == TQ_ENGINE_MATRIX || (engine == TQ_ENGINE_AUTO && q >= 64);
  const int l2 = opts && opts->metric == TQ_METRIC_L2 ? 1 : 0;
  if (matrix && l2) return fail(TQ_ERR_INVALID, "the matrix engine scores Delta only (metric L2 given)");
  if (matrix && tqi::rows_for_k(k) > 2) return fail(TQ_ERR_INVALID, "the matrix engine supports k <= 128 (k=%d)", k);
  if (q > 0) {
    if (matrix) {
      if (!tqi::mfma_supported(k, q))
        return fail(TQ_ERR_INVALID, "matrix engine: qtile=%d is not 64, 128 or 256", q);
    } else {
      if (q != 2 && q != 4 && q != 8 && q != 16)
        return fail(TQ_ERR_INVALID, "qtile=%d is not 2, 4, 8, 16, 64 or 128", q);
      if (q > tqi::batched_max_qtile(k))
        return fail(TQ_ERR_INVALID, "qtile=%d exceeds %d for k=%d", q, tqi::batched_max_qtile(k), k);
    }
  }
  const int row_words = 2 * db->dev.W;
  for (int q0 = 0; q0 < nq; q0 += kMaxBucket) {
    const int m = std::min(kMaxBucket, nq - q0);
    const Shape sh = shape_for(db, k, bucket_of(m), m, opts);
    int rc = run_chunk(db, qcodes + static_cast<int64_t>(q0) * row_words, m, k, ids + static_cast<int64_t>(q0) * k,
                       scores + static_cast<int64_t>(q0) * k, sh, use_graph, s, l2);
    if (rc) return rc;
  }
  return TQ_OK;
}

void batched_release(tq_db *db) {
  if (!db->batched) return;
  for (auto &kv : db->batched->entries) free_entry(kv.second);
  if (db->batched->capture) (void)hipStreamDestroy(db->batched->capture);
  delete db->batched;
  db->batched = nullptr;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------

// Times one configuration (plain path when sh.plain) on `s`: a first run
// that builds graphs and buffers, then kTuneReps timed runs; the median.
constexpr int kTuneReps = 3;

static int time_config(tq_db *db, const uint32_t *q, int nq, int k, int32_t *ids, int32_t *scores, const Shape &sh,
                       hipStream_t s, float *ms_out) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return fail(TQ_ERR_DEVICE, "hipEventCreate");
  }
  int rc = TQ_OK;
  float times[kTuneReps];
  for (int rep = 0; rep <= kTuneReps && rc == TQ_OK; ++rep) {
    (void)hipEventRecord(a, s);
    if (sh.plain)
      rc = search_plain(db, q, nq, k, ids, scores, 0, TQ_ENGINE_AUTO, s);
    else
      rc = run_chunk(db, q, nq, k, ids, scores, sh, true, s);
    (void)hipEventRecord(b, s);
    if (hipEventSynchronize(b) != hipSuccess) rc = fail(TQ_ERR_DEVICE, "hipEventSynchronize");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    if (rep > 0) times[rep - 1] = ms;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  std::sort(times, times + kTuneReps);
  *ms_out = rc == TQ_OK ? times[kTuneReps / 2] : 1e30f;
  return rc;
}

// splitmix64 (Steele, Lea, Flood 2014): the seeded generator of the tuning
// queries.
static uint64_t splitmix64(uint64_t &state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Tuning queries: distinct codes near the data but not in it.  Each starts
// as a database row (canonical layout, host memory) and a quarter of its
// non-zeros move to random zero coordinates with random signs, so the number
// of non-zeros (the database's x) is kept; where a row has no zero
// coordinate (x = d) those non-zeros flip sign instead.
static void perturb_rows(uint32_t *rows, int count, int d, int W, uint64_t seed) {
  std::vector<int> nz, zero;
  for (int r = 0; r < count; ++r) {
    uint64_t st = seed ^ (0xD1B54A32D192ED03ull * static_cast<uint64_t>(r + 1));
    uint32_t *plus = rows + static_cast<size_t>(r) * 2 * W, *minus = plus + W;
    nz.clear();
    zero.clear();
    for (int i = 0; i < d; ++i) {
      const uint32_t bit = 1u << (i % 32);
      ((plus[i / 32] | minus[i / 32]) & bit ? nz : zero).push_back(i);
    }
    const int moves = std::max<int>(nz.empty() ? 0 : 1, static_cast<int>(nz.size()) / 4);
    for (int m = 0; m < moves; ++m) {
      const size_t a = splitmix64(st) % nz.size();
      const int i = nz[a];
      const uint32_t bi = 1u << (i % 32);
      const bool neg = (splitmix64(st) & 1) != 0;
      if (zero.empty()) {  // x = d: flip the sign
        plus[i / 32] ^= bi;
        minus[i / 32] ^= bi;
        continue;
      }
      const size_t b = splitmix64(st) % zero.size();
      const int j = zero[b];
      const uint32_t bj = 1u << (j % 32);
      plus[i / 32] &= ~bi;
      minus[i / 32] &= ~bi;
      (neg ? minus : plus)[j / 32] |= bj;
      nz[a] = j;  // j is now a non-zero, i a zero
      zero[b] = i;
    }
  }
}

int autotune(tq_db *db, int nq_max, const int *ks, int nks, hipStream_t s, int verbose) {
  const int maxb = bucket_of(std::min(std::max(nq_max, 1), kMaxBucket));
  // queries: the first database rows (valid codes of the right (d, x)),
  // repeated up to the largest bucket, each perturbed in its own way
  const int nqq = std::min<int64_t>(maxb, db->dev.n);
  uint32_t *q = nullptr;
  int32_t *ids = nullptr, *scores = nullptr;
  const int W = db->dev.W;
  const size_t row_bytes = static_cast<size_t>(2 * W) * sizeof(uint32_t);
  hipError_t err = dev_malloc(&q, static_cast<size_t>(maxb) * row_bytes);
  int kmax = 1;
  for (int i = 0; i < nks; ++i) kmax = std::max(kmax, ks[i]);
  if (err == hipSuccess) err = dev_malloc(&ids, static_cast<size_t>(maxb) * kmax * sizeof(int32_t));
  if (err == hipSuccess) err = dev_malloc(&scores, static_cast<size_t>(maxb) * kmax * sizeof(int32_t));
  tqi::DbDev head = db->dev;
  head.n = nqq;
  head.ntiles = (nqq + 63) / 64;
  std::vector<uint32_t> host(static_cast<size_t>(maxb) * 2 * W);
  if (err == hipSuccess) err = tqi::export_launch(head, q, s);
  if (err == hipSuccess) err = hipMemcpyAsync(host.data(), q, nqq * row_bytes, hipMemcpyDeviceToHost, s);
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  if (err == hipSuccess) {
    for (int r = nqq; r < maxb; r += nqq)
      std::memcpy(host.data() + static_cast<size_t>(r) * 2 * W, host.data(),
                  static_cast<size_t>(std::min(nqq, maxb - r)) * row_bytes);
    perturb_rows(host.data(), maxb, db->dev.d, W, 0x7E57C0DE2506ull);
    err = hipMemcpyAsync(q, host.data(), maxb * row_bytes, hipMemcpyHostToDevice, s);
  }
  if (err == hipSuccess) err = hipStreamSynchronize(s);
  int rc = err == hipSuccess ? TQ_OK : hip_fail(err, "autotune set-up");
  const int cu = db->num_cu > 0 ? db->num_cu : 256;
  for (int ki = 0; ki < nks && rc == TQ_OK; ++ki) {
    const int k = ks[ki];
    if (k < 1 || k > TQ_MAX_K || k > db->dev.n) {
      rc = fail(TQ_ERR_INVALID, "autotune: k=%d outside [1, min(n, %d)]", k, TQ_MAX_K);
      break;
    }
    for (int b = 1; b <= maxb && rc == TQ_OK; b <<= 1) {
      std::vector<Shape> cands;
      Shape p;
      p.plain = true;
      if (b <= 8) cands.push_back(p);
      // the two largest query tiles that the bucket can fill, on 2x / 4x CU workgroups
      const int qmax = std::min(tqi::batched_max_qtile(k), std::max(2, b));
      for (int qt : {qmax / 2, qmax}) {
        if (qt < 2) continue;
        for (int gm : {2, 4}) {
          Shape c;
          c.qtile = qt;
          c.grid = cu * gm;
          cands.push_back(c);
        }
      }
      // matrix engine: the query tiles the bucket can fill, on 1x / 2x the
      // workgroups that fit at once
      for (int qt : {64, 128, 256}) {
        if (!tqi::mfma_supported(k, qt) || (qt > 64 && b <= qt / 2)) continue;
        const int resident = cu * mfma_resident_per_cu(k, qt);
        for (int gm : {1, 2}) {
          Shape c;
          c.engine = TQ_ENGINE_MATRIX;
          c.qtile = qt;
          c.grid = resident * gm;
          cands.push_back(c);
        }
      }
      Shape best;
      float best_ms = 1e30f;
      Shape per_tile[3];  // the best matrix shape with 64-, 128- and 256-query tiles
      for (const Shape &c : cands) {
        float ms = 0.f;
        rc = time_config(db, q, b, k, ids, scores, c, s, &ms);
        if (rc) break;
        if (verbose)
          std::fprintf(stderr, "[tq tune] k=%d bucket=%d %s qtile=%d grid=%d: %.3f ms\n", k, b,
                       c.plain ? "plain" : c.engine == TQ_ENGINE_MATRIX ? "matrix" : "popcount", c.qtile, c.grid, ms);
        if (ms < best_ms) {
          best_ms = ms;
          best = c;
          best.ms = ms;
        }
        if (!c.plain && c.engine == TQ_ENGINE_MATRIX) {
          Shape &t = per_tile[c.qtile == 64 ? 0 : c.qtile == 128 ? 1 : 2];
          if (t.ms <= 0.f || ms < t.ms) {
            t = c;
            t.ms = ms;
          }
        }
      }
      if (rc == TQ_OK)
        for (const Shape &t : per_tile)
          if (t.ms > 0.f) tune_store(db->dev, k, b, t, t.qtile);
      if (rc == TQ_OK) {
        if (best.plain) {  // keep a batched shape for explicit batched calls
          Shape d = default_shape(db, k, b);
          best.qtile = d.qtile;
          best.grid = d.grid;
          best.engine = d.engine;
        }
        tune_store(db->dev, k, b, best);
      }
    }
  }
  (void)hipStreamSynchronize(s);
  if (q) dev_free(q);
  if (ids) dev_free(ids);
  if (scores) dev_free(scores);
  return rc;
}

}  // namespace tqr
