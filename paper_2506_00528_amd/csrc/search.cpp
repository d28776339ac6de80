// search.cpp -- the plain search path: one full database pass per query.
#include <algorithm>

#include "tq_runtime.h"

namespace tqr {

namespace {
// Partial lists of one merge round stay under this many bytes of scratch.
constexpr size_t kPartialBudget = size_t(64) << 20;
// Sample scans: every 32nd tile, on databases of at least 2 048 tiles (the
// sample then holds >= 4 096 vectors, eight times the largest k), when a wave
// scans fewer than 7 k vectors, or fewer than 32 k for k > 128 -- then a large
// share of all keys would enter some wave's list.  Measured per query: on
// N = 1e7, d = 1024 (4 883 vectors per wave) k = 512 falls from about 0.95 ms
// to 0.49 ms and k = 200 is 0.43 ms, while at k = 100 (49 k per wave) the
// sample would cost 0.03 ms more than it saves; on N = 1e6, d = 768 (488 per
// wave) k = 100 falls from 0.069 ms to 0.049 ms and k = 128 from 0.077 ms to
// 0.048 ms, while k = 32 would rise from 0.038 ms to 0.045 ms.
constexpr int kSampleStride = 32;
constexpr int64_t kSampleMinTiles = 2048;
bool use_sample(int64_t per_wave, int k) {
  return per_wave < 7 * static_cast<int64_t>(k) || (k > 128 && per_wave < 32 * static_cast<int64_t>(k));
}
}  // namespace

// Two workgroups of four waves per compute unit keep 16 KiB of loads in flight
// per wave (d = 1024); never more waves than tiles.
int default_plain_grid(const tq_db *db) {
  const int64_t by_tiles = (db->dev.ntiles + 3) / 4;
  const int64_t by_cu = static_cast<int64_t>(db->num_cu > 0 ? db->num_cu : 256) * 2;
  return static_cast<int>(std::max<int64_t>(1, std::min(by_tiles, by_cu)));
}

// The index-list scan holds few registers and reads at most half the bytes
// per vector: eight workgroups per compute unit keep enough loads in flight.
static int default_sparse_grid(const tq_db *db) {
  const int64_t by_tiles = (db->dev.ntiles + 3) / 4;
  const int64_t by_cu = static_cast<int64_t>(db->num_cu > 0 ? db->num_cu : 256) * 8;
  return static_cast<int>(std::max<int64_t>(1, std::min(by_tiles, by_cu)));
}

int search_plain(tq_db *db, const uint32_t *qcodes, int nq, int k, int32_t *ids, int32_t *scores, int grid,
                 int engine, hipStream_t s, const ScratchSpan *ext, int metric) {
  const int l2 = metric == TQ_METRIC_L2 ? 1 : 0;
  if (l2 && engine == TQ_ENGINE_SPARSE) return fail(TQ_ERR_INVALID, "the index-list engine scores Delta only");
  const bool sparse =
      engine == TQ_ENGINE_SPARSE || (engine == TQ_ENGINE_AUTO && !l2 && tqi::sparse_preferred(db->dev));
  if (sparse && !db->dev.sparse) return fail(TQ_ERR_INVALID, "no index-list copy of this database");
  const int G = grid > 0 ? grid : sparse ? default_sparse_grid(db) : default_plain_grid(db);
  // Large k against the vectors a wave scans: each wave keeps k keys of its
  // share, so many keys enter some list.  A first scan of every
  // kSampleStride-th tile gives each query a floor (the sample's k-th key,
  // never above the k-th key overall) below which the full scan drops keys.
  const int64_t per_wave = db->dev.ntiles * 64 / (static_cast<int64_t>(G) * 4);
  const bool sampled = !sparse && db->dev.ntiles >= kSampleMinTiles && use_sample(per_wave, k);
  const size_t per_query = static_cast<size_t>(G) * k * sizeof(uint64_t);
  const size_t per_query_all = per_query + (sampled ? 2 * static_cast<size_t>(k) * sizeof(int32_t) : 0);
  int chunk;
  void *p = nullptr;
  if (ext) {
    // A caller's fixed buffer: as many queries per merge round as fit, with
    // the merge's intermediate keys (linear in the round's query count).
    const size_t need1 = per_query_all + static_cast<size_t>(tqi::merge_mid_keys(1, G, k)) * sizeof(uint64_t);
    if (need1 > ext->bytes)
      return fail(TQ_ERR_INVALID, "grid=%d, k=%d needs %zu bytes of scratch per query, more than the %zu available",
                  G, k, need1, ext->bytes);
    chunk = static_cast<int>(std::min<size_t>(nq, ext->bytes / need1));
    p = ext->p;
  } else {
    chunk = static_cast<int>(std::max<size_t>(1, std::min<size_t>(nq, kPartialBudget / per_query_all)));
  }
  const size_t mid_keys = static_cast<size_t>(tqi::merge_mid_keys(chunk, G, k));
  if (!ext) {
    int rc = scratch_get(db->scratch, s, per_query_all * chunk + mid_keys * sizeof(uint64_t), &p);
    if (rc) return rc;
  }
  const bool timed = ext == nullptr;  // event creation stays off the no-allocation path
  uint64_t *partial = static_cast<uint64_t *>(p);
  uint64_t *mid = partial + static_cast<size_t>(chunk) * G * k;
  // sample results: chunk x k ids, then chunk x k scores
  int32_t *smp_ids = reinterpret_cast<int32_t *>(mid + mid_keys);
  int32_t *smp_scores = smp_ids + static_cast<size_t>(chunk) * k;
  const int row_words = 2 * db->dev.W;
  for (int q0 = 0; q0 < nq; q0 += chunk) {
    const int nc = std::min(chunk, nq - q0);
    if (sampled) {
      tqi::PlainScanOpts o;
      o.tstride = kSampleStride;
      o.l2 = l2;
      for (int i = 0; i < nc; ++i) {
        TimedLaunch t(kTimePlain, s, timed);
        hipError_t e = tqi::scan_plain_launch(db->dev, qcodes + static_cast<int64_t>(q0 + i) * row_words, k, G,
                                              partial + static_cast<size_t>(i) * G * k, s, o);
        if (e != hipSuccess) return hip_fail(e, "sample scan launch");
      }
      hipError_t e = tqi::merge_launch(partial, nc, G, k, smp_ids, smp_scores, mid, s);
      if (e != hipSuccess) return hip_fail(e, "sample merge launch");
    }
    for (int i = 0; i < nc; ++i) {
      TimedLaunch t(sparse ? kTimeSparse : kTimePlain, s, timed);
      const uint32_t *qc = qcodes + static_cast<int64_t>(q0 + i) * row_words;
      uint64_t *dst = partial + static_cast<size_t>(i) * G * k;
      tqi::PlainScanOpts o;
      o.l2 = l2;
      if (sampled) {
        o.floor_ids = smp_ids + static_cast<size_t>(i) * k;
        o.floor_scores = smp_scores + static_cast<size_t>(i) * k;
      }
      hipError_t e = sparse ? tqi::scan_sparse_launch(db->dev, qc, k, G, dst, s)
                            : tqi::scan_plain_launch(db->dev, qc, k, G, dst, s, o);
      if (e != hipSuccess) return hip_fail(e, "plain scan launch");
    }
    hipError_t e = tqi::merge_launch(partial, nc, G, k, ids + static_cast<int64_t>(q0) * k,
                                     scores + static_cast<int64_t>(q0) * k, mid, s);
    if (e != hipSuccess) return hip_fail(e, "merge launch");
  }
  return TQ_OK;
}

// Masked addition of float queries (one database pass per query, like the
// plain path); the merge's int32 scores are the order-preserving key words of
// the float scores and are turned back into floats in place.
// The table reads need every resident slot filled to hide their latency: by
// default one workgroup per slot on every compute unit.
static int default_masked_grid(const tq_db *db, int k) {
  const int64_t by_tiles = (db->dev.ntiles + 3) / 4;
  const int per_cu = std::max(2, tqi::scan_masked_resident(db->dev.nc, k));
  const int64_t by_cu = static_cast<int64_t>(db->num_cu > 0 ? db->num_cu : 256) * per_cu;
  return static_cast<int>(std::max<int64_t>(1, std::min(by_tiles, by_cu)));
}

int search_masked(tq_db *db, const float *Q, int nq, int k, int32_t *ids, float *scores, int grid, hipStream_t s) {
  const int G = grid > 0 ? grid : default_masked_grid(db, k);
  // the plain path's sample floor, on the same rule (measured on N = 1e7,
  // d = 1024 at the default grid: k = 200 0.73 -> 0.57 ms, k = 512 1.38 ->
  // 0.66 ms per query; at k <= 100 the sample would cost more than it saves,
  // 0.49 -> 0.52 ms at k = 10)
  const int64_t per_wave = db->dev.ntiles * 64 / (static_cast<int64_t>(G) * 4);
  const bool sampled = db->dev.ntiles >= kSampleMinTiles && use_sample(per_wave, k);
  const size_t per_query = static_cast<size_t>(G) * k * sizeof(uint64_t);
  const size_t per_query_all = per_query + (sampled ? 2 * static_cast<size_t>(k) * sizeof(int32_t) : 0);
  const int chunk = static_cast<int>(std::max<size_t>(1, std::min<size_t>(nq, kPartialBudget / per_query_all)));
  const size_t mid_keys = static_cast<size_t>(tqi::merge_mid_keys(chunk, G, k));
  void *p = nullptr;
  int rc = scratch_get(db->scratch, s, per_query_all * chunk + mid_keys * sizeof(uint64_t), &p);
  if (rc) return rc;
  uint64_t *partial = static_cast<uint64_t *>(p);
  uint64_t *mid = partial + static_cast<size_t>(chunk) * G * k;
  // sample results: chunk x k ids, then chunk x k order-preserving score words
  int32_t *smp_ids = reinterpret_cast<int32_t *>(mid + mid_keys);
  int32_t *smp_scores = smp_ids + static_cast<size_t>(chunk) * k;
  int32_t *iscores = reinterpret_cast<int32_t *>(scores);
  for (int q0 = 0; q0 < nq; q0 += chunk) {
    const int nc = std::min(chunk, nq - q0);
    if (sampled) {
      tqi::MaskedScanOpts o;
      o.tstride = kSampleStride;
      for (int i = 0; i < nc; ++i) {
        TimedLaunch t(kTimeMasked, s);
        hipError_t e = tqi::scan_masked_launch(db->dev, Q + static_cast<int64_t>(q0 + i) * db->dev.d, k, G,
                                               partial + static_cast<size_t>(i) * G * k, s, o);
        if (e != hipSuccess) return hip_fail(e, "masked sample scan launch");
      }
      hipError_t e = tqi::merge_launch(partial, nc, G, k, smp_ids, smp_scores, mid, s);
      if (e != hipSuccess) return hip_fail(e, "masked sample merge launch");
    }
    for (int i = 0; i < nc; ++i) {
      TimedLaunch t(kTimeMasked, s);
      tqi::MaskedScanOpts o;
      if (sampled) {
        o.floor_ids = smp_ids + static_cast<size_t>(i) * k;
        o.floor_scores = smp_scores + static_cast<size_t>(i) * k;
      }
      hipError_t e = tqi::scan_masked_launch(db->dev, Q + static_cast<int64_t>(q0 + i) * db->dev.d, k, G,
                                             partial + static_cast<size_t>(i) * G * k, s, o);
      if (e != hipSuccess) return hip_fail(e, "masked scan launch");
    }
    hipError_t e = tqi::merge_launch(partial, nc, G, k, ids + static_cast<int64_t>(q0) * k,
                                     iscores + static_cast<int64_t>(q0) * k, mid, s);
    if (e == hipSuccess) e = tqi::rank_to_float_launch(iscores + static_cast<int64_t>(q0) * k,
                                                       static_cast<int64_t>(nc) * k, s);
    if (e != hipSuccess) return hip_fail(e, "masked merge launch");
  }
  return TQ_OK;
}

}  // namespace tqr
