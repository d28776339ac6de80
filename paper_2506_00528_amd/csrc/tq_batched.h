// tq_batched.h -- internals of the batched search path shared by its kernels
// (batched_kernels.hip, scan.hip's merge) and its host runtime (batched.cpp).
#pragma once

#include "tq_internal.h"

namespace tqi {

// Per-call values of a batched search, written on the device by
// batch_prep_kernel so that the scan and merge launches keep fixed arguments
// (and can be replayed from a captured hipGraph).
struct BatchParams {
  int nq;                  // real queries of the call (<= bucket)
  int nqt;                 // query tiles: ceil(nq / qtile)
  int parts;               // database parts: the grid gets nqt * parts work items
  int l2;                  // 1: score 2 Delta - nnz(v) (TQ_METRIC_L2), 0: Delta
  int64_t tiles_per_part;  // 64-vector tiles per part
  int64_t tile_lo;         // database tiles scanned: [tile_lo, tile_hi)
  int64_t tile_hi;
  const int *slots;        // optional: query i's running list is row slots[i] of
                           // `running` (else row i); the scan always reads query
                           // rows compactly (row i for query i)
  uint64_t *running;       // optional: per-row running top-k merged with this
                           // pass and written back instead of ids / scores
  int64_t running_stride;  // keys per running row (>= the call's k)
  int32_t *ids;            // caller's outputs, nq x k (when running is null)
  int32_t *scores;
  uint64_t *bound;         // optional: nq x parts x kBoundSlotsPerPart keys,
                           // zero before the scan; the scans publish there the
                           // m-th keys of their (query, part) or (query, part,
                           // wave) lists and drop keys below the smallest of a
                           // query's (see scan_mfma_kernel,
                           // scan_batched_kernel); null: no such pruning
};
// Bound slots per (query, part): the popcount scan's four waves each keep
// their own lists; the matrix scan uses the first slot block only.
constexpr int kBoundSlotsPerPart = 4;

// Work items are (query tile, database part) pairs.  The hardware dispatcher
// places workgroup b on XCD b mod 8, and a persistent workgroup keeps item
// indices b, b + grid, ... (grid a multiple of 8), so an item's XCD is its
// index mod 8.  Items are numbered so that every query tile of a database
// part runs on the same XCD at about the same time and shares the part's
// tiles through that XCD's L2: item i -> XCD x = i mod 8, r = i div 8,
// query tile r mod nqt, part 8 (r div nqt) + x.  The part count is a multiple
// of 8 (trailing parts may be empty).
constexpr int kXcds = 8;

__host__ __device__ inline void item_coords(int item, int nqt, int *qt, int *part) {
  const int x = item % kXcds, r = item / kXcds;
  *qt = r % nqt;
  *part = (r / nqt) * kXcds + x;
}

// Fill of the derived split of a batch over tiles [lo, hi).  The grid is
// persistent: its workgroups take items (query tile, part) in rounds of
// `grid`, and a launch lasts about rounds x (tiles per part).  The part count
// (a multiple of 8) minimises rounds / parts over one or two rounds; a
// second round is considered only where one round leaves more than a quarter
// of the grid idle, and must then promise a tenth less, since more parts also
// cost list fills (k keys each) and merge work.  So nq x parts <= kMaxRounds x qtile x grid + 8 nq (the list
// buffers' size) and parts <= kMaxRounds x grid + 8 (the merge's bound).  A count rounded up from grid / nqt instead would leave a
// few items for a second round and nearly double the launch (3 query tiles
// on 512 workgroups: 528 items); one round of fewer items can instead leave
// compute units with a single workgroup (40 query tiles: 320 items), where
// two full rounds of smaller parts finish sooner.
constexpr int kMaxRounds = 2;
__host__ __device__ inline void batch_split(BatchParams &b, int nq, int qtile, int grid, int64_t lo, int64_t hi) {
  b.nq = nq;
  b.nqt = (nq + qtile - 1) / qtile;
  const int64_t ntiles = hi - lo;
  const int64_t cap = (ntiles + kXcds - 1) / kXcds * kXcds;  // no more parts than tiles, rounded up
  int64_t parts = kXcds;
  if (b.nqt > 0 && grid > 0) {
    int64_t best_rounds = 0;
    for (int r = 1; r <= kMaxRounds; ++r) {
      int64_t p = static_cast<int64_t>(r) * grid / (static_cast<int64_t>(kXcds) * b.nqt) * kXcds;
      if (p > cap) p = cap;
      if (p < kXcds) p = kXcds;
      const int64_t rounds = (static_cast<int64_t>(b.nqt) * p + grid - 1) / grid;
      if (r == 1 || 10 * rounds * parts < 9 * best_rounds * p) {
        parts = p;
        best_rounds = rounds;
      }
      // one round that fills three quarters of the grid is kept
      if (r == 1 && 4 * static_cast<int64_t>(b.nqt) * p >= 3 * static_cast<int64_t>(grid)) break;
    }
  }
  b.parts = static_cast<int>(parts);
  b.l2 = 0;
  b.running_stride = 0;
  b.tiles_per_part = (ntiles + parts - 1) / parts;
  b.tile_lo = lo;
  b.tile_hi = hi;
}

// The split of a sample pass over every `tstride`-th tile of the call's range
// [prm.tile_lo, prm.tile_hi): sample tile i is database tile
// prm.tile_lo + i tstride, and the sample is split like a database of
// ceil(range / tstride) tiles.  (Its lists only feed a floor, never a result.)
__host__ __device__ inline void sample_split(BatchParams &b, const BatchParams &prm, int qtile, int grid,
                                             int tstride) {
  batch_split(b, prm.nq, qtile, grid, 0, (prm.tile_hi - prm.tile_lo + tstride - 1) / tstride);
  b.slots = nullptr;
  b.running = nullptr;
  b.ids = nullptr;
  b.scores = nullptr;
  b.bound = nullptr;
}

// Keys kept per (query, part) by a sample pass for a search of k: 8 where the
// parts can hold at least 2k of them, else 16 (kGroupMaxK).
__host__ __device__ inline int sample_list_len(int parts, int k) { return parts * 8 >= 2 * k ? 8 : 16; }

// Bounds that hold for every split of up to `nq` queries on `grid`
// workgroups: the parts of one query, and the (query, part) lists of a call.
inline int batch_max_parts(int grid) { return kMaxRounds * grid + kXcds; }
inline size_t batch_max_lists(int qtile, int grid, int nq) {
  return static_cast<size_t>(kMaxRounds) * qtile * grid + static_cast<size_t>(kXcds + 1) * nq;
}

// Largest query tile the batched scan supports for this k.
int batched_max_qtile(int k);

// `bound` (may be null) holds at least nq * parts * kBoundSlotsPerPart keys;
// the prep kernel zeroes them.
// `l2` selects the score (BatchParams::l2).
hipError_t batch_prep_launch(const uint32_t *qcodes, int nq, int bucket, const DbDev &db, int qtile, int grid,
                             int32_t *ids, int32_t *scores, uint32_t *qprep, BatchParams *prm, uint64_t *bound,
                             int l2, hipStream_t s);
hipError_t scan_batched_launch(const DbDev &db, const uint32_t *qprep, const BatchParams *prm, int k, int qtile,
                               int grid, uint64_t *partial, hipStream_t s);
// The same scan on the fp4 matrix cores (mfma_kernels.hip): k <= 128 with
// query tiles of 64, 128 or 256 per workgroup.
constexpr int kGroupMaxK = 16;
bool mfma_supported(int k, int qtile);
// max_part_tiles: an upper bound on prm->tiles_per_part for this launch (the
// k > 16 scan keys ids relative to their part where parts span <= 2^20 vectors).
// Sample floor (k > 16 only; sample.stride == 0: none): a first pass scores
// every stride-th tile with lists of sample_list_len keys, a per-query
// histogram of those keys gives the largest score s that at least k of them
// reach (no key of the final top-k scores below s), and the full scan drops
// keys scoring below s.  sample.floor holds one key per query of the bucket;
// the sample's lists reuse `partial` (at most 16 < k keys per list).
struct MfmaSample {
  int stride = 0;
  int bucket = 0;
  uint64_t *floor = nullptr;
};
hipError_t scan_mfma_launch(const DbDev &db, const uint32_t *qprep, const BatchParams *prm, int k, int qtile,
                            int grid, int64_t max_part_tiles, uint64_t *partial, hipStream_t s,
                            const MfmaSample &sample = MfmaSample());
// one plane width (mfma_kernels.hip, compiled per NC); called by scan_mfma_launch
template <int NC>
hipError_t scan_mfma_launch_nc(const DbDev &db, const uint32_t *qprep, const BatchParams *prm, int k, int qtile,
                               int grid, int64_t max_part_tiles, uint64_t *partial, hipStream_t s,
                               const MfmaSample &sample);
// Per-query merge of the (query, part) lists; the query count, part count and
// output pointers come from `prm`; at most max_parts parts per query.  With
// prm->running set, each query's running list joins the merge and receives
// the result.  `mid` holds merge_batched_mid_keys(bucket, max_parts, k) keys.
int64_t merge_batched_mid_keys(int bucket, int max_parts, int k);
hipError_t merge_batched_launch(const uint64_t *partial, const BatchParams *prm, int bucket, int k, int max_parts,
                                uint64_t *mid, hipStream_t s);

// Canonical query codes -> nz/ng rows (the layout the batched scan reads).
hipError_t prep_rows_launch(const uint32_t *qcodes, int nq, const DbDev &db, uint32_t *rows, hipStream_t s);
// rows[i] = src[slots[i]] for `count` rows of `words` 32-bit words.
hipError_t gather_rows_launch(const uint32_t *src, const int *slots, int count, int words, uint32_t *rows,
                              hipStream_t s);
// Zero `count` 64-bit words (a fill kernel, safe inside captured graphs).
hipError_t fill_zero_launch(uint64_t *p, int64_t count, hipStream_t s);
// ids / scores from the running lists of rows slots[0..count): row slots[i]
// of `ids` / `scores` (k per row) receives that row's result.
hipError_t running_results_launch(const uint64_t *running, const int *slots, int count, int k, int32_t *ids,
                                  int32_t *scores, hipStream_t s);

}  // namespace tqi
