// tq_internal.h -- internals shared by the HIP kernels and the host runtime of
// the ternary EVP search library.  Not part of the public ABI (include/tq.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tqi {

// ---------------------------------------------------------------------------
// Resident database layout
// ---------------------------------------------------------------------------
//
// The canonical code row (public layout) is [v+ : W words][v- : W words].
// On the device the database is re-tiled for streaming:
//
//   * 64 vectors form a tile, one vector per lane of a wave;
//   * each plane is padded to W4 = 4*nc words (nc 16-byte chunks);
//   * the planes are stored as nz = v+ | v- (the non-zero mask) and
//     ng = v- (the negative mask), a lossless re-coding of (v+, v-) that
//     lets Delta be evaluated with 5 integer operations per 32 coordinates
//     (see delta_word in tq_device.h);
//   * within a tile, chunk c of plane p of all 64 vectors is one contiguous
//     1 KiB run: uint4 index ((tile * 2 + p) * nc + c) * 64 + lane.
//
// Rows past n in the last tile are all-zero and are never reported.
constexpr int kTileVecs = 64;
constexpr int kMaxNc = 8;  // d <= 1024

struct DbDev {
  const uint4 *tiles;
  int64_t n;
  int64_t ntiles;
  int d, x, W, nc;
  // Index-list copy (sparse.hip) of a database with 8 x <= d, else null:
  // sc 16-byte chunks of 8 uint16 entries per vector, tiled like the planes.
  const uint4 *sparse = nullptr;
  int sc = 0;
};

constexpr int kMaxSparseChunks = 16;  // x <= 128 (8 x <= d <= 1024)

// ---------------------------------------------------------------------------
// Result keys
// ---------------------------------------------------------------------------
//
// A (score, id) pair is folded into one 64-bit key that orders "nearer" as
// "larger": high word = Delta + 2^31 (so unsigned order is score order), low
// word = 0xFFFFFFFF - id (so on equal score the lower id is larger).  The key
// is a strict total order over a database, so every partial top-k can be
// merged in any order to the same result.  0 is never a valid key (the high
// word of a valid key is at least 2^31 - x > 0) and marks an empty slot.
constexpr uint32_t kScoreBias = 0x80000000u;

__host__ __device__ inline uint64_t make_key(int32_t score, uint32_t id) {
  return (static_cast<uint64_t>(static_cast<uint32_t>(score) + kScoreBias) << 32) |
         static_cast<uint64_t>(0xFFFFFFFFu - id);
}
__host__ __device__ inline int32_t key_score(uint64_t key) {
  return static_cast<int32_t>(static_cast<uint32_t>(key >> 32) - kScoreBias);
}
__host__ __device__ inline int32_t key_id(uint64_t key) {
  return static_cast<int32_t>(0xFFFFFFFFu - static_cast<uint32_t>(key));
}

// Per-wave top-k lists hold 64*R keys (R per lane); R is one of 1, 2, 4, 8.
inline int rows_for_k(int k) {
  int r = (k + 63) / 64;
  return r <= 1 ? 1 : r <= 2 ? 2 : r <= 4 ? 4 : 8;
}

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files); all asynchronous on `s`.
// ---------------------------------------------------------------------------

// encode.hip
hipError_t encode_launch(const float *X, int64_t n, int d, int x, uint32_t *codes, int *flags,
                         int num_cu, hipStream_t s);

// b1.58 quantisation of each row (Sec. 4.3), same code layout and flags.
hipError_t b158_launch(const float *X, int64_t n, int d, uint32_t *codes, int *flags, int num_cu, hipStream_t s);

// layout.hip
hipError_t repack_launch(const uint32_t *codes, int64_t n, int d, uint4 *tiles, int64_t ntiles,
                         int nc, hipStream_t s);
hipError_t export_launch(const DbDev &db, uint32_t *codes, hipStream_t s);
hipError_t validate_launch(const uint32_t *codes, int64_t n, int d, int x,
                           unsigned long long *bad_rows, hipStream_t s);

// scan.hip
// One query against the whole database; `grid` workgroups, each writing one
// sorted list of k keys to partial[block * k ...].  Options: tstride > 1
// scans every tstride-th tile only (a sample); floor_ids / floor_scores (k
// each: a sample scan's result row for this query, device) let the scan drop
// keys below that row's k-th key.
// l2 != 0 scores 2 Delta - nnz(v) (the euclidean order between ternary
// vectors of varying non-zero counts) instead of Delta.
struct PlainScanOpts {
  int tstride = 1;
  const int32_t *floor_ids = nullptr;
  const int32_t *floor_scores = nullptr;
  int l2 = 0;
};
hipError_t scan_plain_launch(const DbDev &db, const uint32_t *qcode, int k, int grid,
                             uint64_t *partial, hipStream_t s, const PlainScanOpts &o = PlainScanOpts());
// For each of nq queries, merge its `nlists` sorted lists of k keys (laid out
// partial[(q * nlists + l) * k + i]) into the final ids / scores.  `mid`
// holds merge_mid_keys(nq, nlists, k) keys of scratch (may be null when 0).
int64_t merge_mid_keys(int nq, int nlists, int k);
hipError_t merge_launch(const uint64_t *partial, int nq, int nlists, int k, int32_t *ids,
                        int32_t *scores, uint64_t *mid, hipStream_t s);
hipError_t delta_dump_launch(const DbDev &db, const uint32_t *qcodes, int nq, int32_t *out,
                             hipStream_t s);

// sparse.hip: chunks of the index-list copy for (d, x), 0 where none is
// kept (x = 0 or 8 x > d); the copy is built from the resident bit planes
// (sc = sparse_chunks(d, x) chunks per vector, ntiles * sc * 64 uint4), and
// scanned like scan_plain_launch.
int sparse_chunks(int d, int x);
hipError_t sparse_repack_launch(const DbDev &db, uint4 *out, int sc, hipStream_t s);
hipError_t scan_sparse_launch(const DbDev &db, const uint32_t *qcode, int k, int grid, uint64_t *partial,
                              hipStream_t s);
// The plain path takes the index-list scan by itself where the list is at
// most half the bit planes' bytes (2x <= d/8).
inline bool sparse_preferred(const DbDev &db) { return db.sparse != nullptr && 16 * db.x <= db.d; }

// masked.hip: the masked-addition scan of one float query (d floats, device)
// against the database, writing `grid` sorted lists of k keys like
// scan_plain_launch; after merge_launch, rank_to_float_launch turns the int32
// scores (order-preserving key words of the float scores) into floats.
// The masked scan's options, as PlainScanOpts: a sample scan of every
// tstride-th tile, and the floor from a sample's merged result row (k ids,
// then k order-preserving score words) of this query.
struct MaskedScanOpts {
  int tstride = 1;
  const int32_t *floor_ids = nullptr;
  const int32_t *floor_scores = nullptr;
};
hipError_t scan_masked_launch(const DbDev &db, const float *q, int k, int grid, uint64_t *partial, hipStream_t s,
                              const MaskedScanOpts &o = MaskedScanOpts());
hipError_t rank_to_float_launch(int32_t *scores, int64_t count, hipStream_t s);
// Workgroups of the masked scan for (nc, k) that one compute unit holds at
// once (registers and LDS); 0 if the runtime cannot say.
int scan_masked_resident(int nc, int k);

// rerank.hip: the k best of each query's ncand candidate rows of X (n x d
// floats) by the double-precision scalar product with the query (nq x d).
constexpr int kMaxRerank = 1024;  // candidates per query
hipError_t rerank_launch(const float *X, int64_t n, int d, const float *Q, int nq, const int32_t *cand, int ncand,
                         int k, int32_t *ids, double *scores, hipStream_t s);

}  // namespace tqi
