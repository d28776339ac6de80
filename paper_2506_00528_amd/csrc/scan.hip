// scan.hip -- exhaustive kNN of one query over the resident database with the
// b2sp / Delta proxy (Sec. 5.1.2), and the per-query top-k merge.
//
// Plain single-query scan: the database is streamed once per query.  Work is
// split in tiles of 64 vectors; wave w of the grid takes tiles w, w + #waves,
// w + 2 #waves, ..., so at any moment the whole grid sweeps one contiguous
// window of memory (the access order that reaches the highest HBM read rate).
// A lane scores its tile vector against the query, whose nz / ng words sit in
// scalar registers; the wave keeps its best k keys in a register list and only
// offers keys above its current k-th key, so insertions are rare.  At the end
// the workgroup's wave lists are tree-merged in LDS and written out; a second
// kernel merges the workgroup lists of every query into ids and scores.
#include "tq_batched.h"
#include "tq_device.h"

namespace tqi {
namespace {

constexpr int kScanWaves = 4;
constexpr int kScanBlock = 64 * kScanWaves;

// `tstride` > 1 scans only every tstride-th tile (a sample of the database).
// `l2` != 0 scores 2 Delta - nnz(v) instead of Delta.
// With `floor_at` (the result row of a sample scan of this query, k ids then
// k scores), keys below the sample's k-th key are dropped from the start: the
// k-th key of a subset is never above the k-th key of the whole database.
template <int NC, int R>
__global__ __launch_bounds__(kScanBlock, 2) void scan_plain_kernel(const uint4 *__restrict__ tiles, int64_t n,
                                                               int64_t ntiles, int W,
                                                               const uint32_t *__restrict__ qcode, int k,
                                                               uint64_t *__restrict__ partial, int tstride,
                                                               const int32_t *__restrict__ floor_ids,
                                                               const int32_t *__restrict__ floor_scores, int l2) {
  __shared__ uint64_t lds[2][kScanWaves * 64 * R];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * kScanWaves;

  QueryWords<NC> q;
  q.load(qcode, W);

  WaveList<R> list;
  list.clear();
  uint64_t floor = 0;  // keys below the sample's k-th key are outside the result
  if (floor_ids && floor_ids[k - 1] >= 0)
    floor = make_key(floor_scores[k - 1], static_cast<uint32_t>(floor_ids[k - 1])) - 1;
  uint64_t thr = floor;
  const int km1 = k - 1;
  ntiles = (ntiles + tstride - 1) / tstride;  // tiles of this scan: t * tstride

  // Two tile buffers: the next tile's loads are in flight while the current
  // one is scored (past the end a wave re-reads the last tile, so the loads
  // need no branch).
  auto score = [&](const TileVec<NC> &v, int64_t t) {
    int32_t delta = vec_delta<NC>(v, q);
    if (l2) delta = 2 * delta - vec_nnz<NC>(v.vz);
    const int64_t id = t * tstride * 64 + lane;
    offer_keys<R>(list, thr, make_key(delta, static_cast<uint32_t>(id)), id < n, km1, floor);
  };
  const uint4 *last = tiles + ((ntiles - 1) * tstride) * (2 * NC * 64);
  auto tile_at = [&](int64_t t) { return t < ntiles ? tiles + (t * tstride) * (2 * NC * 64) : last; };
  int64_t t = static_cast<int64_t>(blockIdx.x) * kScanWaves + wave;
  if (t < ntiles) {
    TileVec<NC> a, b;
    a.load(tile_at(t), lane);
    while (true) {
      b.load(tile_at(t + nwaves), lane);
      score(a, t);
      t += nwaves;
      if (t >= ntiles) break;
      a.load(tile_at(t + nwaves), lane);
      score(b, t);
      t += nwaves;
      if (t >= ntiles) break;
    }
  }

  // workgroup merge of the wave lists (positions 0 .. k-1 of each)
  uint64_t *a = lds[0];
  uint64_t *b = lds[1];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = r * 64 + lane;
    if (p < k) a[wave * k + p] = list.v[r];
  }
  uint64_t *res = tree_merge(a, b, kScanWaves, k);
  for (int p = threadIdx.x; p < k; p += kScanBlock) partial[static_cast<int64_t>(blockIdx.x) * k + p] = res[p];
}

// Per-query merge of many sorted lists of k keys.  A workgroup tree-merges
// the lists in LDS in rounds of `chunk` lists (slot 0 carries the running
// result).  Many lists are merged in two stages: merge_groups_kernel gives
// every group of gl lists its own workgroup, then merge_lists_kernel merges
// the group results, so a query's merge is spread over several CUs.
constexpr int kMergeBlock = 1024;
constexpr int kMergeLdsKeys = 4096;  // per buffer (two buffers: 64 KiB)

// Stage 1: workgroup (q, g) merges lists [g*gl, (g+1)*gl) of query q (layout
// src[(q * nlists + l) * k]) into mid[(q * gmax + g) * k].  With `prm` the
// query and list counts come from the device parameter block.
__global__ __launch_bounds__(kMergeBlock) void merge_groups_kernel(const uint64_t *__restrict__ src, int nlists,
                                                                   int k, int gl, int gmax,
                                                                   const BatchParams *__restrict__ prm,
                                                                   uint64_t *__restrict__ mid) {
  __shared__ uint64_t buf[2][kMergeLdsKeys];
  const int q = blockIdx.x, g = blockIdx.y;
  if (prm) {
    if (q >= prm->nq) return;
    nlists = prm->parts;
  }
  const int first = g * gl;
  if (first >= nlists) return;
  const int take = min(gl, nlists - first);
  const uint64_t *lists = src + (static_cast<int64_t>(q) * nlists + first) * k;
  for (int i = threadIdx.x; i < gl * k; i += kMergeBlock) buf[0][i] = (i / k < take) ? lists[i] : 0ull;
  const uint64_t *res = tree_merge(buf[0], buf[1], gl, k);
  for (int i = threadIdx.x; i < k; i += kMergeBlock) mid[(static_cast<int64_t>(q) * gmax + g) * k + i] = res[i];
}

// Final stage: one workgroup per query merges its `nlists` lists (qstride
// lists per query in `src`).  With `prm`: the query count and outputs come
// from the parameter block; nlists = prm->parts, or ceil(prm->parts / gl_div)
// group results when the first stage ran; with prm->running set, the query's
// running list joins the merge and receives the result.
__global__ __launch_bounds__(kMergeBlock) void merge_lists_kernel(const uint64_t *__restrict__ src, int nlists,
                                                                  int qstride, int k, int chunk,
                                                                  int32_t *__restrict__ ids,
                                                                  int32_t *__restrict__ scores,
                                                                  const BatchParams *__restrict__ prm, int gl_div) {
  __shared__ uint64_t buf[2][kMergeLdsKeys];
  const int q = blockIdx.x;
  uint64_t *running = nullptr;
  if (prm) {
    if (q >= prm->nq) return;
    nlists = gl_div ? (prm->parts + gl_div - 1) / gl_div : prm->parts;
    if (!gl_div) qstride = nlists;
    ids = prm->ids;
    scores = prm->scores;
    if (prm->running)
      running = prm->running + static_cast<int64_t>(prm->slots ? prm->slots[q] : q) * prm->running_stride;
  }
  const uint64_t *lists = src + static_cast<int64_t>(q) * qstride * k;
  uint64_t *a = buf[0];
  uint64_t *b = buf[1];
  for (int i = threadIdx.x; i < k; i += kMergeBlock) a[i] = running ? running[i] : 0ull;
  for (int l0 = 0; l0 < nlists; l0 += chunk - 1) {
    const int take = min(chunk - 1, nlists - l0);
    for (int i = threadIdx.x; i < (chunk - 1) * k; i += kMergeBlock) {
      const int l = i / k;
      a[k + i] = (l < take) ? lists[static_cast<int64_t>(l0 + l) * k + (i - l * k)] : 0ull;
    }
    uint64_t *res = tree_merge(a, b, chunk, k);
    if (res != a) {
      for (int i = threadIdx.x; i < k; i += kMergeBlock) a[i] = res[i];
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < k; i += kMergeBlock) {
    const uint64_t key = a[i];
    if (running) {
      running[i] = key;
    } else {
      ids[static_cast<int64_t>(q) * k + i] = key ? key_id(key) : -1;
      scores[static_cast<int64_t>(q) * k + i] = key ? key_score(key) : 0;
    }
  }
}

// Delta of every (query, database vector) pair, for parity checks.
template <int NC>
__global__ __launch_bounds__(256) void delta_dump_kernel(const uint4 *__restrict__ tiles, int64_t n,
                                                         int64_t ntiles, int W,
                                                         const uint32_t *__restrict__ qcodes,
                                                         int32_t *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t t = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int qi = blockIdx.y;
  if (t >= ntiles) return;
  QueryWords<NC> q;
  q.load(qcodes + static_cast<int64_t>(qi) * 2 * W, W);
  const int32_t delta = tile_delta<NC>(tiles + t * (2 * NC * 64), lane, q);
  const int64_t id = t * 64 + lane;
  if (id < n) out[static_cast<int64_t>(qi) * n + id] = delta;
}

template <int NC, int R>
hipError_t scan_nc_r(const DbDev &db, const uint32_t *qcode, int k, int grid, uint64_t *partial,
                     const PlainScanOpts &o, hipStream_t s) {
  hipLaunchKernelGGL((scan_plain_kernel<NC, R>), dim3(grid), dim3(kScanBlock), 0, s, db.tiles, db.n,
                     db.ntiles, db.W, qcode, k, partial, o.tstride, o.floor_ids, o.floor_scores, o.l2);
  return hipGetLastError();
}

template <int NC>
hipError_t scan_nc(const DbDev &db, const uint32_t *qcode, int k, int grid, uint64_t *partial,
                   const PlainScanOpts &o, hipStream_t s) {
  switch (rows_for_k(k)) {
    case 1: return scan_nc_r<NC, 1>(db, qcode, k, grid, partial, o, s);
    case 2: return scan_nc_r<NC, 2>(db, qcode, k, grid, partial, o, s);
    case 4: return scan_nc_r<NC, 4>(db, qcode, k, grid, partial, o, s);
    default: return scan_nc_r<NC, 8>(db, qcode, k, grid, partial, o, s);
  }
}

template <int NC>
hipError_t dump_nc(const DbDev &db, const uint32_t *qcodes, int nq, int32_t *out, hipStream_t s) {
  const unsigned gx = static_cast<unsigned>((db.ntiles + 3) / 4);
  hipLaunchKernelGGL((delta_dump_kernel<NC>), dim3(gx, nq), dim3(256), 0, s, db.tiles, db.n, db.ntiles, db.W,
                     qcodes, out);
  return hipGetLastError();
}

}  // namespace

hipError_t scan_plain_launch(const DbDev &db, const uint32_t *qcode, int k, int grid, uint64_t *partial,
                             hipStream_t s, const PlainScanOpts &o) {
  if (o.tstride < 1) return hipErrorInvalidValue;
  switch (db.nc) {
    case 1: return scan_nc<1>(db, qcode, k, grid, partial, o, s);
    case 2: return scan_nc<2>(db, qcode, k, grid, partial, o, s);
    case 3: return scan_nc<3>(db, qcode, k, grid, partial, o, s);
    case 4: return scan_nc<4>(db, qcode, k, grid, partial, o, s);
    case 5: return scan_nc<5>(db, qcode, k, grid, partial, o, s);
    case 6: return scan_nc<6>(db, qcode, k, grid, partial, o, s);
    case 7: return scan_nc<7>(db, qcode, k, grid, partial, o, s);
    case 8: return scan_nc<8>(db, qcode, k, grid, partial, o, s);
    default: return hipErrorInvalidValue;
  }
}

// Lists per merge round: the largest power of two with chunk * k keys in one
// LDS buffer (at most 512).
static int merge_chunk(int k) {
  int chunk = 2;
  while (chunk * 2 * k <= kMergeLdsKeys && chunk < 512) chunk *= 2;
  return chunk;
}

int64_t merge_mid_keys(int nq, int nlists, int k) {
  const int chunk = merge_chunk(k);
  if (nlists <= chunk - 1) return 0;
  return static_cast<int64_t>(nq) * ((nlists + chunk - 1) / chunk) * k;
}

hipError_t merge_launch(const uint64_t *partial, int nq, int nlists, int k, int32_t *ids, int32_t *scores,
                        uint64_t *mid, hipStream_t s) {
  const int chunk = merge_chunk(k);
  if (chunk * k > kMergeLdsKeys) return hipErrorInvalidValue;
  if (nlists <= chunk - 1) {
    hipLaunchKernelGGL(merge_lists_kernel, dim3(nq), dim3(kMergeBlock), 0, s, partial, nlists, nlists, k, chunk, ids,
                       scores, static_cast<const BatchParams *>(nullptr), 0);
    return hipGetLastError();
  }
  const int gmax = (nlists + chunk - 1) / chunk;
  hipLaunchKernelGGL(merge_groups_kernel, dim3(nq, gmax), dim3(kMergeBlock), 0, s, partial, nlists, k, chunk, gmax,
                     static_cast<const BatchParams *>(nullptr), mid);
  hipLaunchKernelGGL(merge_lists_kernel, dim3(nq), dim3(kMergeBlock), 0, s, static_cast<const uint64_t *>(mid), gmax,
                     gmax, k, chunk, ids, scores, static_cast<const BatchParams *>(nullptr), 0);
  return hipGetLastError();
}

int64_t merge_batched_mid_keys(int bucket, int max_parts, int k) {
  const int chunk = merge_chunk(k);
  return static_cast<int64_t>(bucket) * ((max_parts + chunk - 1) / chunk) * k;
}

hipError_t merge_batched_launch(const uint64_t *partial, const BatchParams *prm, int bucket, int k, int max_parts,
                                uint64_t *mid, hipStream_t s) {
  const int chunk = merge_chunk(k);
  if (chunk * k > kMergeLdsKeys) return hipErrorInvalidValue;
  const int gmax = (max_parts + chunk - 1) / chunk;
  hipLaunchKernelGGL(merge_groups_kernel, dim3(bucket, gmax), dim3(kMergeBlock), 0, s, partial, 0, k, chunk, gmax,
                     prm, mid);
  hipLaunchKernelGGL(merge_lists_kernel, dim3(bucket), dim3(kMergeBlock), 0, s, static_cast<const uint64_t *>(mid), 0,
                     gmax, k, chunk, static_cast<int32_t *>(nullptr), static_cast<int32_t *>(nullptr), prm, chunk);
  return hipGetLastError();
}

hipError_t delta_dump_launch(const DbDev &db, const uint32_t *qcodes, int nq, int32_t *out, hipStream_t s) {
  switch (db.nc) {
    case 1: return dump_nc<1>(db, qcodes, nq, out, s);
    case 2: return dump_nc<2>(db, qcodes, nq, out, s);
    case 3: return dump_nc<3>(db, qcodes, nq, out, s);
    case 4: return dump_nc<4>(db, qcodes, nq, out, s);
    case 5: return dump_nc<5>(db, qcodes, nq, out, s);
    case 6: return dump_nc<6>(db, qcodes, nq, out, s);
    case 7: return dump_nc<7>(db, qcodes, nq, out, s);
    case 8: return dump_nc<8>(db, qcodes, nq, out, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tqi
