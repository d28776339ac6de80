// batched_kernels.hip -- all queries of a batch share each database pass.
//
// A persistent grid walks work items (query tile, database part); item i is
// tile (i mod nqt) of part (i div nqt), so consecutive workgroups read the
// same database part at the same time and share it through L2.  The four
// waves of a workgroup split the part's 64-vector tiles; a lane keeps its
// tile vector's two planes in VGPRs and scores it against every query of the
// tile, reading the query words through the scalar unit.  Each wave keeps one
// register top-k list per query; at the end of an item the four wave lists of
// each query are tree-merged in LDS and written as that (query, part) list.
//
// Per-call values (query count, derived split) sit in a small device block
// written by batch_prep_kernel, so the scan and merge launches have fixed
// arguments and can be captured once in a hipGraph per batch-size bucket and
// replayed.  Query tiles past the real query count are skipped, never scored.
#include "tq_batched.h"
#include "tq_device.h"

namespace tqi {
namespace {

constexpr int kBatchWaves = 4;
constexpr int kBatchBlock = 64 * kBatchWaves;
static_assert(kBatchWaves == kBoundSlotsPerPart, "one bound slot per wave of a part");

// Canonical query codes -> nz/ng words padded to 4*nc per plane (the layout
// the scan reads); rows in [nq, rows) are written as zeros.
__global__ __launch_bounds__(256) void prep_rows_kernel(const uint32_t *__restrict__ qcodes, int nq, int rows, int W,
                                                        int nc, uint32_t *__restrict__ qprep) {
  const int W4 = 4 * nc;
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= static_cast<int64_t>(rows) * W4) return;
  const int q = static_cast<int>(g / W4);
  const int w = static_cast<int>(g - static_cast<int64_t>(q) * W4);
  uint32_t p = 0, m = 0;
  if (q < nq && w < W) {
    p = qcodes[static_cast<int64_t>(q) * 2 * W + w];
    m = qcodes[static_cast<int64_t>(q) * 2 * W + W + w];
  }
  qprep[static_cast<int64_t>(q) * 2 * W4 + w] = p | m;
  qprep[static_cast<int64_t>(q) * 2 * W4 + W4 + w] = m;
}

// Query rows for one search call plus the call's parameters.
__global__ __launch_bounds__(256) void batch_prep_kernel(const uint32_t *__restrict__ qcodes, int nq, int bucket,
                                                         int W, int nc, int qtile, int grid, int64_t ntiles,
                                                         int32_t *ids, int32_t *scores, uint32_t *__restrict__ qprep,
                                                         BatchParams *__restrict__ prm, uint64_t *__restrict__ bound,
                                                         int l2) {
  const int W4 = 4 * nc;
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (bound) {
    BatchParams b;
    batch_split(b, nq, qtile, grid, 0, ntiles);
    const int64_t nb = static_cast<int64_t>(nq) * b.parts * kBoundSlotsPerPart;
    for (int64_t i = g; i < nb; i += static_cast<int64_t>(gridDim.x) * blockDim.x) bound[i] = 0;
  }
  if (g < static_cast<int64_t>(bucket) * W4) {
    const int q = static_cast<int>(g / W4);
    const int w = static_cast<int>(g - static_cast<int64_t>(q) * W4);
    uint32_t p = 0, m = 0;
    if (q < nq && w < W) {
      p = qcodes[static_cast<int64_t>(q) * 2 * W + w];
      m = qcodes[static_cast<int64_t>(q) * 2 * W + W + w];
    }
    qprep[static_cast<int64_t>(q) * 2 * W4 + w] = p | m;
    qprep[static_cast<int64_t>(q) * 2 * W4 + W4 + w] = m;
  }
  if (g == 0) {
    BatchParams b;
    batch_split(b, nq, qtile, grid, 0, ntiles);
    b.slots = nullptr;
    b.running = nullptr;
    b.ids = ids;
    b.scores = scores;
    b.bound = bound;
    b.l2 = l2;
    *prm = b;
  }
}

// rows[i] = src[slots[i]] for rows of `words` 32-bit words.
__global__ __launch_bounds__(256) void gather_rows_kernel(const uint32_t *__restrict__ src,
                                                          const int *__restrict__ slots, int count, int words,
                                                          uint32_t *__restrict__ rows) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= static_cast<int64_t>(count) * words) return;
  const int i = static_cast<int>(g / words);
  const int w = static_cast<int>(g - static_cast<int64_t>(i) * words);
  rows[g] = src[static_cast<int64_t>(slots[i]) * words + w];
}

__global__ __launch_bounds__(256) void fill_zero_kernel(uint64_t *__restrict__ p, int64_t count) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g < count) p[g] = 0;
}

__global__ __launch_bounds__(256) void running_results_kernel(const uint64_t *__restrict__ running,
                                                              const int *__restrict__ slots, int count, int k,
                                                              int32_t *__restrict__ ids,
                                                              int32_t *__restrict__ scores) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= static_cast<int64_t>(count) * k) return;
  const int i = static_cast<int>(g / k);
  const int j = static_cast<int>(g - static_cast<int64_t>(i) * k);
  const int64_t at = static_cast<int64_t>(slots[i]) * k + j;
  const uint64_t key = running[at];
  ids[at] = key ? key_id(key) : -1;
  scores[at] = key ? key_score(key) : 0;
}

// delta_word with each accumulation kept as one popcount-and-add: the empty
// asm makes the running sums opaque, so the compiler cannot regroup the adds
// into three-input sums of separate popcounts (two popcounts and an add per
// two words instead of two popcount-accumulates).
__device__ __forceinline__ void delta_word_chained(DeltaAcc &a, uint32_t qnz, uint32_t qng, uint32_t vnz,
                                                   uint32_t vng) {
  const uint32_t both = qnz & vnz;
  const uint32_t dis = both & (qng ^ vng);
  a.both = __popc(both) + a.both;
  a.dis = __popc(dis) + a.dis;
  asm volatile("" : "+v"(a.both), "+v"(a.dis));
}

// offer_keys with the lanes that hold a vector given as a ballot taken once
// per tile: the candidate mask is the ballot of the compare itself, with no
// detour through a 0/1 register
template <int R>
__device__ __forceinline__ void offer_keys_masked(WaveList<R> &list, uint64_t &thr, uint64_t key, uint64_t okmask,
                                                  int k_minus_1, uint64_t floor) {
  uint64_t m = __builtin_amdgcn_ballot_w64(key > thr) & okmask;
  while (m) {
    const int src = __builtin_ctzll(m);
    m &= m - 1;
    const uint64_t c = readlane64(key, src);
    if (c > thr) {
      list.insert(c);
      thr = list.at(k_minus_1);
      if (thr < floor) thr = floor;
    }
  }
}

template <int NC, int R, int QT>
__global__ __launch_bounds__(kBatchBlock) void scan_batched_kernel(const uint4 *__restrict__ tiles, int64_t n,
                                                                  int64_t ntiles,
                                                                  const uint32_t *__restrict__ qprep,
                                                                  const BatchParams *__restrict__ prm, int k,
                                                                  uint64_t *__restrict__ partial) {
  __shared__ uint64_t lds[2][kBatchWaves * 64 * R];
  __shared__ uint64_t lbs[kBatchWaves * QT];  // each query's bound from the other waves and parts
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nq = prm->nq, nqt = prm->nqt, parts = prm->parts;
  // score = Delta * mul - sub: Delta, or 2 Delta - nnz(v) for the l2 order
  const int32_t mul = prm->l2 ? 2 : 1;
  uint64_t *const lb = lbs + wave * QT;
  const int64_t tpp = prm->tiles_per_part;
  const int64_t tile_lo = prm->tile_lo, tile_hi = prm->tile_hi;
  const int items = nqt * parts;
  const int km1 = k - 1;

  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    int qt, part;
    item_coords(item, nqt, &qt, &part);
    const int q0 = qt * QT;
    const int nact = min(QT, nq - q0);
    const int64_t t0 = tile_lo + static_cast<int64_t>(part) * tpp;
    const int64_t t1 = min(tile_hi, t0 + tpp);

    WaveList<R> list[QT];
    uint64_t thr[QT];
#pragma unroll
    for (int qi = 0; qi < QT; ++qi) {
      list[qi].clear();
      thr[qi] = 0;
    }
    if (R >= 4 && lane < QT) lb[lane] = 0;

    // Cross-part bound (as in the matrix kernel, with each wave's share of a
    // part -- tiles t0 + wave + 4 i -- as its own sub-part): with S sub-parts
    // holding tiles and m = ceil(k / S), every sub-part publishes the m-th key
    // of its list to its own slot, and the smallest slot of a query (0 while
    // one is empty) is a lower bound on the query's k-th key overall; keys
    // not above it are dropped.
    auto refresh = [&]() {
      uint64_t *bound = prm->bound;
      const int peff = static_cast<int>(max<int64_t>(1, min<int64_t>(parts, (tile_hi - tile_lo + tpp - 1) / tpp)));
      const int nsub = peff * kBatchWaves;
      const int mth = (k + nsub - 1) / nsub;
#pragma unroll
      for (int qi = 0; qi < QT; ++qi) {
        if (qi < nact) {
          const uint64_t mk = list[qi].at(mth - 1);
          if (lane == 0 && mk)
            __hip_atomic_store(bound + (static_cast<int64_t>(q0 + qi) * parts + part) * kBatchWaves + wave, mk,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      // lane l reads slots l / QT, l / QT + 64 / QT, ... of query l % QT: the
      // loads of all queries are in flight together
      const int rq = lane % QT;
      uint64_t mn = 0;
      if (rq < nact)
        mn = min_published_keys(bound + static_cast<int64_t>(q0 + rq) * parts * kBatchWaves, lane / QT, nsub, 64 / QT);
#pragma unroll
      for (int off = QT; off < 64; off <<= 1) {
        const uint64_t o = __shfl_xor(static_cast<unsigned long long>(mn), off);
        mn = o < mn ? o : mn;
      }
#pragma unroll
      for (int qi = 0; qi < QT; ++qi) {
        const uint64_t b = readlane64(mn, qi);
        if (b > thr[qi]) thr[qi] = b;
      }
      if (lane < QT) lb[lane] = mn;
      __builtin_amdgcn_wave_barrier();
    };
    // (lists of 256 or 512 keys only: for smaller k the refreshes cost more
    // than the insertions they save)
    const bool prune = R >= 4 && prm->bound != nullptr;
    int next = 1, done = 0;

    for (int64_t t = t0 + wave; t < t1; t += kBatchWaves) {
      const uint4 *tp = tiles + t * (2 * NC * 64);
      u32x4 vz[NC], vg[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        vz[c] = load_stream(tp + c * 64 + lane);
        vg[c] = load_stream(tp + (NC + c) * 64 + lane);
      }
      const int64_t id = t * 64 + lane;
      const uint64_t okmask = __builtin_amdgcn_ballot_w64(id < n);
      const int32_t sub = mul == 2 ? vec_nnz<NC>(vz) : 0;
#pragma unroll
      for (int qi = 0; qi < QT; ++qi) {
        if (qi < nact) {
          const uint32_t *qw = qprep + static_cast<int64_t>(q0 + qi) * (8 * NC);
          // the query's words first (wide scalar loads, all in flight before
          // the chained sums), then one popcount-accumulate per count and word
          uint32_t qn[4 * NC], qg[4 * NC];
#pragma unroll
          for (int w = 0; w < 4 * NC; ++w) {
            qn[w] = qw[w];
            qg[w] = qw[4 * NC + w];
          }
          DeltaAcc a;
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            delta_word_chained(a, qn[4 * c + 0], qg[4 * c + 0], vz[c].x, vg[c].x);
            delta_word_chained(a, qn[4 * c + 1], qg[4 * c + 1], vz[c].y, vg[c].y);
            delta_word_chained(a, qn[4 * c + 2], qg[4 * c + 2], vz[c].z, vg[c].z);
            delta_word_chained(a, qn[4 * c + 3], qg[4 * c + 3], vz[c].w, vg[c].w);
          }
          const uint64_t key = make_key(delta_value(a) * mul - sub, static_cast<uint32_t>(id));
          offer_keys_masked<R>(list[qi], thr[qi], key, okmask, km1, prune ? lb[qi] : 0ull);
        }
      }
      if (prune && ++done >= next) {
        refresh();
        next = next < 64 ? 2 * next : next + 64;
      }
    }

    // merge the four wave lists of each active query of the tile
#pragma unroll
    for (int qi = 0; qi < QT; ++qi) {
      if (qi < nact) {
        uint64_t *a = lds[0];
        uint64_t *b = lds[1];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int p = r * 64 + lane;
          if (p < k) a[wave * k + p] = list[qi].v[r];
        }
        uint64_t *res = tree_merge(a, b, kBatchWaves, k);
        uint64_t *dst = partial + (static_cast<int64_t>(q0 + qi) * parts + part) * k;
        for (int p = threadIdx.x; p < k; p += kBatchBlock) dst[p] = res[p];
        __syncthreads();
      }
    }
  }
}

template <int NC, int R, int QT>
hipError_t launch3(const DbDev &db, const uint32_t *qprep, const BatchParams *prm, int k, int grid,
                   uint64_t *partial, hipStream_t s) {
  hipLaunchKernelGGL((scan_batched_kernel<NC, R, QT>), dim3(grid), dim3(kBatchBlock), 0, s, db.tiles, db.n,
                     db.ntiles, qprep, prm, k, partial);
  return hipGetLastError();
}

template <int NC, int R, int QMAX>
hipError_t launch2(const DbDev &db, const uint32_t *qprep, const BatchParams *prm, int k, int qtile, int grid,
                   uint64_t *partial, hipStream_t s) {
  if (qtile > QMAX) return hipErrorInvalidValue;
  switch (qtile) {
    case 2: return launch3<NC, R, 2>(db, qprep, prm, k, grid, partial, s);
    case 4: return launch3<NC, R, 4>(db, qprep, prm, k, grid, partial, s);
    case 8: return launch3<NC, R, (QMAX >= 8 ? 8 : 4)>(db, qprep, prm, k, grid, partial, s);
    case 16: return launch3<NC, R, (QMAX >= 16 ? 16 : 4)>(db, qprep, prm, k, grid, partial, s);
    default: return hipErrorInvalidValue;
  }
}

template <int NC>
hipError_t launch1(const DbDev &db, const uint32_t *qprep, const BatchParams *prm, int k, int qtile, int grid,
                   uint64_t *partial, hipStream_t s) {
  switch (rows_for_k(k)) {
    case 1: return launch2<NC, 1, 16>(db, qprep, prm, k, qtile, grid, partial, s);
    case 2: return launch2<NC, 2, 16>(db, qprep, prm, k, qtile, grid, partial, s);
    case 4: return launch2<NC, 4, 8>(db, qprep, prm, k, qtile, grid, partial, s);
    default: return launch2<NC, 8, 4>(db, qprep, prm, k, qtile, grid, partial, s);
  }
}

}  // namespace

int batched_max_qtile(int k) {
  const int r = rows_for_k(k);
  return r <= 2 ? 16 : r == 4 ? 8 : 4;
}

hipError_t batch_prep_launch(const uint32_t *qcodes, int nq, int bucket, const DbDev &db, int qtile, int grid,
                             int32_t *ids, int32_t *scores, uint32_t *qprep, BatchParams *prm, uint64_t *bound,
                             int l2, hipStream_t s) {
  const int64_t threads = static_cast<int64_t>(bucket) * 4 * db.nc;
  const unsigned blocks = static_cast<unsigned>((threads + 255) / 256);
  hipLaunchKernelGGL(batch_prep_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, qcodes, nq, bucket, db.W,
                     db.nc, qtile, grid, db.ntiles, ids, scores, qprep, prm, bound, l2);
  return hipGetLastError();
}

hipError_t prep_rows_launch(const uint32_t *qcodes, int nq, const DbDev &db, uint32_t *rows, hipStream_t s) {
  const int64_t threads = static_cast<int64_t>(nq) * 4 * db.nc;
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(prep_rows_kernel, dim3(static_cast<unsigned>((threads + 255) / 256)), dim3(256), 0, s, qcodes,
                     nq, nq, db.W, db.nc, rows);
  return hipGetLastError();
}

hipError_t gather_rows_launch(const uint32_t *src, const int *slots, int count, int words, uint32_t *rows,
                              hipStream_t s) {
  const int64_t threads = static_cast<int64_t>(count) * words;
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_rows_kernel, dim3(static_cast<unsigned>((threads + 255) / 256)), dim3(256), 0, s, src,
                     slots, count, words, rows);
  return hipGetLastError();
}

hipError_t fill_zero_launch(uint64_t *p, int64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

hipError_t running_results_launch(const uint64_t *running, const int *slots, int count, int k, int32_t *ids,
                                  int32_t *scores, hipStream_t s) {
  const int64_t threads = static_cast<int64_t>(count) * k;
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(running_results_kernel, dim3(static_cast<unsigned>((threads + 255) / 256)), dim3(256), 0, s,
                     running, slots, count, k, ids, scores);
  return hipGetLastError();
}

hipError_t scan_batched_launch(const DbDev &db, const uint32_t *qprep, const BatchParams *prm, int k, int qtile,
                               int grid, uint64_t *partial, hipStream_t s) {
  if (qtile > batched_max_qtile(k)) return hipErrorInvalidValue;
  switch (db.nc) {
    case 1: return launch1<1>(db, qprep, prm, k, qtile, grid, partial, s);
    case 2: return launch1<2>(db, qprep, prm, k, qtile, grid, partial, s);
    case 3: return launch1<3>(db, qprep, prm, k, qtile, grid, partial, s);
    case 4: return launch1<4>(db, qprep, prm, k, qtile, grid, partial, s);
    case 5: return launch1<5>(db, qprep, prm, k, qtile, grid, partial, s);
    case 6: return launch1<6>(db, qprep, prm, k, qtile, grid, partial, s);
    case 7: return launch1<7>(db, qprep, prm, k, qtile, grid, partial, s);
    case 8: return launch1<8>(db, qprep, prm, k, qtile, grid, partial, s);
    default: return hipErrorInvalidValue;
  }
}

bool mfma_supported(int k, int qtile) {
  return rows_for_k(k) <= 2 && (qtile == 64 || qtile == 128 || qtile == 256);
}

hipError_t scan_mfma_launch(const DbDev &db, const uint32_t *qprep, const BatchParams *prm, int k, int qtile,
                            int grid, int64_t max_part_tiles, uint64_t *partial, hipStream_t s,
                            const MfmaSample &sample) {
  if (!mfma_supported(k, qtile)) return hipErrorInvalidValue;
  switch (db.nc) {
    case 1: return scan_mfma_launch_nc<1>(db, qprep, prm, k, qtile, grid, max_part_tiles, partial, s, sample);
    case 2: return scan_mfma_launch_nc<2>(db, qprep, prm, k, qtile, grid, max_part_tiles, partial, s, sample);
    case 3: return scan_mfma_launch_nc<3>(db, qprep, prm, k, qtile, grid, max_part_tiles, partial, s, sample);
    case 4: return scan_mfma_launch_nc<4>(db, qprep, prm, k, qtile, grid, max_part_tiles, partial, s, sample);
    case 5: return scan_mfma_launch_nc<5>(db, qprep, prm, k, qtile, grid, max_part_tiles, partial, s, sample);
    case 6: return scan_mfma_launch_nc<6>(db, qprep, prm, k, qtile, grid, max_part_tiles, partial, s, sample);
    case 7: return scan_mfma_launch_nc<7>(db, qprep, prm, k, qtile, grid, max_part_tiles, partial, s, sample);
    case 8: return scan_mfma_launch_nc<8>(db, qprep, prm, k, qtile, grid, max_part_tiles, partial, s, sample);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tqi
