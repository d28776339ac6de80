// sparse.hip -- the index-list copy of a database with few non-zeros, and
// its single-query scan.
//
// A code with x non-zeros is equally well described by the list of its x
// non-zero coordinates with their signs.  When x is small against d that list
// is shorter than the two bit planes (2x bytes against d/4), and Delta -- the
// scalar product of the two ternary vectors (Sec. 5.1.2) -- becomes a gather:
// the sum, over the database vector's list, of the query's value at each
// listed coordinate, negated where the database sign is negative.  The paper
// leaves faster search at small x open (Sec. 6); this is the bandwidth side of
// it: the scan still streams every vector once, but reads 2x bytes per vector
// instead of d/4.
//
// Entry of one non-zero coordinate i: uint16 (i << 1) | [v_i = -1], listed by
// increasing i and padded with the neutral entry (d << 1) to a multiple of 8.
// Tiles mirror the bit-plane layout: 64 vectors per tile, and chunk c (8
// entries, 16 bytes) of all 64 vectors is one contiguous 1 KiB run, uint4
// index (tile * sc + c) * 64 + lane.  Vectors past n hold only padding.
//
// The query becomes a table of 2 d + 2 signed bytes in LDS, tab[(i << 1) | s]
// = (s ? -q_i : q_i), with tab[2 d] = tab[2 d + 1] = 0, so an entry is its own
// table address and a vector's Delta is x table reads and adds.
#include "tq_batched.h"
#include "tq_device.h"

namespace tqi {
namespace {

constexpr int kSparseWaves = 4;
constexpr int kSparseBlock = 64 * kSparseWaves;
constexpr int kTabBytes = 2 * (kMaxNc * 128) + 16;  // 2 d + 2 for d <= 1024, rounded up

// One thread per vector slot: its non-zeros, read from the nz / ng bit planes
// of the resident tiles (coalesced per chunk), become sc chunks of entries.
__global__ __launch_bounds__(256) void sparse_repack_kernel(const uint4 *__restrict__ tiles, int64_t ntiles, int nc,
                                                            int d, int sc, uint4 *__restrict__ out) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= ntiles * 64) return;
  const int64_t t = g >> 6;
  const int lane = static_cast<int>(g & 63);
  const uint32_t pad = static_cast<uint32_t>(d) << 1;
  uint32_t acc[4];
  int cnt = 0, c = 0;
  auto flush = [&]() {
    // entries cnt .. 7 of the chunk are padding
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j >= cnt) acc[j >> 1] |= pad << (16 * (j & 1));
    if (c < sc) out[(t * sc + c) * 64 + lane] = make_uint4(acc[0], acc[1], acc[2], acc[3]);
    ++c;
    cnt = 0;
  };
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = 0;
  for (int ch = 0; ch < nc; ++ch) {
    const uint4 z = tiles[((t * 2 + 0) * nc + ch) * 64 + lane];
    const uint4 n = tiles[((t * 2 + 1) * nc + ch) * 64 + lane];
    const uint32_t zw[4] = {z.x, z.y, z.z, z.w};
    const uint32_t nw[4] = {n.x, n.y, n.z, n.w};
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      uint32_t m = zw[w];
      while (m) {
        const int b = __builtin_ctz(m);
        m &= m - 1;
        const uint32_t i = static_cast<uint32_t>((ch * 4 + w) * 32 + b);
        const uint32_t e = (i << 1) | ((nw[w] >> b) & 1u);
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j == cnt) acc[j >> 1] |= e << (16 * (j & 1));
        if (++cnt == 8) {
          flush();
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[j] = 0;
        }
      }
    }
  }
  while (c < sc) {
    flush();
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = 0;
  }
}

// Sum of the table values addressed by the 8 entries of one chunk.
__device__ __forceinline__ int32_t chunk_sum(const int8_t *tab, const u32x4 &e) {
  return static_cast<int32_t>(tab[e.x & 0xFFFFu]) + static_cast<int32_t>(tab[e.x >> 16]) +
         static_cast<int32_t>(tab[e.y & 0xFFFFu]) + static_cast<int32_t>(tab[e.y >> 16]) +
         static_cast<int32_t>(tab[e.z & 0xFFFFu]) + static_cast<int32_t>(tab[e.z >> 16]) +
         static_cast<int32_t>(tab[e.w & 0xFFFFu]) + static_cast<int32_t>(tab[e.w >> 16]);
}

// Tiles are dealt to the waves of the grid as in the bit-plane scan (wave w
// takes tiles w, w + #waves, ...); each wave has its next tile's loads in
// flight while it scores the current one (past the end it re-reads the last
// tile, so the loads need no branch).
template <int SC, int R>
__global__ __launch_bounds__(kSparseBlock) void scan_sparse_kernel(const uint4 *__restrict__ sp, int64_t n,
                                                                   int64_t ntiles, int d, int W,
                                                                   const uint32_t *__restrict__ qcode, int k,
                                                                   uint64_t *__restrict__ partial) {
  __shared__ int8_t tab[kTabBytes];
  __shared__ uint64_t lds[2][kSparseWaves * 64 * R];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * kSparseWaves;

  for (int i = threadIdx.x; i <= d; i += kSparseBlock) {
    int v = 0;
    if (i < d) {
      const uint32_t bit = 1u << (i & 31);
      v = ((qcode[i >> 5] & bit) ? 1 : 0) - ((qcode[W + (i >> 5)] & bit) ? 1 : 0);
    }
    tab[2 * i] = static_cast<int8_t>(v);
    tab[2 * i + 1] = static_cast<int8_t>(-v);
  }
  __syncthreads();

  WaveList<R> list;
  list.clear();
  uint64_t thr = 0;
  const int km1 = k - 1;

  int64_t t = static_cast<int64_t>(blockIdx.x) * kSparseWaves + wave;
  if (t < ntiles) {
    u32x4 cur[SC];
#pragma unroll
    for (int c = 0; c < SC; ++c) cur[c] = load_stream(sp + (t * SC + c) * 64 + lane);
    for (; t < ntiles; t += nwaves) {
      const int64_t tn = min(t + nwaves, ntiles - 1);
      u32x4 nxt[SC];
#pragma unroll
      for (int c = 0; c < SC; ++c) nxt[c] = load_stream(sp + (tn * SC + c) * 64 + lane);
      int32_t delta = 0;
#pragma unroll
      for (int c = 0; c < SC; ++c) delta += chunk_sum(tab, cur[c]);
      const int64_t id = t * 64 + lane;
      offer_keys<R>(list, thr, make_key(delta, static_cast<uint32_t>(id)), id < n, km1);
#pragma unroll
      for (int c = 0; c < SC; ++c) cur[c] = nxt[c];
    }
  }

  uint64_t *a = lds[0];
  uint64_t *b = lds[1];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = r * 64 + lane;
    if (p < k) a[wave * k + p] = list.v[r];
  }
  uint64_t *res = tree_merge(a, b, kSparseWaves, k);
  for (int p = threadIdx.x; p < k; p += kSparseBlock) partial[static_cast<int64_t>(blockIdx.x) * k + p] = res[p];
}

template <int SC, int R>
hipError_t launch_sr(const DbDev &db, const uint32_t *qcode, int k, int grid, uint64_t *partial, hipStream_t s) {
  hipLaunchKernelGGL((scan_sparse_kernel<SC, R>), dim3(grid), dim3(kSparseBlock), 0, s, db.sparse, db.n, db.ntiles,
                     db.d, db.W, qcode, k, partial);
  return hipGetLastError();
}

template <int SC>
hipError_t launch_s(const DbDev &db, const uint32_t *qcode, int k, int grid, uint64_t *partial, hipStream_t s) {
  switch (rows_for_k(k)) {
    case 1: return launch_sr<SC, 1>(db, qcode, k, grid, partial, s);
    case 2: return launch_sr<SC, 2>(db, qcode, k, grid, partial, s);
    case 4: return launch_sr<SC, 4>(db, qcode, k, grid, partial, s);
    default: return launch_sr<SC, 8>(db, qcode, k, grid, partial, s);
  }
}

}  // namespace

int sparse_chunks(int d, int x) {
  if (x < 1 || d < 1 || d > kMaxNc * 128 || 8 * x > d) return 0;
  return (x + 7) / 8;
}

hipError_t sparse_repack_launch(const DbDev &db, uint4 *out, int sc, hipStream_t s) {
  if (sc < 1 || sc > kMaxSparseChunks) return hipErrorInvalidValue;
  const int64_t threads = db.ntiles * 64;
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(sparse_repack_kernel, dim3(static_cast<unsigned>((threads + 255) / 256)), dim3(256), 0, s,
                     db.tiles, db.ntiles, db.nc, db.d, sc, out);
  return hipGetLastError();
}

hipError_t scan_sparse_launch(const DbDev &db, const uint32_t *qcode, int k, int grid, uint64_t *partial,
                              hipStream_t s) {
  if (!db.sparse || db.d > kMaxNc * 128) return hipErrorInvalidValue;
  switch (db.sc) {
    case 1: return launch_s<1>(db, qcode, k, grid, partial, s);
    case 2: return launch_s<2>(db, qcode, k, grid, partial, s);
    case 3: return launch_s<3>(db, qcode, k, grid, partial, s);
    case 4: return launch_s<4>(db, qcode, k, grid, partial, s);
    case 5: return launch_s<5>(db, qcode, k, grid, partial, s);
    case 6: return launch_s<6>(db, qcode, k, grid, partial, s);
    case 7: return launch_s<7>(db, qcode, k, grid, partial, s);
    case 8: return launch_s<8>(db, qcode, k, grid, partial, s);
    case 9: return launch_s<9>(db, qcode, k, grid, partial, s);
    case 10: return launch_s<10>(db, qcode, k, grid, partial, s);
    case 11: return launch_s<11>(db, qcode, k, grid, partial, s);
    case 12: return launch_s<12>(db, qcode, k, grid, partial, s);
    case 13: return launch_s<13>(db, qcode, k, grid, partial, s);
    case 14: return launch_s<14>(db, qcode, k, grid, partial, s);
    case 15: return launch_s<15>(db, qcode, k, grid, partial, s);
    case 16: return launch_s<16>(db, qcode, k, grid, partial, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tqi
