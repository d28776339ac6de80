// masked.hip -- the single-operand scan: a float query against the ternary
// database codes by masked addition (Sec. 5.1.2: the scalar product of a
// ternary v with any w is the sum of w where v+ is set minus the sum of w
// where v- is set; Sec. 6: comparing the ternary form with the original float
// space is the more accurate variant).
//
// With the resident planes nz = v+ | v- and ng = v-, the score is
//   sum_{nz} q_i - 2 sum_{ng} q_i.
// Each workgroup first tabulates the query in LDS: for every group of four
// coordinates g and every 4-bit mask m, lut[16 g + m] = the sum of the query
// over the set bits of m, in double (exact: four floats).  A lane then scores
// its tile vector with two table reads per nibble of its nz / ng words (all
// lanes read the same group at the same time, so the 16 entries they can hit
// are distinct), accumulating in double; the score is that sum rounded once
// to float.  Summed in double, the score differs from the sum in any other
// order by far less than a float rounding step, so results agree with a
// sequential reference except where a sum falls within ~1e-12 of a float
// rounding boundary.  The rest is the plain scan's: tiles of 64 vectors
// spread over the grid, a register top-k list per wave, an LDS merge per
// workgroup, and the per-query merge.  Keys order floats exactly: the score's
// bit pattern is mapped to an unsigned value with the same order (zeros of
// both signs map to one value) and takes the place of Delta + 2^31 in the
// 64-bit key.  Each chunk's registers take the same chunk of the wave's next
// tile once scored, so loads overlap the table reads at no register cost.
#include "tq_batched.h"
#include "tq_device.h"

namespace tqi {
namespace {

constexpr int kMaskedWaves = 4;
constexpr int kMaskedBlock = 64 * kMaskedWaves;

// float -> int32 whose (value + 2^31) is the order-preserving key word
__device__ __forceinline__ int32_t float_rank(float f) {
  const uint32_t u = __float_as_uint(f + 0.0f);  // -0 + +0 = +0
  const uint32_t k = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
  return static_cast<int32_t>(k - kScoreBias);
}

// With tstride > 1 the scan covers tiles 0, tstride, 2 tstride, ... (a
// sample); with floor_ids (the sample's merged result row of this query: k
// ids, then its k scores in floor_scores) keys below the sample's k-th key,
// which is never above the k-th key of the whole database, are dropped.
template <int NC, int R>
__global__ __launch_bounds__(kMaskedBlock) void scan_masked_kernel(const uint4 *__restrict__ tiles, int64_t n,
                                                                  int64_t ntiles, int d, const float *__restrict__ q,
                                                                  int k, uint64_t *__restrict__ partial, int tstride,
                                                                  const int32_t *__restrict__ floor_ids,
                                                                  const int32_t *__restrict__ floor_scores) {
  constexpr int kGroups = 32 * NC;  // 4 NC words per plane, 8 nibbles per word
  __shared__ double lut[kGroups * 16];
  __shared__ uint64_t lds[2][kMaskedWaves * 64 * R];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * kMaskedWaves;

  for (int e = threadIdx.x; e < kGroups * 16; e += kMaskedBlock) {
    const int g = e >> 4, m = e & 15;
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = 4 * g + b;
      if ((m >> b) & 1) s += i < d ? static_cast<double>(q[i]) : 0.0;
    }
    lut[e] = s;
  }
  __syncthreads();

  WaveList<R> list;
  list.clear();
  uint64_t floor = 0;  // keys below the sample's k-th key are outside the result
  if (floor_ids && floor_ids[k - 1] >= 0)
    floor = make_key(floor_scores[k - 1], static_cast<uint32_t>(floor_ids[k - 1])) - 1;
  uint64_t thr = floor;
  const int km1 = k - 1;
  const int64_t nscan = (ntiles + tstride - 1) / tstride;  // tiles of this scan: t * tstride
  const int64_t tile_words = static_cast<int64_t>(tstride) * (2 * NC * 64);

  // A chunk's registers take the same chunk of the wave's next tile as soon
  // as it has been scored, so the next tile's loads overlap this tile's table
  // reads without a second set of registers (the last tile re-reads itself).
  const int64_t t_first = static_cast<int64_t>(blockIdx.x) * kMaskedWaves + wave;
  u32x4 vz[NC], vg[NC];
  if (t_first < nscan) {
    const uint4 *tile = tiles + t_first * tile_words;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      vz[c] = load_stream(tile + c * 64 + lane);
      vg[c] = load_stream(tile + (NC + c) * 64 + lane);
    }
  }
  for (int64_t t = t_first; t < nscan; t += nwaves) {
    const uint4 *next = tiles + (t + nwaves < nscan ? t + nwaves : t) * tile_words;
    double sp[2] = {0.0, 0.0}, sm[2] = {0.0, 0.0};
#pragma unroll
    for (int c = 0; c < NC; ++c) {
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const uint32_t z = vz[c][w], g = vg[c][w];
        // Even nibbles in the low halves of the four bytes, odd nibbles
        // likewise: each table offset is then one byte of these words
        // shifted by 3, a single instruction with a byte-select operand.
        // The empty asm keeps the compiler from folding the masks back
        // into a shift and a mask per nibble.
        uint32_t z0 = z & 0x0F0F0F0Fu, z1 = (z >> 4) & 0x0F0F0F0Fu;
        uint32_t g0 = g & 0x0F0F0F0Fu, g1 = (g >> 4) & 0x0F0F0F0Fu;
        asm volatile("" : "+v"(z0), "+v"(z1), "+v"(g0), "+v"(g1));
        const double *row = lut + (4 * c + w) * 8 * 16;
        // all sixteen reads of the word are issued before the first add
        double e[16];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          e[4 * b + 0] = row[(2 * b) * 16 + ((z0 >> (8 * b)) & 0xFF)];
          e[4 * b + 1] = row[(2 * b) * 16 + ((g0 >> (8 * b)) & 0xFF)];
          e[4 * b + 2] = row[(2 * b + 1) * 16 + ((z1 >> (8 * b)) & 0xFF)];
          e[4 * b + 3] = row[(2 * b + 1) * 16 + ((g1 >> (8 * b)) & 0xFF)];
        }
        // nibble order within each accumulator: even nibbles into [0], odd into [1]
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          sp[0] += e[4 * b + 0];
          sm[0] += e[4 * b + 1];
          sp[1] += e[4 * b + 2];
          sm[1] += e[4 * b + 3];
        }
      }
      vz[c] = load_stream(next + c * 64 + lane);
      vg[c] = load_stream(next + (NC + c) * 64 + lane);
    }
    const float score = static_cast<float>((sp[0] + sp[1]) - 2.0 * (sm[0] + sm[1]));
    const int64_t id = t * tstride * 64 + lane;
    const uint64_t key = make_key(float_rank(score), static_cast<uint32_t>(id));
    offer_keys<R>(list, thr, key, id < n, km1, floor);
  }

  uint64_t *a = lds[0];
  uint64_t *b = lds[1];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int p = r * 64 + lane;
    if (p < k) a[wave * k + p] = list.v[r];
  }
  uint64_t *res = tree_merge(a, b, kMaskedWaves, k);
  for (int p = threadIdx.x; p < k; p += kMaskedBlock) partial[static_cast<int64_t>(blockIdx.x) * k + p] = res[p];
}

// The merge writes key_score(key) = key word - 2^31 into the int32 scores;
// turn those back into the floats they encode, in place.
__global__ void rank_to_float_kernel(int32_t *__restrict__ scores, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint32_t k = static_cast<uint32_t>(scores[i]) + kScoreBias;
  const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  scores[i] = static_cast<int32_t>(u);
}

template <int NC, int R>
hipError_t launch_m(const DbDev &db, const float *q, int k, int grid, uint64_t *partial, hipStream_t s,
                    const MaskedScanOpts &o) {
  hipLaunchKernelGGL((scan_masked_kernel<NC, R>), dim3(grid), dim3(kMaskedBlock), 0, s, db.tiles, db.n, db.ntiles,
                     db.d, q, k, partial, o.tstride, o.floor_ids, o.floor_scores);
  return hipGetLastError();
}

template <int NC>
hipError_t launch_mr(const DbDev &db, const float *q, int k, int grid, uint64_t *partial, hipStream_t s,
                     const MaskedScanOpts &o) {
  switch (rows_for_k(k)) {
    case 1: return launch_m<NC, 1>(db, q, k, grid, partial, s, o);
    case 2: return launch_m<NC, 2>(db, q, k, grid, partial, s, o);
    case 4: return launch_m<NC, 4>(db, q, k, grid, partial, s, o);
    default: return launch_m<NC, 8>(db, q, k, grid, partial, s, o);
  }
}

template <int NC, int R>
int resident_m() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, scan_masked_kernel<NC, R>, kMaskedBlock, 0) != hipSuccess)
    return 0;
  return n;
}

template <int NC>
int resident_mr(int k) {
  switch (rows_for_k(k)) {
    case 1: return resident_m<NC, 1>();
    case 2: return resident_m<NC, 2>();
    case 4: return resident_m<NC, 4>();
    default: return resident_m<NC, 8>();
  }
}

}  // namespace

hipError_t scan_masked_launch(const DbDev &db, const float *q, int k, int grid, uint64_t *partial, hipStream_t s,
                              const MaskedScanOpts &o) {
  if (o.tstride < 1) return hipErrorInvalidValue;
  switch (db.nc) {
    case 1: return launch_mr<1>(db, q, k, grid, partial, s, o);
    case 2: return launch_mr<2>(db, q, k, grid, partial, s, o);
    case 3: return launch_mr<3>(db, q, k, grid, partial, s, o);
    case 4: return launch_mr<4>(db, q, k, grid, partial, s, o);
    case 5: return launch_mr<5>(db, q, k, grid, partial, s, o);
    case 6: return launch_mr<6>(db, q, k, grid, partial, s, o);
    case 7: return launch_mr<7>(db, q, k, grid, partial, s, o);
    case 8: return launch_mr<8>(db, q, k, grid, partial, s, o);
    default: return hipErrorInvalidValue;
  }
}

int scan_masked_resident(int nc, int k) {
  switch (nc) {
    case 1: return resident_mr<1>(k);
    case 2: return resident_mr<2>(k);
    case 3: return resident_mr<3>(k);
    case 4: return resident_mr<4>(k);
    case 5: return resident_mr<5>(k);
    case 6: return resident_mr<6>(k);
    case 7: return resident_mr<7>(k);
    case 8: return resident_mr<8>(k);
    default: return 0;
  }
}

hipError_t rank_to_float_launch(int32_t *scores, int64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(rank_to_float_kernel, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, s, scores,
                     count);
  return hipGetLastError();
}

}  // namespace tqi
