// mfma_kernels.hip -- the batched scan on the matrix cores.
//
// When one database pass serves many queries, Delta for all (query, vector)
// pairs is exactly the product of two ternary matrices (the scalar products
// of Sec. 5.1.2).  {-1, 0, +1} are exact fp4 (e2m1) values and every partial
// sum (at most d <= 1024 in magnitude) is exact in fp32, so the gfx950 fp4
// MFMA V_MFMA_SCALE_F32_16X16X128_F8F6F4 (scales 2^0) gives the same integers
// as the popcount form, at several times its rate.
//
// Operand re-coding.  A product over k is unchanged by any permutation of k
// applied to both operands, so one 32-coordinate word of the nz / ng planes
// becomes 32 fp4 operand values without spreading bits: dimension 4j + q of
// the word becomes nibble j of dword q, with nibble value 0b0010 (+1.0) where
// nz is set and 0b1010 (-1.0) where ng is set too, i.e.
//   dword q = ((nz >> (q-1)) & 0x22222222) | ((ng << (3-q)) & 0x88888888).
// Queries (operand A, 16 rows) and database vectors (operand B, 16 columns)
// use the same re-coding; lane l supplies row / column l % 16 and the word
// 4s + l / 16 of K-step s (128 coordinates, one 16-byte chunk of a plane).
//
// Work: a persistent grid walks (query tile, database part) items like the
// popcount kernel, but here each of a workgroup's WV waves (four or eight)
// owns 16*RB queries of the tile (16*RB*WV per tile) and all of them sweep
// the same database tiles.
// Each 64-vector tile is read from HBM once per workgroup, re-coded to fp4
// operands by the whole workgroup while it is staged into LDS (double
// buffered: the next tile's loads are in flight while the current one is
// multiplied), and read by every wave from LDS.  A wave accumulates a
// 16*RB x 64 block of Delta in fp32, compares each value with its row's
// current k-th score (a float kept per lane), and only on the rare candidates
// builds exact keys and inserts them, in id order, into its register top-k
// list for that query.  A query belongs to one wave, so a wave's list is the
// (query, part) result and no merge inside the workgroup is needed.
#include <type_traits>

#include "tq_batched.h"
#include "tq_device.h"

namespace tqi {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kMfmaWaves = 4;  // waves per workgroup unless a tile says otherwise
constexpr int kScaleOne = 0x7f7f7f7f;  // e8m0 exponent 127 in every byte: scale 2^0

// 32 coordinates (one word of each plane) -> 32 fp4 operand values (16 bytes).
__device__ __forceinline__ v4i fp4_operand(uint32_t nz, uint32_t ng) {
  const uint32_t d0 = ((nz << 1) & 0x22222222u) | ((ng << 3) & 0x88888888u);
  const uint32_t d1 = (nz & 0x22222222u) | ((ng << 2) & 0x88888888u);
  const uint32_t d2 = ((nz >> 1) & 0x22222222u) | ((ng << 1) & 0x88888888u);
  const uint32_t d3 = ((nz >> 2) & 0x22222222u) | (ng & 0x88888888u);
  v4i r = {static_cast<int>(d0), static_cast<int>(d1), static_cast<int>(d2), static_cast<int>(d3)};
  return r;
}

// fp4 operands use the low four dwords of the instruction's eight.
__device__ __forceinline__ v4f mfma_fp4(const v4i &a, const v4i &b, const v4f &c) {
  const v8i a8 = {a.x, a.y, a.z, a.w, 0, 0, 0, 0};
  const v8i b8 = {b.x, b.y, b.z, b.w, 0, 0, 0, 0};
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a8, b8, c, 4, 4, 0, kScaleOne, 0, kScaleOne);
}

__device__ __forceinline__ float score_of(uint64_t thr) {
  // the k-th key's score as a float; an empty slot lets everything through
  return thr ? static_cast<float>(key_score(thr)) : -1e30f;
}

// Prefilter threshold of a row from its list's k-th key `own` and the bound
// `lb` published by the other parts.  Keys of this part arrive in increasing
// id order, so beating `own` takes a larger score; `lb` may come from a part
// of higher ids, where an equal score with a lower id is a larger key.
// A bound with the largest id field of its score (the sample floor's form)
// cannot be beaten by an equal score, so there the prefilter admits larger
// scores only.
__device__ __forceinline__ float row_threshold(uint64_t own, uint64_t lb) {
  if (lb <= own) return score_of(own);
  return static_cast<float>(key_score(lb)) - (static_cast<uint32_t>(lb) == 0xFFFFFFFFu ? 0.f : 0.5f);
}

// The wave list of tq_device.h with 32-bit keys (one register per 64
// positions, one lane move per register and insertion).
template <int R>
struct WaveList32 {
  uint32_t v[R];

  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = 0;
  }

  __device__ __forceinline__ uint32_t at(int p) const {
    uint32_t res = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r == (p >> 6)) res = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v[r]), p & 63));
    return res;
  }

  __device__ __forceinline__ void insert(uint32_t key) {
    uint32_t prev[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t carry =
          (r == 0) ? ~0u : static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v[r - 1]), 63));
      prev[r] = __builtin_amdgcn_update_dpp(carry, v[r], kDppWaveShr1, 0xf, 0xf, false);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = (v[r] > key) ? v[r] : ((prev[r] > key) ? key : prev[r]);
  }
};

// Part-relative 32-bit keys for the k > 16 scan.  Within one database part
// of at most 2^20 vectors starting at id `base`, the key
//   ((score + kK32Bias) << 20) | (2^20 - 1 - (id - base))
// orders (score, id) pairs exactly like the 64-bit key (score descending, then
// id ascending): |score| <= d <= 1024, so score + kK32Bias lies in [1, 2049]
// (12 bits) and every real key is non-zero, like the 64-bit form.
constexpr int32_t kK32Bias = 1025;
constexpr uint32_t kLidMask = (1u << 20) - 1;

__device__ __forceinline__ int32_t score32(uint32_t key) { return static_cast<int32_t>(key >> 20) - kK32Bias; }

__device__ __forceinline__ float row_threshold(uint32_t own, uint32_t lb) {
  if (lb <= own) return own ? static_cast<float>(score32(own)) : -1e30f;
  return static_cast<float>(score32(lb)) - ((lb & kLidMask) == kLidMask ? 0.f : 0.5f);
}

// A 64-bit key from anywhere in the database as the threshold it sets on this
// part's 32-bit keys: local > to_local(T) exactly when the 64-bit key of the
// same (score, id) is > T.  0 stays 0 (no bound).
__device__ __forceinline__ uint32_t to_local(uint64_t t, int64_t base) {
  if (!t) return 0;
  const uint32_t hi = static_cast<uint32_t>(key_score(t) + kK32Bias) << 20;
  const int64_t id = static_cast<int64_t>(~static_cast<uint32_t>(t));
  if (id < base) return hi | kLidMask;       // equal scores here have larger ids
  if (id - base > kLidMask) return hi - 1u;  // equal scores here have smaller ids
  return hi | (kLidMask - static_cast<uint32_t>(id - base));
}

__device__ __forceinline__ uint64_t to_global(uint32_t key, int64_t base) {
  return key ? make_key(score32(key), static_cast<uint32_t>(base + (kLidMask - (key & kLidMask)))) : 0;
}

__device__ __forceinline__ uint32_t readlane_key(uint32_t v, int l) {
  return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), l));
}
__device__ __forceinline__ uint64_t readlane_key(uint64_t v, int l) { return readlane64(v, l); }

// Relaxed stores at device scope: the published keys are read by workgroups
// on other XCDs, around the non-coherent L2s (min_published_keys).
__device__ __forceinline__ void store_shared_key(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Staging of one 64-vector tile.  Thread j reads 16-byte chunks s = j / 64,
// j / 64 + 4 (< NC) of both planes of vector v = j % 64 -- a wave reads one
// contiguous 1 KiB run per load -- and re-codes word w of chunk s into the
// operand that lane 16 w + v % 16 of every wave takes for column block v / 16
// at K-step s.  The loads are ordinary (cached) loads: the workgroups that
// scan the same database part for other query tiles run at the same time on
// the same XCD and find the tile in its L2.
template <int NC, int WV = kMfmaWaves>
struct TileStage {
  static constexpr int kPer = (NC + WV - 1) / WV;
  uint4 nz[kPer], ng[kPer];

  // Every thread issues the same loads (a chunk past NC re-reads chunk
  // NC - 1 and is not stored), so no branch separates the loads of one tile
  // from the next and two tiles can stay in flight.
  __device__ __forceinline__ void load(const uint4 *__restrict__ tiles, int64_t t, int j) {
    const int v = j & 63, s0 = j >> 6;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int s = min(s0 + WV * i, NC - 1);
      nz[i] = tiles[((t * 2 + 0) * NC + s) * 64 + v];
      ng[i] = tiles[((t * 2 + 1) * NC + s) * 64 + v];
    }
  }
  // operand (s, cb) of lane l lives at op[(s * 4 + cb) * 64 + l]
  __device__ __forceinline__ void store(v4i *op, int j) const {
    const int v = j & 63, s0 = j >> 6;
    v4i *dst = op + (v >> 4) * 64 + (v & 15);
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int s = s0 + WV * i;
      if (s < NC) {
        dst[s * 256 + 0] = fp4_operand(nz[i].x, ng[i].x);
        dst[s * 256 + 16] = fp4_operand(nz[i].y, ng[i].y);
        dst[s * 256 + 32] = fp4_operand(nz[i].z, ng[i].z);
        dst[s * 256 + 48] = fp4_operand(nz[i].w, ng[i].w);
      }
    }
  }
};

// Two workgroups per CU (their LDS fits) wherever the registers allow it;
// RB = 2 (256-query tiles, eight waves of 32 queries) keeps two waves per SIMD.
// K32: keys relative to the part's first id (every part spans at most 2^20
// vectors), half the list registers and lane moves of the 64-bit form.
template <int NC, int R, int RB, int WV, bool K32>
__global__ __launch_bounds__(64 * WV, RB == 2 ? 2 : ((K32 ? R : 2 * R) * RB * WV <= 16 ? 8 / WV : 1)) void scan_mfma_kernel(
    const uint4 *__restrict__ tiles, int64_t n, const uint32_t *__restrict__ qprep,
    const BatchParams *__restrict__ prm, int k, uint64_t *__restrict__ partial, const uint64_t *__restrict__ floor) {
  using Key = typename std::conditional<K32, uint32_t, uint64_t>::type;
  using List = typename std::conditional<K32, WaveList32<R>, WaveList<R>>::type;
  constexpr int QW = 16 * RB;            // queries per wave
  constexpr int QT = WV * QW;            // queries per workgroup tile
  __shared__ v4i op[2][NC * 4 * 64];     // two staged tiles of fp4 operands
  __shared__ Key lbs[WV * QW];           // each query's bound from the other parts
  const int j = threadIdx.x;
  const int lane = j & 63;
  const int wave = j >> 6;
  const int col = lane & 15;  // operand row / column of this lane
  const int grp = lane >> 4;  // k-block of this lane; also its output row group
  Key *const lb = lbs + wave * QW;
  const int nq = prm->nq, nqt = prm->nqt, parts = prm->parts;
  const int64_t tpp = prm->tiles_per_part;
  const int64_t tile_lo = prm->tile_lo, tile_hi = prm->tile_hi;
  const int items = nqt * parts;
  const int km1 = k - 1;
  // Cross-part pruning.  With P parts holding tiles and m = ceil(k / P), if
  // every part's list holds m keys >= T then the union holds P m >= k keys
  // >= T, so the query's k-th key overall is >= T, and keys below T can be
  // dropped by every part without changing the result.  A part's m-th key
  // only grows, so any value it has published is such a T for that part, and
  // the smallest published value over the P parts (0 while one has not
  // published) is a bound for the query.
  // (RB = 2 has no registers to spare for it and relies on the floor.)
  // Behind a sample floor the exchange pays only with few parts (at most k):
  // there the bound from m = ceil(k / P) keys per part outranks the floor,
  // while with many parts each exchange reads many slots for a bound near
  // the floor (on the large workload, 16 queries at k = 100 on 512 parts:
  // 0.80 ms with the exchange, 0.70 ms without; 1 024 queries on 32 parts:
  // 8.7 ms with it, 10.1 ms without).
  constexpr bool kPrune = RB == 1;
  constexpr int kLanesPerQuery = 64 / QW;  // lanes that read one query's bounds
  const bool prune = kPrune && prm->bound != nullptr && (floor == nullptr || prm->parts <= k);

  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    int qt, part;
    item_coords(item, nqt, &qt, &part);
    const int q0 = qt * QT + wave * QW;  // this wave's first query
    const int nact = max(0, min(QW, nq - q0));
    const int64_t t0 = tile_lo + static_cast<int64_t>(part) * tpp;
    const int64_t t1 = min(tile_hi, t0 + tpp);
    const int64_t base = t0 * 64;  // first id of the part
    // (score, id) -> this form's key; this form's key -> the 64-bit key
    auto make = [&](int32_t score, int64_t id) -> Key {
      if constexpr (K32)
        return (static_cast<uint32_t>(score + kK32Bias) << 20) | (kLidMask - static_cast<uint32_t>(id - base));
      else
        return make_key(score, static_cast<uint32_t>(id));
    };
    auto global = [&](Key key) -> uint64_t {
      if constexpr (K32) return to_global(key, base);
      else return key;
    };

    // operand A: this wave's queries, re-coded once per item
    v4i a[RB][NC];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int qi = rb * 16 + col;
      const uint32_t *qw = qprep + static_cast<int64_t>(q0 + qi) * (8 * NC);
#pragma unroll
      for (int s = 0; s < NC; ++s) {
        uint32_t nz = 0, ng = 0;
        if (qi < nact) {
          nz = qw[4 * s + grp];
          ng = qw[4 * NC + 4 * s + grp];
        }
        a[rb][s] = fp4_operand(nz, ng);
      }
    }
    List list[QW];
#pragma unroll
    for (int qi = 0; qi < QW; ++qi) list[qi].clear();
    // the sample floor (a key no final key of the query is below) starts
    // each query's bound
    auto floor_of = [&](int qi) -> uint64_t { return floor && qi < nact ? floor[q0 + qi] : 0; };
    auto local = [&](uint64_t t) -> Key {
      if constexpr (K32) return to_local(t, base);
      else return t;
    };
    if (lane < QW) lb[lane] = local(floor_of(lane));
    // tv[rb][i]: k-th score of this lane's output row 16 rb + 4 grp + i;
    // rows past the real queries never pass
    float tv[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i) tv[rb][i] = (rb * 16 + 4 * grp + i < nact) ? -1e30f : 1e30f;

    // Pipeline: while tile t is multiplied out of LDS, tile t + 1 (loaded
    // during the previous tile) is re-coded into the other LDS buffer and
    // tile t + 2 is in flight to registers.  Loads past the part re-read its
    // last tile, so every thread issues the same loads on every step.
    TileStage<NC, WV> sa, sb;
    auto step = [&](int64_t t, const v4i *cur, v4i *nxt, TileStage<NC, WV> &fill, const TileStage<NC, WV> &ready) {
      fill.load(tiles, min(t + 2, t1 - 1), j);
      if (nact > 0) {
        v4f acc[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < NC; ++s) {
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) {
            const v4i b = cur[(s * 4 + cb) * 64 + lane];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[rb][cb] = mfma_fp4(a[rb][s], b, acc[rb][cb]);
          }
        }
        // rows with a value above their k-th score (rare once lists are full)
        uint64_t rows[RB][4];
        bool any = false;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            bool c = false;
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) c |= acc[rb][cb][i] > tv[rb][i];
            rows[rb][i] = __ballot(c);
            any |= rows[rb][i] != 0;
          }
        if (any) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              if (!rows[rb][i]) continue;
#pragma unroll
              for (int g = 0; g < 4; ++g) {
                // lanes of group g carry row 16 rb + 4 g + i
                const int qi = rb * 16 + 4 * g + i;
                if (!(rows[rb][i] & (0xFFFFull << (16 * g))) || qi >= nact) continue;
                const Key lbq = lb[qi];
                Key own = list[qi].at(km1);
                Key thr = own > lbq ? own : lbq;
#pragma unroll
                for (int cb = 0; cb < 4; ++cb) {  // increasing ids
                  const int64_t id = t * 64 + cb * 16 + col;
                  const float v = acc[rb][cb][i];
                  const Key key = make(static_cast<int32_t>(v), id);
                  uint64_t m = __ballot(grp == g && id < n && key > thr);
                  while (m) {
                    const int src = __builtin_ctzll(m);
                    m &= m - 1;
                    const Key c = readlane_key(key, src);
                    if (c > thr) {
                      list[qi].insert(c);
                      own = list[qi].at(km1);
                      thr = own > lbq ? own : lbq;
                    }
                  }
                }
                if (grp == g) tv[rb][i] = row_threshold(own, lbq);
              }
            }
          }
        }
      }
      ready.store(nxt, j);
      __syncthreads();
    };
    // Publish this wave's m-th keys for its part and read its queries'
    // bounds (lanes kLanesPerQuery q .. + kLanesPerQuery - 1 take query q's
    // parts).  A row's prefilter threshold takes the new bound the next time
    // the row has candidates.
    auto refresh = [&]() {
      uint64_t *bound = prm->bound;
      const int peff = static_cast<int>(max<int64_t>(1, min<int64_t>(parts, (tile_hi - tile_lo + tpp - 1) / tpp)));
      const int mth = (k + peff - 1) / peff;
#pragma unroll
      for (int qi = 0; qi < QW; ++qi) {
        if (qi < nact) {
          const Key mk = list[qi].at(mth - 1);
          if (lane == 0 && mk) store_shared_key(bound + static_cast<int64_t>(q0 + qi) * parts + part, global(mk));
        }
      }
      const int rq = lane / kLanesPerQuery;
      uint64_t mn = 0;
      if (rq < nact)
        mn = min_published_keys(bound + static_cast<int64_t>(q0 + rq) * parts, lane % kLanesPerQuery, peff,
                                kLanesPerQuery);
#pragma unroll
      for (int off = 1; off < kLanesPerQuery; off <<= 1) {
        const uint64_t o = __shfl_xor(static_cast<unsigned long long>(mn), off);
        mn = o < mn ? o : mn;
      }
      if (lane % kLanesPerQuery == 0) {
        const uint64_t f = floor_of(rq);
        lb[rq] = local(mn > f ? mn : f);
      }
      __builtin_amdgcn_wave_barrier();
    };
    if (t0 < t1) {
      sa.load(tiles, t0, j);
      sb.load(tiles, min(t0 + 1, t1 - 1), j);
      sa.store(op[0], j);
      __syncthreads();
      // bounds are exchanged after 1, 2, 4, ..., 64 tiles, then every 64
      int next = 1;
      for (int64_t t = t0; t < t1; t += 2) {
        step(t, op[0], op[1], sa, sb);
        if (t + 1 < t1) step(t + 1, op[1], op[0], sb, sa);
        if (kPrune && prune && nact > 0 && static_cast<int>(t + 2 - t0) >= next) {
          refresh();
          next = next < 64 ? 2 * next : next + 64;
        }
      }
    }

    // a query belongs to one wave: its list is the (query, part) result
#pragma unroll
    for (int qi = 0; qi < QW; ++qi) {
      if (qi < nact) {
        uint64_t *dst = partial + (static_cast<int64_t>(q0 + qi) * parts + part) * k;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int p = r * 64 + lane;
          if (p < k) dst[p] = global(list[qi].v[r]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Small k (k <= 16): lists per 16-lane group, wider query tiles
// ---------------------------------------------------------------------------
//
// The accumulator of one 16x16 product holds, in lane l, rows 4 (l / 16) + i
// (i = 0..3) of column l % 16: the sixteen lanes of a group carry one query
// row's scores for sixteen database vectors.  For k <= 16 each query's list
// lives in exactly those lanes -- entry l % 16 of the list of row
// 4 (l / 16) + i sits in register i of lane l -- so a list costs a quarter of a
// register pair, the four groups insert their own candidates at the same
// time, and a wave holds 16 RB queries: 64-query tiles are four waves with
// RB = 1, 128-query tiles eight waves with RB = 1 (half the staging work per
// thread), 256-query tiles eight waves with RB = 2 (twice the operand reuse in
// every wave as well).

// 16 keys per group, descending; empty entries are 0.
struct GroupList {
  uint64_t v;

  // insert c (this lane's group candidate) where `act`; entries shift down
  __device__ __forceinline__ void insert(uint64_t c, bool act) {
    const uint64_t prev = dpp_move64<kDppRowShr1>(v, ~0ull);  // lane p - 1 of the group; ~0 at p = 0
    const uint64_t nv = (v > c) ? v : ((prev > c) ? c : prev);
    if (act) v = nv;
  }
};

// Entry p (uniform) of this lane's group list, given to every lane of the
// group.
__device__ __forceinline__ uint64_t group_entry(uint64_t v, int gbase, int p) {
  return __shfl(static_cast<unsigned long long>(v), gbase + p);
}

// SAMPLE: the sample pass of the k > 16 scan -- tiles tile_lo + i tstride
// only, i = 0, 1, ..., split over this grid like a database of that many tiles
// (sample_split), with lists of sample_list_len(parts, k) keys; its own
// instantiation, so that the full scan keeps its registers.
template <int NC, int RB, int WV, bool SAMPLE>
__global__ __launch_bounds__(64 * WV, RB * WV <= 8 ? 8 / WV : 1) void scan_mfma_group_kernel(const uint4 *__restrict__ tiles, int64_t n,
                                                                    const uint32_t *__restrict__ qprep,
                                                                    const BatchParams *__restrict__ prm, int k,
                                                                    uint64_t *__restrict__ partial, int stride) {
  const int tstride = SAMPLE ? stride : 1;
  constexpr int QW = 16 * RB;
  constexpr int QT = WV * QW;
  __shared__ v4i op[2][NC * 4 * 64];
  const int j = threadIdx.x;
  const int lane = j & 63;
  const int wave = j >> 6;
  const int col = lane & 15;
  const int grp = lane >> 4;
  const int gbase = lane & ~15;
  BatchParams sp;
  const BatchParams *split = prm;
  int64_t abase = 0;  // database tile of index t: abase + t * tstride
  if (SAMPLE) {
    sample_split(sp, *prm, QT, static_cast<int>(gridDim.x), tstride);
    split = &sp;
    abase = prm->tile_lo;
  }
  const int nq = split->nq, nqt = split->nqt, parts = split->parts;
  const int64_t tpp = split->tiles_per_part;
  const int64_t tile_lo = split->tile_lo, tile_hi = split->tile_hi;
  const int items = nqt * parts;
  const int lk = SAMPLE ? sample_list_len(parts, k) : k;  // keys per list
  const int km1 = lk - 1;

  for (int item = blockIdx.x; item < items; item += gridDim.x) {
    int qt, part;
    item_coords(item, nqt, &qt, &part);
    const int q0 = qt * QT + wave * QW;
    const int nact = max(0, min(QW, nq - q0));
    const int64_t t0 = tile_lo + static_cast<int64_t>(part) * tpp;
    const int64_t t1 = min(tile_hi, t0 + tpp);

    v4i a[RB][NC];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int qi = rb * 16 + col;
      const uint32_t *qw = qprep + static_cast<int64_t>(q0 + qi) * (8 * NC);
#pragma unroll
      for (int s = 0; s < NC; ++s) {
        uint32_t nz = 0, ng = 0;
        if (qi < nact) {
          nz = qw[4 * s + grp];
          ng = qw[4 * NC + 4 * s + grp];
        }
        a[rb][s] = fp4_operand(nz, ng);
      }
    }
    // list[rb][i] of lane l: entry l % 16 of row 16 rb + 4 (l / 16) + i;
    // tv[rb][i]: that row's k-th score (rows past the real queries never pass)
    GroupList list[RB][4];
    float tv[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        list[rb][i].v = 0;
        tv[rb][i] = (rb * 16 + 4 * grp + i < nact) ? -1e30f : 1e30f;
      }

    TileStage<NC, WV> sa, sb;
    auto step = [&](int64_t t, const v4i *cur, v4i *nxt, TileStage<NC, WV> &fill, const TileStage<NC, WV> &ready) {
      fill.load(tiles, abase + min(t + 2, t1 - 1) * tstride, j);
      if (nact > 0) {
        v4f acc[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) acc[rb][cb] = v4f{0.f, 0.f, 0.f, 0.f};
        // K-steps with the next step's four B operands already in flight
        v4i bq[2][4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) bq[0][cb] = cur[cb * 64 + lane];
#pragma unroll
        for (int s = 0; s < NC; ++s) {
          if (s + 1 < NC) {
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) bq[(s + 1) & 1][cb] = cur[((s + 1) * 4 + cb) * 64 + lane];
          }
#pragma unroll
          for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[rb][cb] = mfma_fp4(a[rb][s], bq[s & 1][cb], acc[rb][cb]);
        }
        uint64_t rows[RB][4];
        bool any = false;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            // (the scores are small integers: plain compares, no NaN handling)
            const bool c = acc[rb][0][i] > tv[rb][i] || acc[rb][1][i] > tv[rb][i] || acc[rb][2][i] > tv[rb][i] ||
                           acc[rb][3][i] > tv[rb][i];
            rows[rb][i] = __builtin_amdgcn_ballot_w64(c);
            any |= rows[rb][i] != 0;
          }
        if (any) {
#pragma unroll
          for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              if (!rows[rb][i]) continue;
              GroupList &L = list[rb][i];
              uint64_t thr = group_entry(L.v, gbase, km1);
#pragma unroll
              for (int cb = 0; cb < 4; ++cb) {
                const int64_t id = (abase + t * tstride) * 64 + cb * 16 + col;
                const uint64_t key = make_key(static_cast<int32_t>(acc[rb][cb][i]), static_cast<uint32_t>(id));
                uint64_t m = __ballot(id < n && key > thr);
                while (m) {
                  // every group takes its lowest pending lane
                  const uint32_t mg = static_cast<uint32_t>(m >> gbase) & 0xFFFFu;
                  const int src = gbase + __builtin_ctz(mg | 0x10000u);
                  const uint64_t c = __shfl(static_cast<unsigned long long>(key), src & 63);
                  L.insert(c, mg != 0 && c > thr);
                  m &= ~__ballot(mg != 0 && lane == src);
                  thr = group_entry(L.v, gbase, km1);
                  m &= __ballot(key > thr);
                }
              }
              tv[rb][i] = score_of(thr);
            }
          }
        }
      }
      ready.store(nxt, j);
      __syncthreads();
    };
    if (t0 < t1) {
      sa.load(tiles, abase + t0 * tstride, j);
      sb.load(tiles, abase + min(t0 + 1, t1 - 1) * tstride, j);
      sa.store(op[0], j);
      __syncthreads();
      for (int64_t t = t0; t < t1; t += 2) {
        step(t, op[0], op[1], sa, sb);
        if (t + 1 < t1) step(t + 1, op[1], op[0], sb, sa);
      }
    }

    // entry p < k of row 16 rb + 4 grp + i is lane 16 grp + p of list[rb][i]
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int qi = rb * 16 + 4 * grp + i;
        if (qi < nact && col < lk)
          partial[(static_cast<int64_t>(q0 + qi) * parts + part) * lk + col] = list[rb][i].v;
      }
  }
}

// ---------------------------------------------------------------------------
// Sample floor for k > 16
// ---------------------------------------------------------------------------
//
// The sample pass keeps the top 8 or 16 keys of every (query, part) of every
// stride-th tile.  Those keys are database keys, so if at least k of them score
// >= s, the query's k-th key overall scores >= s and no key scoring below s
// can be in its result.  One workgroup per query counts the sample keys per
// score and takes the largest such s; the floor is the largest key of score
// s - 1 (the id field of id 0), so exactly the keys scoring >= s pass it.
constexpr int kFloorBlock = 256;
constexpr int kScoreSpan = 1024;                            // |Delta| <= d <= 1024
constexpr int kBinsPerThread = (2 * kScoreSpan + 1 + kFloorBlock - 1) / kFloorBlock;  // 9
constexpr int kBins = kBinsPerThread * kFloorBlock;         // score s -> bin s + kScoreSpan

__global__ __launch_bounds__(kFloorBlock) void sample_floor_kernel(const uint64_t *__restrict__ sp,
                                                                   const BatchParams *__restrict__ prm, int qtile,
                                                                   int grid, int tstride, int k,
                                                                   uint64_t *__restrict__ floor) {
  __shared__ int hist[kBins];
  __shared__ int chunk[kFloorBlock];
  BatchParams b;
  sample_split(b, *prm, qtile, grid, tstride);
  const int q = blockIdx.x;
  if (q >= b.nq) return;
  const int j = threadIdx.x;
  for (int i = j; i < kBins; i += kFloorBlock) hist[i] = 0;
  __syncthreads();
  const int64_t cnt = static_cast<int64_t>(b.parts) * sample_list_len(b.parts, k);
  const uint64_t *src = sp + static_cast<int64_t>(q) * cnt;
  for (int64_t i = j; i < cnt; i += kFloorBlock) {
    const uint64_t key = src[i];
    if (key) atomicAdd(&hist[min(max(key_score(key), -kScoreSpan), kScoreSpan) + kScoreSpan], 1);
  }
  __syncthreads();
  int c = 0;
#pragma unroll
  for (int i = 0; i < kBinsPerThread; ++i) c += hist[j * kBinsPerThread + i];
  chunk[j] = c;
  __syncthreads();
  if (j >= 64) return;
  // lane l holds chunks 255 - 4l .. 252 - 4l (highest scores first)
  int c4[4], sum = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    c4[i] = chunk[kFloorBlock - 1 - 4 * j - i];
    sum += c4[i];
  }
  int incl = sum;  // keys in the chunks of lanes 0..l
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(incl, off);
    if (j >= off) incl += o;
  }
  const uint64_t reach = __ballot(incl >= k);
  if (!reach) {
    if (j == 0) floor[q] = 0;  // fewer than k sample keys: no floor
    return;
  }
  if (j != __builtin_ctzll(reach)) return;
  int above = incl - sum;  // keys scoring above this lane's chunks
  for (int i = 0; i < 4; ++i) {
    const int ch = kFloorBlock - 1 - 4 * j - i;
    if (above + c4[i] >= k) {
      for (int bin = ch * kBinsPerThread + kBinsPerThread - 1;; --bin) {
        above += hist[bin];
        if (above >= k) {
          floor[q] = make_key(bin - kScoreSpan - 1, 0);
          return;
        }
      }
    }
    above += c4[i];
  }
}

template <int NC, int RB, int WV = kMfmaWaves>
hipError_t launch_g(const DbDev &db, const uint32_t *qprep, const BatchParams *prm, int k, int grid,
                    uint64_t *partial, hipStream_t s, int tstride = 1) {
  if (tstride > 1)
    hipLaunchKernelGGL((scan_mfma_group_kernel<NC, RB, WV, true>), dim3(grid), dim3(64 * WV), 0, s, db.tiles, db.n,
                       qprep, prm, k, partial, tstride);
  else
    hipLaunchKernelGGL((scan_mfma_group_kernel<NC, RB, WV, false>), dim3(grid), dim3(64 * WV), 0, s, db.tiles, db.n,
                       qprep, prm, k, partial, 1);
  return hipGetLastError();
}

template <int NC, int R, int RB, int WV = kMfmaWaves>
hipError_t launch_m3(const DbDev &db, const uint32_t *qprep, const BatchParams *prm, int k, int grid, bool k32,
                     uint64_t *partial, const uint64_t *floor, hipStream_t s) {
  if (k32)
    hipLaunchKernelGGL((scan_mfma_kernel<NC, R, RB, WV, true>), dim3(grid), dim3(64 * WV), 0, s, db.tiles, db.n,
                       qprep, prm, k, partial, floor);
  else
    hipLaunchKernelGGL((scan_mfma_kernel<NC, R, RB, WV, false>), dim3(grid), dim3(64 * WV), 0, s, db.tiles, db.n,
                       qprep, prm, k, partial, floor);
  return hipGetLastError();
}

}  // namespace

template <int NC>
hipError_t scan_mfma_launch_nc(const DbDev &db, const uint32_t *qprep, const BatchParams *prm, int k, int qtile,
                               int grid, int64_t max_part_tiles, uint64_t *partial, hipStream_t s,
                               const MfmaSample &sample) {
  const bool k32 = max_part_tiles * 64 <= static_cast<int64_t>(kLidMask) + 1;
  if (k <= kGroupMaxK) {
    if (qtile == 64) return launch_g<NC, 1>(db, qprep, prm, k, grid, partial, s);
    if (qtile == 128) return launch_g<NC, 1, 8>(db, qprep, prm, k, grid, partial, s);  // eight waves of 16
    return launch_g<NC, 2, 8>(db, qprep, prm, k, grid, partial, s);  // 256: eight waves of 32
  }
  const uint64_t *floor = nullptr;
  if (sample.stride > 1) {
    if (!sample.floor || sample.bucket < 1) return hipErrorInvalidValue;
    // the sample takes the group kernel of the same query tile, so both
    // passes and the floor kernel split the batch alike
    hipError_t e = qtile == 64 ? launch_g<NC, 1>(db, qprep, prm, k, grid, partial, s, sample.stride)
                   : qtile == 128 ? launch_g<NC, 1, 8>(db, qprep, prm, k, grid, partial, s, sample.stride)
                                  : launch_g<NC, 2, 8>(db, qprep, prm, k, grid, partial, s, sample.stride);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sample_floor_kernel, dim3(sample.bucket), dim3(kFloorBlock), 0, s,
                       static_cast<const uint64_t *>(partial), prm, qtile, grid, sample.stride, k, sample.floor);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    floor = sample.floor;
  }
  const int r = rows_for_k(k);
  if (qtile == 64) return r == 1 ? launch_m3<NC, 1, 1>(db, qprep, prm, k, grid, k32, partial, floor, s)
                                 : launch_m3<NC, 2, 1>(db, qprep, prm, k, grid, k32, partial, floor, s);
  // 128-query tiles: eight waves of 16 queries share each staged tile
  if (qtile == 128) return r == 1 ? launch_m3<NC, 1, 1, 8>(db, qprep, prm, k, grid, k32, partial, floor, s)
                                  : launch_m3<NC, 2, 1, 8>(db, qprep, prm, k, grid, k32, partial, floor, s);
  // 256-query tiles: eight waves of 32 queries, each B operand read feeds two
  // products (half the LDS reads of the 128-query form per product)
  return r == 1 ? launch_m3<NC, 1, 2, 8>(db, qprep, prm, k, grid, k32, partial, floor, s)
                : launch_m3<NC, 2, 2, 8>(db, qprep, prm, k, grid, k32, partial, floor, s);
}

// This file is compiled once per plane width (-DTQ_NC=1..8), so that the
// eight instantiations build in parallel.
#ifndef TQ_NC
#error "compile mfma_kernels.hip with -DTQ_NC=<1..8>"
#endif
template hipError_t scan_mfma_launch_nc<TQ_NC>(const DbDev &, const uint32_t *, const BatchParams *, int, int, int,
                                               int64_t, uint64_t *, hipStream_t, const MfmaSample &);

}  // namespace tqi
