// tq_device.h -- device-side building blocks shared by the scan kernels:
// Delta over bit planes, wave-wide register top-k lists, LDS list merges.
#pragma once

#include "tq_internal.h"

namespace tqi {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Streaming 16-byte load that should not displace reused data from the caches.
__device__ __forceinline__ u32x4 load_stream(const uint4 *p) {
  return __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
}

// ---------------------------------------------------------------------------
// Delta (b2sp, Sec. 5.1.2) on the nz / ng re-coding
// ---------------------------------------------------------------------------
//
// With q+, q-, v+, v- the paper's bit vectors, b2sp is
//   (|q+ & v+| + |q- & v-|) - (|q+ & v-| + |q- & v+|).
// Let both = nz_q & nz_v (coordinates where both vectors are non-zero) and
// dis = both & (ng_q ^ ng_v) (those where the signs differ).  Each coordinate
// in `both` contributes +1 if the signs agree and -1 if they differ, so
//   b2sp = |both| - 2 |dis|,
// the same integer, from 5 operations per 32 coordinates (and, xor, and, and
// two popcount-accumulates) instead of 8.  Accumulators are per lane.
struct DeltaAcc {
  uint32_t both = 0;
  uint32_t dis = 0;
};

__device__ __forceinline__ void delta_word(DeltaAcc &a, uint32_t qnz, uint32_t qng, uint32_t vnz,
                                           uint32_t vng) {
  const uint32_t both = qnz & vnz;
  const uint32_t dis = both & (qng ^ vng);
  a.both += __popc(both);
  a.dis += __popc(dis);
}

__device__ __forceinline__ int32_t delta_value(const DeltaAcc &a) {
  return static_cast<int32_t>(a.both) - 2 * static_cast<int32_t>(a.dis);
}

// Query words in nz / ng form for chunks [0, NC); words past W are zero.
template <int NC>
struct QueryWords {
  uint32_t nz[4 * NC];
  uint32_t ng[4 * NC];
  __device__ __forceinline__ void load(const uint32_t *__restrict__ qcode, int W) {
#pragma unroll
    for (int w = 0; w < 4 * NC; ++w) {
      uint32_t p = 0, m = 0;
      if (w < W) {
        p = qcode[w];
        m = qcode[W + w];
      }
      nz[w] = p | m;
      ng[w] = m;
    }
  }
};

// This lane's vector of one tile: NC 16-byte chunks of each plane.
template <int NC>
struct TileVec {
  u32x4 vz[NC], vg[NC];
  __device__ __forceinline__ void load(const uint4 *__restrict__ tile, int lane) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      vz[c] = load_stream(tile + c * 64 + lane);
      vg[c] = load_stream(tile + (NC + c) * 64 + lane);
    }
  }
};

template <int NC>
__device__ __forceinline__ int32_t vec_delta(const TileVec<NC> &v, const QueryWords<NC> &q) {
  DeltaAcc a;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    delta_word(a, q.nz[4 * c + 0], q.ng[4 * c + 0], v.vz[c].x, v.vg[c].x);
    delta_word(a, q.nz[4 * c + 1], q.ng[4 * c + 1], v.vz[c].y, v.vg[c].y);
    delta_word(a, q.nz[4 * c + 2], q.ng[4 * c + 2], v.vz[c].z, v.vg[c].z);
    delta_word(a, q.nz[4 * c + 3], q.ng[4 * c + 3], v.vz[c].w, v.vg[c].w);
  }
  return delta_value(a);
}

// Non-zeros of this lane's vector (popcount of its nz plane): with it,
// 2 Delta - nnz(v) = nnz(q) - |q - v|^2 orders ternary vectors of varying
// non-zero counts by euclidean distance.
template <int NC>
__device__ __forceinline__ int32_t vec_nnz(const u32x4 (&vz)[NC]) {
  uint32_t s = 0;
#pragma unroll
  for (int c = 0; c < NC; ++c) s += __popc(vz[c].x) + __popc(vz[c].y) + __popc(vz[c].z) + __popc(vz[c].w);
  return static_cast<int32_t>(s);
}

// Delta of the query against the 64 vectors of one tile (this lane's vector).
template <int NC>
__device__ __forceinline__ int32_t tile_delta(const uint4 *__restrict__ tile, int lane,
                                              const QueryWords<NC> &q) {
  u32x4 vz[NC], vg[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    vz[c] = load_stream(tile + c * 64 + lane);
    vg[c] = load_stream(tile + (NC + c) * 64 + lane);
  }
  DeltaAcc a;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    delta_word(a, q.nz[4 * c + 0], q.ng[4 * c + 0], vz[c].x, vg[c].x);
    delta_word(a, q.nz[4 * c + 1], q.ng[4 * c + 1], vz[c].y, vg[c].y);
    delta_word(a, q.nz[4 * c + 2], q.ng[4 * c + 2], vz[c].z, vg[c].z);
    delta_word(a, q.nz[4 * c + 3], q.ng[4 * c + 3], vz[c].w, vg[c].w);
  }
  return delta_value(a);
}

// ---------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
  const uint32_t lo = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v)), l);
  const uint32_t hi = __builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(v >> 32)), l);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// DPP lane moves (one VALU instruction each, no LDS round trip).  A lane
// whose source lies outside the wave or row keeps `fill`.  Callers run with
// every lane of the wave active.
constexpr int kDppWaveShr1 = 0x138;  // lane l takes lane l - 1 of the wave
constexpr int kDppRowShr1 = 0x111;   // lane l takes lane l - 1 of its row of 16

template <int Ctrl>
__device__ __forceinline__ uint64_t dpp_move64(uint64_t v, uint64_t fill) {
  const uint32_t lo = __builtin_amdgcn_update_dpp(static_cast<uint32_t>(fill), static_cast<uint32_t>(v), Ctrl, 0xf,
                                                  0xf, false);
  const uint32_t hi = __builtin_amdgcn_update_dpp(static_cast<uint32_t>(fill >> 32), static_cast<uint32_t>(v >> 32),
                                                  Ctrl, 0xf, 0xf, false);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Value of lane (l - 1) for lanes 1..63; lane 0 gets `fill`.
__device__ __forceinline__ uint64_t shift_up1(uint64_t v, uint64_t fill) { return dpp_move64<kDppWaveShr1>(v, fill); }

// ---------------------------------------------------------------------------
// Wave-wide sorted list in registers
// ---------------------------------------------------------------------------
//
// 64*R keys, descending, striped: position r*64 + lane lives in list[r] of
// that lane.  Empty slots hold 0.  Every lane must call insert with the same
// (uniform) key.
template <int R>
struct WaveList {
  uint64_t v[R];

  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = 0;
  }

  // Key at position p (p uniform, 0 <= p < 64*R); uniform result.
  __device__ __forceinline__ uint64_t at(int p) const {
    uint64_t res = 0;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (r == (p >> 6)) res = readlane64(v[r], p & 63);
    return res;
  }

  __device__ __forceinline__ void insert(uint64_t key) {
    uint64_t prev[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t carry = (r == 0) ? ~0ull : readlane64(v[r - 1], 63);
      prev[r] = shift_up1(v[r], carry);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      // keep the entry if it beats the key; else the key goes in the first
      // such place and every later entry moves down by one
      v[r] = (v[r] > key) ? v[r] : ((prev[r] > key) ? key : prev[r]);
    }
  }
};

// Offer this lane's key (valid only where `ok`) to the wave's list; `thr` is
// the current k-th key (uniform), updated in place, and never below `floor`
// (keys at or below it are known to be outside the result).  Candidates are
// taken in lane order, i.e. in increasing database id within the tile.
template <int R>
__device__ __forceinline__ void offer_keys(WaveList<R> &list, uint64_t &thr, uint64_t key, bool ok,
                                           int k_minus_1, uint64_t floor = 0) {
  uint64_t m = __ballot(ok && key > thr);
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

// Smallest of the keys p[first], p[first + step], ... below p[end], read with
// relaxed device-scope loads (keys other workgroups publish); ~0 if there are
// none.  Eight loads are issued before the first is waited for: one at a time,
// each would cost a full round trip to the device-coherent level.  The last
// group re-reads p[first] in place of the indices past `end`, which cannot
// change a minimum.
__device__ __forceinline__ uint64_t min_published_keys(const uint64_t *p, int first, int end, int step) {
  uint64_t mn = ~0ull;
  if (first >= end) return mn;
  constexpr int kInFlight = 8;
  for (int i0 = first; i0 < end; i0 += kInFlight * step) {
    uint64_t v[kInFlight];
#pragma unroll
    for (int b = 0; b < kInFlight; ++b) {
      const int i = i0 + b * step;
      v[b] = __hip_atomic_load(p + (i < end ? i : first), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int b = 0; b < kInFlight; ++b) mn = v[b] < mn ? v[b] : mn;
  }
  return mn;
}

// ---------------------------------------------------------------------------
// Workgroup-wide merge of sorted lists in LDS
// ---------------------------------------------------------------------------
//
// `a` and `b` hold k keys each, descending, unique apart from 0 (empty).
// Writes the k largest of their union, descending, to `out`, which the
// caller has zero-filled.  Each non-empty key's place in the union is its
// own index plus the number of keys of the other list that beat it (a binary
// search), and those places are distinct because the keys are.
__device__ __forceinline__ void merge_pair_scatter(const uint64_t *a, const uint64_t *b,
                                                   uint64_t *out, int k, int e) {
  const bool in_a = e < k;
  const int p = in_a ? e : e - k;
  const uint64_t *self = in_a ? a : b;
  const uint64_t *other = in_a ? b : a;
  const uint64_t key = self[p];
  if (key == 0) return;
  int lo = 0, hi = k;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (other[mid] > key)
      lo = mid + 1;
    else
      hi = mid;
  }
  const int place = p + lo;
  if (place < k) out[place] = key;
}

// Tree-merge `nl` (a power of two) sorted lists of k keys stored back to back
// in `buf`, using `tmp` (same size) as scratch.  All threads of the block must
// call it; it starts and ends with a barrier.  Returns the buffer holding the
// merged list in its first k slots.
__device__ inline uint64_t *tree_merge(uint64_t *buf, uint64_t *tmp, int nl, int k) {
  const int tid = threadIdx.x, nt = blockDim.x;
  __syncthreads();
  for (int w = nl; w > 1; w >>= 1) {
    const int half = w >> 1;
    for (int i = tid; i < half * k; i += nt) tmp[i] = 0;
    __syncthreads();
    for (int i = tid; i < half * 2 * k; i += nt) {
      const int m = i / (2 * k);
      const int e = i - m * 2 * k;
      merge_pair_scatter(buf + (2 * m) * k, buf + (2 * m + 1) * k, tmp + m * k, k, e);
    }
    __syncthreads();
    uint64_t *t = buf;
    buf = tmp;
    tmp = t;
  }
  return buf;
}

}  // namespace tqi
