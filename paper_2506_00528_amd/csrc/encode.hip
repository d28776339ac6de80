// encode.hip -- nearest {x,d} EVP vertex of each float row, written as the
// two bit planes v+ / v- (Sec. 2.4 mapping, Sec. 5.1.2 / Table 3 bit vectors).
//
// One wave per row.  Lane l holds coordinates l, l+64, l+128, ... so the row
// is read with coalesced loads and every 64-bit ballot over one register is
// exactly two 32-bit words of a bit plane (coordinates 64j .. 64j+63).
//
// Selecting the x largest magnitudes: |u_i| is compared as the unsigned bit
// pattern of the float with its sign cleared, which orders finite floats
// exactly (subnormals included).  A bisection over those 31-bit patterns
// finds the x-th largest magnitude t (the largest t with count(|u| >= t) >=
// x); it stops early at any cut with exactly x magnitudes at or above it.
// Then every coordinate above t is taken, and among those equal to t the
// lowest indices fill the remaining places (ties go to the lower index).
// The sign is "-1 iff u_i < 0", i.e. sign bit set and magnitude non-zero, so
// both zeros give +1.
#include "tq_internal.h"

namespace tqi {
namespace {

constexpr int kEncodeBlock = 256;

template <int J>
__global__ __launch_bounds__(kEncodeBlock) void encode_kernel(const float *__restrict__ X, int64_t n,
                                                             int d, int x, int W,
                                                             uint32_t *__restrict__ codes,
                                                             int *__restrict__ flags) {
  constexpr int kWordsPerLane = (4 * J + 63) / 64;  // 2W <= 4J code words per row
  const int lane = threadIdx.x & 63;
  const int64_t waves_per_block = kEncodeBlock / 64;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * waves_per_block;
  const int row_words = 2 * W;

  for (int64_t row = static_cast<int64_t>(blockIdx.x) * waves_per_block + (threadIdx.x >> 6); row < n;
       row += nwaves) {
    const float *u = X + row * d;
    uint32_t mag[J];
    bool neg[J], valid[J];
    bool bad = false;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int i = j * 64 + lane;
      valid[j] = i < d;
      uint32_t bits = 0;
      if (valid[j]) bits = __float_as_uint(__builtin_nontemporal_load(u + i));
      mag[j] = bits & 0x7FFFFFFFu;
      neg[j] = (bits >> 31) != 0 && mag[j] != 0;
      bad |= mag[j] >= 0x7F800000u;  // infinity or NaN
    }
    uint32_t out[kWordsPerLane];
#pragma unroll
    for (int s = 0; s < kWordsPerLane; ++s) out[s] = 0;

    if (__any(bad)) {
      if (lane == 0) atomicOr(flags, 1);
    } else {
      // --- the x-th largest magnitude -------------------------------------
      uint32_t t = 0;       // invariant: count(mag >= t) >= x
      uint32_t cut = 0;     // set when a cut with exactly x at or above is met
      for (int b = 30; b >= 0; --b) {
        const uint32_t cand = t | (1u << b);
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < J; ++j) cnt += __popcll(__ballot(mag[j] >= cand));
        if (cnt == x) {
          cut = cand;
          break;
        }
        if (cnt > x) t = cand;
      }
      // take mag >= lo outright; if there was no exact cut, also take the
      // lowest-index `need` coordinates with mag == t
      const bool exact = cut != 0;
      const uint32_t lo = exact ? cut : t + 1;
      int above = 0;
#pragma unroll
      for (int j = 0; j < J; ++j) above += __popcll(__ballot(mag[j] >= lo));
      const int need = x - above;
      int eq_before = 0;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const uint64_t gt = __ballot(mag[j] >= lo);
        const uint64_t eq = exact ? 0ull : __ballot(valid[j] && mag[j] == t);
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
            static_cast<uint32_t>(eq >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(eq), 0u));
        const bool take = ((eq >> lane) & 1ull) && (eq_before + static_cast<int>(rank) < need);
        const uint64_t sel = gt | __ballot(take);
        eq_before += __popcll(eq);
        const uint64_t negm = __ballot(neg[j]);
        const uint64_t plus = sel & ~negm;
        const uint64_t minus = sel & negm;
        // plane words 2j and 2j+1 (coordinates 64j .. 64j+63)
        const uint32_t wv[4] = {static_cast<uint32_t>(plus), static_cast<uint32_t>(plus >> 32),
                                static_cast<uint32_t>(minus), static_cast<uint32_t>(minus >> 32)};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const int pw = 2 * j + (h & 1);  // word within the plane
          if (pw >= W) continue;
          const int w = (h < 2 ? 0 : W) + pw;  // word within the row
#pragma unroll
          for (int s = 0; s < kWordsPerLane; ++s)
            if (w == s * 64 + lane) out[s] = wv[h];
        }
      }
    }
    uint32_t *dst = codes + row * row_words;
#pragma unroll
    for (int s = 0; s < kWordsPerLane; ++s) {
      const int w = s * 64 + lane;
      if (w < row_words) dst[w] = out[s];
    }
  }
}

template <int J>
hipError_t launch_j(const float *X, int64_t n, int d, int x, uint32_t *codes, int *flags, int num_cu,
                    hipStream_t s) {
  int64_t blocks = (n + 3) / 4;  // one wave per row, four waves per block
  const int64_t cap = static_cast<int64_t>(num_cu > 0 ? num_cu : 256) * 16;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(encode_kernel<J>, dim3(static_cast<unsigned>(blocks)), dim3(kEncodeBlock), 0, s, X,
                     n, d, x, (d + 31) / 32, codes, flags);
  return hipGetLastError();
}

}  // namespace

hipError_t encode_launch(const float *X, int64_t n, int d, int x, uint32_t *codes, int *flags,
                         int num_cu, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int j = (d + 63) / 64;
  if (j <= 1) return launch_j<1>(X, n, d, x, codes, flags, num_cu, s);
  if (j <= 2) return launch_j<2>(X, n, d, x, codes, flags, num_cu, s);
  if (j <= 4) return launch_j<4>(X, n, d, x, codes, flags, num_cu, s);
  if (j <= 6) return launch_j<6>(X, n, d, x, codes, flags, num_cu, s);
  if (j <= 8) return launch_j<8>(X, n, d, x, codes, flags, num_cu, s);
  if (j <= 12) return launch_j<12>(X, n, d, x, codes, flags, num_cu, s);
  return launch_j<16>(X, n, d, x, codes, flags, num_cu, s);
}

}  // namespace tqi
