// encode.hip -- nearest {x,d} EVP vertex of each float row, written as the
// two bit planes v+ / v- (Sec. 2.4 mapping, Sec. 5.1.2 / Table 3 bit vectors).
//
// One wave per row.  Lane l holds coordinates l, l+64, l+128, ... so the row
// is read with coalesced loads and every 64-bit ballot over one register is
// exactly two 32-bit words of a bit plane (coordinates 64j .. 64j+63).
//
// Selecting the x largest magnitudes: magnitudes are compared as floats
// with the sign dropped (|u_i|), which orders finite values exactly like the
// unsigned bit patterns of |u_i| (subnormals included: f32 denormals are not
// flushed).  The x-th largest magnitude t is the largest pattern with
// count(|u| >= t) >= x; it is found by a binary search over patterns on an
// interval [lo, hi) with count(>= lo) >= x > count(>= hi), stopping early at
// any cut with exactly x magnitudes at or above it.
//   * A wave scans rows one after another, and rows of one data set have
//     similar thresholds, so the search starts by bracketing the previous
//     row's t with galloping steps; a wave's first row starts from a quarter
//     of its largest magnitude (a good guess only saves work; the result
//     never depends on it).
//   * Each count over the whole row costs one compare and one ballot per
//     register.  Once the interval holds at most 64 magnitudes, they are
//     compacted through LDS into one value per lane (without branches: lanes
//     outside the interval write to a slot of their own that is never read)
//     and the rest of the search costs one compare per step.
// Then every coordinate above t is taken, and among those equal to t the
// lowest indices fill the remaining places (ties go to the lower index).  The
// sign is "-1 iff u_i < 0" (a float compare), so both zeros give +1.  When
// exactly x magnitudes are >= a cut c > 0 (the usual case), v+ is u_i >= c and
// v- is u_i <= -c: two compares and no mask arithmetic per register.
#include <utility>

#include "tq_internal.h"

namespace tqi {

// The compiler's lane-write intrinsic (v_writelane_b32).  Unlike inline
// assembly it is visible to the hazard recognizer, which inserts the wait
// states a lane write needs when a vector compare has just written its
// operand (a ballot written to VCC and read at once).  (Declared outside the
// anonymous namespace: it names an intrinsic, not a function of this file.)
__device__ int amdgcn_writelane(int val, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

namespace {

constexpr int kEncodeBlock = 256;
// First bracketing step, in magnitude patterns: 1/16 of a binade (measured
// best among 2^13 .. 2^22 on the Gaussian-mixture workloads at d = 384 .. 1024).
constexpr uint32_t kGallop = 1u << 19;
// A wave's first row has no previous threshold: it starts from a quarter of
// the row's largest magnitude (two binades down) with steps of 2^21 patterns
// (about 4.5 full-row counts instead of 10 on the same workloads).
constexpr uint32_t kFirstDrop = 2u << 23;
constexpr uint32_t kGallopFirst = 1u << 21;
constexpr uint32_t kInfBits = 0x7F800000u;  // above every finite magnitude

__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }

// lanes whose predicate holds (the compare masks combine without a detour
// through a 0/1 integer)
__device__ __forceinline__ uint64_t vote(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ float pat(uint32_t p) { return __uint_as_float(p); }

// The row's magnitudes are folded with the IEEE-754 (2019) maximum, which
// returns NaN when an operand is NaN (three operands per instruction), so one
// compare of the result finds every infinity and NaN.

__device__ __forceinline__ int lanes_below(uint64_t m) {
  return static_cast<int>(
      __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u)));
}


// v with lane L replaced by the uniform value `val`
template <int L>
__device__ __forceinline__ uint32_t put_lane(uint32_t v, uint32_t val) {
  return static_cast<uint32_t>(amdgcn_writelane(static_cast<int>(val), L, static_cast<int>(v)));
}

// Plane words 2j and 2j+1 (coordinates 64j .. 64j+63) of the selection
// sel(j): the v+ words go to lanes 2j, 2j+1 of *plus, the v- words to the same
// lanes of *minus.
template <int J, typename Sel, int... Js>
__device__ __forceinline__ void pack_planes(const float (&v)[J], Sel sel, uint32_t *plus, uint32_t *minus,
                                            std::integer_sequence<int, Js...>) {
  auto one = [&](auto jc) {
    constexpr int j = decltype(jc)::value;
    const uint64_t s = sel(j);
    const uint64_t neg = vote(v[j] < 0.0f);
    const uint64_t p = s & ~neg, m = s & neg;
    *plus = put_lane<2 * j>(*plus, static_cast<uint32_t>(p));
    *plus = put_lane<2 * j + 1>(*plus, static_cast<uint32_t>(p >> 32));
    *minus = put_lane<2 * j>(*minus, static_cast<uint32_t>(m));
    *minus = put_lane<2 * j + 1>(*minus, static_cast<uint32_t>(m >> 32));
  };
  (one(std::integral_constant<int, Js>{}), ...);
}

// The same for the exact-cut case: v+ and v- are ballots of their own
// predicates (u_i >= c and u_i <= -c).
template <int J, typename Pos, typename Neg, int... Js>
__device__ __forceinline__ void pack_signed(Pos pos, Neg neg, uint32_t *plus, uint32_t *minus,
                                            std::integer_sequence<int, Js...>) {
  auto one = [&](auto jc) {
    constexpr int j = decltype(jc)::value;
    const uint64_t p = pos(j), m = neg(j);
    *plus = put_lane<2 * j>(*plus, static_cast<uint32_t>(p));
    *plus = put_lane<2 * j + 1>(*plus, static_cast<uint32_t>(p >> 32));
    *minus = put_lane<2 * j>(*minus, static_cast<uint32_t>(m));
    *minus = put_lane<2 * j + 1>(*minus, static_cast<uint32_t>(m >> 32));
  };
  (one(std::integral_constant<int, Js>{}), ...);
}

// J registers of 64 coordinates per row; the first JV are always inside the
// row (d >= 64 JV for every d this instantiation serves).
template <int J, int JV>
__global__ __launch_bounds__(kEncodeBlock) void encode_kernel(const float *__restrict__ X, int64_t n,
                                                             int d, int x, int W,
                                                             uint32_t *__restrict__ codes,
                                                             int *__restrict__ flags) {
  // 2W <= 4J <= 64 code words per row: one word per lane
  __shared__ uint32_t pool[2 * kEncodeBlock];
  const int lane = threadIdx.x & 63;
  // this wave's 64 compaction slots, then one discard slot per lane
  uint32_t *slot = pool + 128 * __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t waves_per_block = kEncodeBlock / 64;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * waves_per_block;
  const int row_words = 2 * W;
  uint32_t guess = 0;  // threshold of this wave's previous row (0: none yet)

  const int64_t first = static_cast<int64_t>(blockIdx.x) * waves_per_block + (threadIdx.x >> 6);
  const float *u = X + first * d + lane;
  uint32_t *out = codes + first * row_words + lane;
  auto valid = [&](int j) { return j < JV || j * 64 + lane < d; };
  // The wave's next row is loaded while this one is encoded (its loads are
  // waited for only at the top of the next iteration).
  float nxt[J];
  auto load_row = [&](const float *p) {
#pragma unroll
    for (int j = 0; j < J; ++j) nxt[j] = valid(j) ? __builtin_nontemporal_load(p + 64 * j) : 0.0f;
  };
  if (first < n) load_row(u);
  for (int64_t row = first; row < n; row += nwaves, u += nwaves * d, out += nwaves * row_words) {
    float v[J];
    float top = 0.0f;  // largest magnitude; NaN if the row holds one
#pragma unroll
    for (int j = 0; j < J; ++j) {
      v[j] = nxt[j];
      top = __builtin_elementwise_maximum(top, fabsf(v[j]));
    }
    if (row + nwaves < n) load_row(u + nwaves * d);
    uint32_t plus = 0, minus = 0;

    if (__any(!(top < __builtin_huge_valf()))) {  // infinity or NaN
      if (lane == 0) atomicOr(flags, 1);
    } else {
      // count(|u| >= c) over the row, for patterns c >= 1 (padding holds 0)
      // (all J compares are issued first, each into its own scalar register
      // pair, and then the popcounts: a popcount right after the compare it
      // reads would wait for that compare's result every time)
      auto count_ge = [&](uint32_t c) {
        const float cf = pat(c);
        uint64_t mk[J];
#pragma unroll
        for (int j = 0; j < J; ++j) mk[j] = vote(fabsf(v[j]) >= cf);
        int cnt = 0;
#pragma unroll
        for (int j = 0; j < J; ++j) cnt += popc64(mk[j]);
        __builtin_amdgcn_sched_group_barrier(0x002, J, 0);      // vector ALU: the compares
        __builtin_amdgcn_sched_group_barrier(0x004, 2 * J, 0);  // scalar ALU: popcounts, sums
        return cnt;
      };
      uint32_t lo = 0, hi = kInfBits, cut = 0;
      int clo = d, chi = 0;  // count(|u| >= lo), count(|u| >= hi)
      // --- bracket the previous row's threshold ---------------------------
      uint32_t step0 = kGallop;
      if (guess == 0) {
        float m = top;  // finite here
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
        const uint32_t tb = __builtin_amdgcn_readfirstlane(__float_as_uint(m));
        guess = tb > kFirstDrop ? tb - kFirstDrop : (tb != 0 ? 1u : 0u);
        step0 = kGallopFirst;
      }
      if (guess != 0) {
        const int c = count_ge(guess);
        if (c == x) {
          cut = guess;
        } else if (c > x) {
          lo = guess;
          clo = c;
          for (uint32_t step = step0; step < hi - lo; step <<= 1) {
            const uint32_t h = lo + step;
            const int ch = count_ge(h);
            if (ch == x) {
              cut = h;
              break;
            }
            if (ch < x) {
              hi = h;
              chi = ch;
              break;
            }
            lo = h;
            clo = ch;
          }
        } else {
          hi = guess;
          chi = c;
          for (uint32_t step = step0; step < hi - lo; step <<= 1) {
            const uint32_t l = hi - step;
            const int cl = count_ge(l);
            if (cl == x) {
              cut = l;
              break;
            }
            if (cl > x) {
              lo = l;
              clo = cl;
              break;
            }
            hi = l;
            chi = cl;
          }
        }
      }
      // --- halve on the whole row while the interval holds > 64 ------------
      while (cut == 0 && clo - chi > 64 && hi - lo > 1) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        const int c = count_ge(mid);
        if (c == x) cut = mid;
        else if (c > x) lo = mid, clo = c;
        else hi = mid, chi = c;
      }
      // --- compact the interval's magnitudes into one register, finish ----
      if (cut == 0 && hi - lo > 1) {
        // clo - chi <= 64 magnitudes lie in [lo, hi): slots 0 .. clo - chi - 1
        const float lof = pat(lo), hif = pat(hi);
        uint32_t base = 0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
          const float a = fabsf(v[j]);
          const bool in = valid(j) && a >= lof && a < hif;
          // the ballot of each compare is its own result; one ballot of the
          // conjunction would be rebuilt from a 0/1 register
          uint64_t m = vote(a >= lof) & vote(a < hif);
          if (j >= JV) m &= vote(valid(j));
          const uint32_t at = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                                        __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), base));
          slot[in ? at : 64 + lane] = __float_as_uint(v[j]);
          base += popc64(m);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const float m2 = lane < static_cast<int>(base) ? fabsf(__uint_as_float(slot[lane])) : 0.0f;
        // every magnitude >= hi is outside the register: x - chi of the
        // register's values must be >= the cut
        const int need = x - chi;
        int reg_hi = 0;  // register values >= hi
        while (hi - lo > 1) {
          const uint32_t mid = lo + ((hi - lo) >> 1);
          const int c = popc64(vote(m2 >= pat(mid)));
          if (c == need) {
            cut = mid;
            break;
          }
          if (c > need) lo = mid;
          else hi = mid, reg_hi = c;
        }
        chi += reg_hi;
        __builtin_amdgcn_wave_barrier();  // the slots are rewritten by the next row
      }
      constexpr auto js = std::make_integer_sequence<int, J>{};
      if (cut != 0) {
        // exactly x magnitudes are >= cut > 0
        guess = cut;
        const float cf = pat(cut);
        pack_signed<J>([&](int j) { return vote(v[j] >= cf); }, [&](int j) { return vote(v[j] <= -cf); }, &plus,
                       &minus, js);
      } else {
        // t = lo and chi = count(|u| > t): the lowest-index x - chi
        // coordinates with |u| == t complete the set
        guess = lo;
        const float tf = pat(lo);
        const int need = x - chi;
        int eq_before = 0;
        pack_planes<J>(v, [&](int j) {
          const uint64_t eq = vote(valid(j) && fabsf(v[j]) == tf);
          const bool take = ((eq >> lane) & 1ull) && eq_before + lanes_below(eq) < need;
          eq_before += popc64(eq);
          return vote(fabsf(v[j]) > tf) | vote(take);
        }, &plus, &minus, js);
      }
    }
    // lane w < W holds v+ word w; lane w >= W takes v- word w - W
    const uint32_t mw = __shfl(minus, lane - W);
    if (lane < row_words) *out = lane < W ? plus : mw;
  }
}

// b1.58 quantisation (Sec. 4.3), per embedding: gamma = mean |u_i|, then
// v_i = clip(round(u_i / gamma), -1, 1) with ties to even, so v_i != 0 exactly
// when |u_i / gamma| > 1/2.  gamma is summed in double (each lane its
// coordinates in order, then a fixed shuffle tree; a sequential sum can
// differ in the last bit, which moves a decision only for a quotient within
// ~1e-16 of 1/2) and the quotient is formed in double; an all-zero row gives
// the zero vector.  One wave per row,
// packed with the same ballots as the EVP encoder.
template <int J, int JV>
__global__ __launch_bounds__(kEncodeBlock) void b158_kernel(const float *__restrict__ X, int64_t n, int d, int W,
                                                           uint32_t *__restrict__ codes, int *__restrict__ flags) {
  const int lane = threadIdx.x & 63;
  const int64_t waves_per_block = kEncodeBlock / 64;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * waves_per_block;
  const int row_words = 2 * W;
  for (int64_t row = static_cast<int64_t>(blockIdx.x) * waves_per_block + (threadIdx.x >> 6); row < n;
       row += nwaves) {
    const float *u = X + row * d + lane;
    float v[J];
    float top = 0.0f;  // largest magnitude; NaN if the row holds one
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      if (j < JV) v[j] = __builtin_nontemporal_load(u + 64 * j);
      else v[j] = j * 64 + lane < d ? __builtin_nontemporal_load(u + 64 * j) : 0.0f;
      top = __builtin_elementwise_maximum(top, fabsf(v[j]));
      s += fabs(static_cast<double>(v[j]));
    }
    uint32_t plus = 0, minus = 0;
    if (__any(!(top < __builtin_huge_valf()))) {
      if (lane == 0) atomicOr(flags, 1);
    } else {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
      const double gamma = s / static_cast<double>(d);
      // round(q) is non-zero exactly when |q| > 1/2 (a tie rounds to even 0);
      // q is the correctly rounded double quotient, as in a plain reference
      constexpr auto js = std::make_integer_sequence<int, J>{};
      pack_planes<J>(v, [&](int j) { return vote(gamma > 0.0 && fabs(static_cast<double>(v[j]) / gamma) > 0.5); },
                     &plus, &minus, js);
    }
    const uint32_t mw = __shfl(minus, lane - W);
    if (lane < row_words) codes[row * row_words + lane] = lane < W ? plus : mw;
  }
}

template <int J, int JV>
hipError_t launch_b(const float *X, int64_t n, int d, uint32_t *codes, int *flags, int num_cu, hipStream_t s) {
  int64_t blocks = (n + 3) / 4;
  const int64_t cap = static_cast<int64_t>(num_cu > 0 ? num_cu : 256) * 8;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((b158_kernel<J, JV>), dim3(static_cast<unsigned>(blocks)), dim3(kEncodeBlock), 0, s, X, n, d,
                     (d + 31) / 32, codes, flags);
  return hipGetLastError();
}

template <int J, int JV>
hipError_t launch_j(const float *X, int64_t n, int d, int x, uint32_t *codes, int *flags, int num_cu,
                    hipStream_t s) {
  int64_t blocks = (n + 3) / 4;  // one wave per row, four waves per block
  const int64_t cap = static_cast<int64_t>(num_cu > 0 ? num_cu : 256) * 8;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL((encode_kernel<J, JV>), dim3(static_cast<unsigned>(blocks)), dim3(kEncodeBlock), 0, s, X,
                     n, d, x, (d + 31) / 32, codes, flags);
  return hipGetLastError();
}

}  // namespace

hipError_t encode_launch(const float *X, int64_t n, int d, int x, uint32_t *codes, int *flags,
                         int num_cu, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int j = (d + 63) / 64;
  // whole registers, no ragged tail: d = 384, 512, 768, 1024
  if (d == 64 * 6) return launch_j<6, 6>(X, n, d, x, codes, flags, num_cu, s);
  if (d == 64 * 8) return launch_j<8, 8>(X, n, d, x, codes, flags, num_cu, s);
  if (d == 64 * 12) return launch_j<12, 12>(X, n, d, x, codes, flags, num_cu, s);
  if (d == 64 * 16) return launch_j<16, 16>(X, n, d, x, codes, flags, num_cu, s);
  if (j <= 1) return launch_j<1, 0>(X, n, d, x, codes, flags, num_cu, s);
  if (j <= 2) return launch_j<2, 1>(X, n, d, x, codes, flags, num_cu, s);
  if (j <= 4) return launch_j<4, 2>(X, n, d, x, codes, flags, num_cu, s);
  if (j <= 6) return launch_j<6, 4>(X, n, d, x, codes, flags, num_cu, s);
  if (j <= 8) return launch_j<8, 6>(X, n, d, x, codes, flags, num_cu, s);
  if (j <= 12) return launch_j<12, 8>(X, n, d, x, codes, flags, num_cu, s);
  return launch_j<16, 12>(X, n, d, x, codes, flags, num_cu, s);
}

hipError_t b158_launch(const float *X, int64_t n, int d, uint32_t *codes, int *flags, int num_cu, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int j = (d + 63) / 64;
  if (j <= 1) return launch_b<1, 0>(X, n, d, codes, flags, num_cu, s);
  if (j <= 2) return launch_b<2, 1>(X, n, d, codes, flags, num_cu, s);
  if (j <= 4) return launch_b<4, 2>(X, n, d, codes, flags, num_cu, s);
  if (j <= 6) return launch_b<6, 4>(X, n, d, codes, flags, num_cu, s);
  if (j <= 8) return launch_b<8, 6>(X, n, d, codes, flags, num_cu, s);
  if (j <= 12) return launch_b<12, 8>(X, n, d, codes, flags, num_cu, s);
  return launch_b<16, 12>(X, n, d, codes, flags, num_cu, s);
}

}  // namespace tqi
