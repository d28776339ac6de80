// rerank.hip -- refinement of proxy candidates with the original vectors.
//
// The k@n recall of Sec. 5.3 measures how many true nearest neighbours are
// among a query's n nearest in the proxy space; the search it stands for
// orders those n candidates by the original similarity and keeps k.  For
// l2-normalised embeddings (Sec. 1.1) the nearest in l2 are the largest
// scalar products, so each candidate is scored with the scalar product of the
// float vectors, products and sums in double precision, and the k best are
// kept (larger first; the lower id on equal scores).
//
// One workgroup of eight waves per query (so that even a hundred queries
// keep most SIMDs busy).  The candidate ids are first staged in LDS with one
// coalesced read; each lane holds the query coordinates l, l + 64, ...; a
// wave scores four candidates at a time (the four rows' loads in flight
// together, each row read as coalesced 256-byte runs), reduces each across
// the wave, and parks (score, id) in LDS; a bitonic sort over the padded
// candidate list then puts the best first.  Gather-bound: every candidate row
// is read once (4d bytes).
#include "tq_internal.h"

namespace tqi {
namespace {

constexpr int kRerankWaves = 8;
constexpr int kRerankBlock = 64 * kRerankWaves;
constexpr int kRerankBatch = 4;  // candidates in flight per wave

__device__ __forceinline__ bool refined_before(double sa, int32_t ia, double sb, int32_t ib) {
  return sa > sb || (sa == sb && ia < ib);
}

template <int J>
__global__ __launch_bounds__(kRerankBlock) void rerank_kernel(const float *__restrict__ X, int64_t n, int d,
                                                             const float *__restrict__ Q,
                                                             const int32_t *__restrict__ cand, int ncand, int P,
                                                             int k, int32_t *__restrict__ ids,
                                                             double *__restrict__ scores) {
  __shared__ double sc[kMaxRerank];
  __shared__ int32_t sid[kMaxRerank];
  const int64_t q = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  float qv[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int i = j * 64 + lane;
    qv[j] = i < d ? Q[q * d + i] : 0.0f;
  }
  const int32_t *cq = cand + q * ncand;
  for (int c = threadIdx.x; c < P; c += kRerankBlock) {
    const int32_t id = c < ncand ? cq[c] : -1;
    sid[c] = (id < 0 || id >= n) ? -1 : id;
  }
  __syncthreads();
  for (int c0 = wave * kRerankBatch; c0 < P; c0 += kRerankWaves * kRerankBatch) {
    int32_t cid[kRerankBatch];
    float xv[kRerankBatch][J];
#pragma unroll
    for (int b = 0; b < kRerankBatch; ++b) {
      const int id = sid[c0 + b];
      cid[b] = id;
      const float *xr = X + static_cast<int64_t>(id < 0 ? 0 : id) * d;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int i = j * 64 + lane;
        xv[b][j] = (id >= 0 && i < d) ? xr[i] : 0.0f;
      }
    }
#pragma unroll
    for (int b = 0; b < kRerankBatch; ++b) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < J; ++j) acc = fma(static_cast<double>(qv[j]), static_cast<double>(xv[b][j]), acc);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      if (lane == 0) {
        sc[c0 + b] = cid[b] >= 0 ? acc : -__builtin_huge_val();
        sid[c0 + b] = cid[b] >= 0 ? cid[b] : INT32_MAX;
      }
    }
  }
  __syncthreads();
  // bitonic sort of the P (a power of two) entries, best first
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P / 2; t += kRerankBlock) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool best_first = (lo & size) == 0;
        const double sl = sc[lo], sh = sc[hi];
        const int32_t il = sid[lo], ih = sid[hi];
        const bool swap = best_first ? refined_before(sh, ih, sl, il) : refined_before(sl, il, sh, ih);
        if (swap) {
          sc[lo] = sh;
          sc[hi] = sl;
          sid[lo] = ih;
          sid[hi] = il;
        }
      }
      __syncthreads();
    }
  }
  for (int p = threadIdx.x; p < k; p += kRerankBlock) {
    const bool ok = sid[p] != INT32_MAX;
    ids[q * k + p] = ok ? sid[p] : -1;
    scores[q * k + p] = ok ? sc[p] : -__builtin_huge_val();
  }
}

template <int J>
hipError_t launch_r(const float *X, int64_t n, int d, const float *Q, int nq, const int32_t *cand, int ncand,
                    int k, int32_t *ids, double *scores, hipStream_t s) {
  int P = kRerankBatch;  // a power of two covering the candidates, whole batches
  while (P < ncand) P <<= 1;
  hipLaunchKernelGGL((rerank_kernel<J>), dim3(static_cast<unsigned>(nq)), dim3(kRerankBlock), 0, s, X, n, d, Q,
                     cand, ncand, P, k, ids, scores);
  return hipGetLastError();
}

}  // namespace

hipError_t rerank_launch(const float *X, int64_t n, int d, const float *Q, int nq, const int32_t *cand, int ncand,
                         int k, int32_t *ids, double *scores, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  const int j = (d + 63) / 64;
  if (j <= 2) return launch_r<2>(X, n, d, Q, nq, cand, ncand, k, ids, scores, s);
  if (j <= 4) return launch_r<4>(X, n, d, Q, nq, cand, ncand, k, ids, scores, s);
  if (j <= 8) return launch_r<8>(X, n, d, Q, nq, cand, ncand, k, ids, scores, s);
  if (j <= 12) return launch_r<12>(X, n, d, Q, nq, cand, ncand, k, ids, scores, s);
  return launch_r<16>(X, n, d, Q, nq, cand, ncand, k, ids, scores, s);
}

}  // namespace tqi
