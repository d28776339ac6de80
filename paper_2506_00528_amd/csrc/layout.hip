// layout.hip -- moving codes between the canonical layout of the public ABI
// ([v+ : W words][v- : W words] per row) and the resident tiled layout of the
// database (see tq_internal.h), and checking canonical codes.
#include "tq_internal.h"

namespace tqi {
namespace {

// One thread per (tile, chunk, lane): reads 4 words of each plane of one
// vector and writes one 16-byte chunk of the nz plane and of the ng plane.
__global__ __launch_bounds__(256) void repack_kernel(const uint32_t *__restrict__ codes, int64_t n, int W,
                                                     int nc, int64_t ntiles, uint4 *__restrict__ tiles) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= ntiles * nc * 64) return;
  const int lane = static_cast<int>(g & 63);
  const int64_t tc = g >> 6;
  const int c = static_cast<int>(tc % nc);
  const int64_t t = tc / nc;
  const int64_t v = t * 64 + lane;
  uint32_t p[4] = {0, 0, 0, 0}, m[4] = {0, 0, 0, 0};
  if (v < n) {
    const uint32_t *row = codes + v * 2 * W;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int w = 4 * c + e;
      if (w < W) {
        p[e] = row[w];
        m[e] = row[W + w];
      }
    }
  }
  tiles[((t * 2 + 0) * nc + c) * 64 + lane] = make_uint4(p[0] | m[0], p[1] | m[1], p[2] | m[2], p[3] | m[3]);
  tiles[((t * 2 + 1) * nc + c) * 64 + lane] = make_uint4(m[0], m[1], m[2], m[3]);
}

// One thread per (vector, plane word): v+ = nz & ~ng, v- = ng.
__global__ __launch_bounds__(256) void export_kernel(const uint4 *__restrict__ tiles, int64_t n, int W, int nc,
                                                     uint32_t *__restrict__ codes) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= n * W) return;
  const int64_t v = g / W;
  const int w = static_cast<int>(g - v * W);
  const int64_t t = v >> 6;
  const int lane = static_cast<int>(v & 63);
  const int c = w >> 2, e = w & 3;
  const uint32_t *nz = reinterpret_cast<const uint32_t *>(tiles + ((t * 2 + 0) * nc + c) * 64 + lane);
  const uint32_t *ng = reinterpret_cast<const uint32_t *>(tiles + ((t * 2 + 1) * nc + c) * 64 + lane);
  codes[v * 2 * W + w] = nz[e] & ~ng[e];
  codes[v * 2 * W + W + w] = ng[e];
}

// One thread per row: exactly x non-zeros, disjoint planes, zero padding.
__global__ __launch_bounds__(256) void validate_kernel(const uint32_t *__restrict__ codes, int64_t n, int d,
                                                       int W, int x, unsigned long long *__restrict__ bad) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  unsigned long long nbad = 0;
  const uint32_t pad = (d & 31) ? ~((1u << (d & 31)) - 1u) : 0u;
  for (int64_t r = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; r < n; r += stride) {
    const uint32_t *row = codes + r * 2 * W;
    int cnt = 0;
    bool ok = true;
    for (int w = 0; w < W; ++w) {
      const uint32_t p = row[w], m = row[W + w];
      ok = ok && (p & m) == 0;
      cnt += __popc(p) + __popc(m);
    }
    ok = ok && ((row[W - 1] | row[2 * W - 1]) & pad) == 0 && (x == 0 || cnt == x);
    nbad += ok ? 0 : 1;
  }
  if (nbad) atomicAdd(bad, nbad);
}

inline unsigned blocks_for(int64_t threads, int per_block) {
  return static_cast<unsigned>((threads + per_block - 1) / per_block);
}

}  // namespace

hipError_t repack_launch(const uint32_t *codes, int64_t n, int d, uint4 *tiles, int64_t ntiles, int nc,
                         hipStream_t s) {
  const int64_t threads = ntiles * nc * 64;
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(repack_kernel, dim3(blocks_for(threads, 256)), dim3(256), 0, s, codes, n, (d + 31) / 32,
                     nc, ntiles, tiles);
  return hipGetLastError();
}

hipError_t export_launch(const DbDev &db, uint32_t *codes, hipStream_t s) {
  const int64_t threads = db.n * db.W;
  if (threads == 0) return hipSuccess;
  hipLaunchKernelGGL(export_kernel, dim3(blocks_for(threads, 256)), dim3(256), 0, s, db.tiles, db.n, db.W,
                     db.nc, codes);
  return hipGetLastError();
}

hipError_t validate_launch(const uint32_t *codes, int64_t n, int d, int x, unsigned long long *bad_rows,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(validate_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, codes, n, d,
                     (d + 31) / 32, x, bad_rows);
  return hipGetLastError();
}

}  // namespace tqi
