// tq_batched.h -- internals of the batched search path shared by its kernels
// (batched_kernels.hip, scan.hip's merge) and its host runtime (batched.cpp).
#pragma once

#include "tq_internal.h"

namespace tqi {

// Per-call values of a batched search, written on the device by
// batch_prep_kernel so that the scan and merge launches keep fixed arguments
// (and can be replayed from a captured hipGraph).
struct BatchParams {
  int nq;                  // real queries of the call (<= bucket)
  int nqt;                 // query tiles: ceil(nq / qtile)
  int parts;               // database parts: the grid gets nqt * parts work items
  int pad;
  int64_t tiles_per_part;  // 64-vector tiles per part
  int32_t *ids;            // caller's outputs, nq x k
  int32_t *scores;
};

// Largest query tile the batched scan supports for this k.
int batched_max_qtile(int k);

hipError_t batch_prep_launch(const uint32_t *qcodes, int nq, int bucket, const DbDev &db, int qtile, int grid,
                             int32_t *ids, int32_t *scores, uint32_t *qprep, BatchParams *prm, hipStream_t s);
hipError_t scan_batched_launch(const DbDev &db, const uint32_t *qprep, const BatchParams *prm, int k, int qtile,
                               int grid, uint64_t *partial, hipStream_t s);
// Per-query merge of the (query, part) lists; the query count, part count and
// output pointers come from `prm`; `bucket` workgroups are launched.
hipError_t merge_batched_launch(const uint64_t *partial, const BatchParams *prm, int bucket, int k,
                                hipStream_t s);

}  // namespace tqi
