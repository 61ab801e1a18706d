// Batches of independent instances advanced by one persistent launch: the
// device table the kernels read and the work-queue helpers.
#pragma once

#include "device.h"

namespace shgb {

// One instance of a batch (device form).  Its beams are cut into tiles of
// one workgroup's worth; tile0 is the global index of its first tile.
struct BatchItem {
  DevModel md;
  void *tr;          // trajectory block (double* or float*, by the batch precision)
  double *sc;        // scalar block
  int32_t *comp;
  uint32_t *nhop;
  int64_t n, ld;
  uint64_t gid0, seed;
  int64_t tile0, tiles;
};

// The instance that owns global tile t (items sorted by tile0, t < total).
__device__ inline int batch_find(const BatchItem *__restrict__ items, int n_items, int64_t t) {
  int lo = 0, hi = n_items - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].tile0 <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Next grab of the block's work queue, the same value in every lane (and an
// SGPR): thread 0 takes `count` tiles, LDS broadcasts.
__device__ inline int64_t batch_grab(unsigned long long *queue, int count) {
  __shared__ unsigned long long grab;
  if (threadIdx.x == 0) grab = atomicAdd(queue, (unsigned long long)count);
  __syncthreads();
  const unsigned long long g = grab;
  __syncthreads();
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)g), hi = __builtin_amdgcn_readfirstlane((uint32_t)(g >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

}  // namespace shgb
