// reduce.h — deterministic per-cell reductions across the blocks of a launch.
//
// Every block of a cell reduces its values (fixed shuffle tree), stores the
// block result in the cell's partial buffer and takes a ticket; the block
// that takes the last ticket sums the partials in block order and writes
// the result.  The result therefore does not depend on block scheduling, and
// the same cell gives bit-identical sums alone or inside a batch.
#pragma once
#include "mbx_dev.h"

namespace mbx {

__device__ inline void part_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double part_load(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Take the ticket after this block's partials are stored; returns true in
// every thread of the block that completes the cell.
__device__ inline bool take_ticket(CellDev* cd, bool* lds_flag) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned t = __hip_atomic_fetch_add(cd->ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    *lds_flag = (t == (unsigned)(cd->nblk - 1));
  }
  __syncthreads();
  const bool last = *lds_flag;
  if (last) __threadfence();
  return last;
}

__device__ inline void release_ticket(CellDev* cd) {
  if (threadIdx.x == 0) __hip_atomic_store(cd->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// K values per thread; bit j of maxmask selects max (else sum).  Outputs go
// to out[j] (written by the completing block).
template <int K>
__device__ inline void reduce_cell(CellDev* cd, int blk, const double (&v)[K], unsigned maxmask,
                                   double* out) {
  __shared__ double lds4[4];
  __shared__ bool flag;
  double r[K];
#pragma unroll
  for (int j = 0; j < K; ++j)
    r[j] = ((maxmask >> j) & 1u) ? block_max(v[j], lds4) : block_sum(v[j], lds4);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < K; ++j) part_store(&cd->part[(size_t)blk * kPartStride + j], r[j]);
  }
  if (!take_ticket(cd, &flag)) return;
  const int nb = cd->nblk;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const bool mx = (maxmask >> j) & 1u;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) {
      const double p = part_load(&cd->part[(size_t)b * kPartStride + j]);
      acc = mx ? fmax(acc, p) : acc + p;
    }
    acc = mx ? block_max(acc, lds4) : block_sum(acc, lds4);
    if (threadIdx.x == 0) out[j] = acc;
  }
  release_ticket(cd);
}

}  // namespace mbx
