// reduce.h — deterministic per-cell reductions across the blocks of a launch.
//
// Two-pass scheme: every block of a cell reduces its values (wavefront
// shuffle tree, then the four wavefront results in fixed order) and stores
// them in the cell's partial buffer (column-major: value j of block b at
// j * nblk + b, so the finaliser's reads are coalesced); a finalising kernel
// (one block per cell and column, launched next on the same stream) sums the
// partials in block order.
// The kernel boundary makes the partials visible to the finaliser without
// any in-kernel fence (on this chip an agent-scope release fence writes back
// the XCD's L2), and the fixed summation order makes the result independent
// of block scheduling: the same cell gives bit-identical sums alone or
// inside a batch.
#pragma once
#include "mbx_dev.h"

namespace mbx {

// Block-wide reduction of value j (sum, or max when mx): every thread passes
// its value; the wave result goes to lds[wave * stride + j].  After a
// __syncthreads the caller combines the four wave slots with combine4.
__device__ inline void wave_to_lds(double v, bool mx, double* lds, int stride, int j) {
  v = mx ? wave_max(v) : wave_sum(v);
  if ((threadIdx.x & 63) == 0) lds[(threadIdx.x >> 6) * stride + j] = v;
}
__device__ inline double combine4(const double* lds, int stride, int j, bool mx) {
  const double a = lds[j], b = lds[stride + j], c = lds[2 * stride + j], d = lds[3 * stride + j];
  return mx ? fmax(fmax(a, b), fmax(c, d)) : (a + b) + (c + d);
}

// First pass: K values per thread; bit j of maxmask selects max (else sum);
// the block result goes to the cell's partial row `blk`.
template <int K>
__device__ inline void reduce_block(const CellDev& cd, int blk, const double (&v)[K], unsigned maxmask) {
  __shared__ double lds[4 * K];
#pragma unroll
  for (int j = 0; j < K; ++j) wave_to_lds(v[j], (maxmask >> j) & 1u, lds, K, j);
  __syncthreads();
  if (threadIdx.x < K)
    cd.part[(size_t)threadIdx.x * cd.nblk + blk] = combine4(lds, K, threadIdx.x, (maxmask >> threadIdx.x) & 1u);
}

// Second pass (inside a one-block-per-cell kernel): column j of the partial
// rows summed (or max-reduced) in block order; result valid in all threads.
__device__ inline double finalize_column(const CellDev& cd, int j, bool mx, double* lds4, double* result) {
  // each thread combines blocks t, t + kBlock, t + 2 kBlock, ... in that
  // order; the loads are issued sixteen at a time so that they are in flight
  // together (the additions keep their order: the same bits as one at a time)
  constexpr int kU = 16;
  const double* col = cd.part + (size_t)j * cd.nblk;
  double acc = 0.0;
  int b = threadIdx.x;
  for (; b + (kU - 1) * kBlock < cd.nblk; b += kU * kBlock) {
    double p[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) p[u] = col[b + u * kBlock];
#pragma unroll
    for (int u = 0; u < kU; ++u) acc = mx ? fmax(acc, p[u]) : acc + p[u];
  }
  for (; b < cd.nblk; b += kBlock) {
    const double p = col[b];
    acc = mx ? fmax(acc, p) : acc + p;
  }
  __syncthreads();
  wave_to_lds(acc, mx, lds4, 1, 0);
  __syncthreads();
  if (threadIdx.x == 0) *result = combine4(lds4, 1, 0, mx);
  __syncthreads();
  return *result;
}

}  // namespace mbx
