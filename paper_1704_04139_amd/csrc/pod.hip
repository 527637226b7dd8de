// pod.hip — kernels of the POD of a snapshot set by the method of snapshots
// (Sec. 2.5): the Gram matrix K = S^T W S on the FP64 matrix cores and the
// modes U = S C of the kept eigenvectors.
//
// Snapshots S are n x m, column-major with leading dimension lds (one column
// per snapshot, as the state of a cell is stored).  K is a tall-skinny
// symmetric product: workgroups own one 64x64 tile of its upper triangle and
// one slice of the rows, and a second kernel sums the slices in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mbx_kernels.h"

namespace mbx {
namespace {

constexpr int kGT = 64;        // edge of a Gram tile
constexpr int kGK = 32;        // snapshot rows staged in LDS per step
constexpr int kGThreads = 256; // 4 wavefronts, each owns a 32x32 quarter of the tile
constexpr int kMQ = 32;        // modes computed per thread (one row, kMQ columns)

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Partial Gram tile of tile pair p = (ti, tj), ti <= tj, over the rows
// [y R, min(n, (y+1) R)).  Each wave accumulates 2x2 blocks of 16x16 with
// v_mfma_f64_16x16x4: A (16x4) is the weighted slice W S[:, ti-tile]
// transposed, B (4x16) the slice S[:, tj-tile].  Lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; it receives D[l/16 + 4r][l%16], r = 0..3
// (rows interleaved across the four lane groups).
__global__ void __launch_bounds__(kGThreads)
    k_gram(const double* __restrict__ S, int64_t n, int m, int64_t lds, const double* __restrict__ w, int64_t R,
           const int2* __restrict__ pairs, int npairs, double* __restrict__ part) {
  // one pad column: the 32 rows written by consecutive threads spread over all banks
  __shared__ double As[kGK][kGT + 1];
  __shared__ double Bs[kGK][kGT + 1];
  constexpr int kPer = (kGK * kGT) / kGThreads;   // staged values per thread and tile
  const int p = blockIdx.x;
  const int y = blockIdx.y;
  const int2 tt = pairs[p];
  const int ci = tt.x * kGT, cj = tt.y * kGT;
  const int t = threadIdx.x;
  const int wv = t >> 6, l = t & 63;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;   // the wave's quarter of the tile
  const int li = l & 15, lk = l >> 4;
  // 16x16 blocks that hold no needed entry are skipped (uniform per wave):
  // columns past m, and on a diagonal tile the blocks below the diagonal
  bool live[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const int r0b = wr + a * 16, c0b = wc + b * 16;
      live[a][b] = ci + r0b < m && cj + c0b < m && !(tt.x == tt.y && r0b > c0b + 15);
    }
  dbl4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
  const int64_t r_begin = (int64_t)y * R;
  const int64_t r_end = r_begin + R < n ? r_begin + R : n;
  // 32 consecutive threads read 32 consecutive rows of one column (256
  // contiguous bytes); the next chunk is fetched into registers while the
  // matrix cores work on the current one
  double pa[kPer], pb[kPer];
  auto fetch = [&](int64_t r0) {
    for (int q = 0; q < kPer; ++q) {
      const int e = q * kGThreads + t;
      const int row = e % kGK, col = e / kGK;
      const int64_t rg = r0 + row;
      double va = 0.0, vb = 0.0;
      if (rg < r_end) {
        const double wt = w ? w[rg] : 1.0;
        if (ci + col < m) va = wt * S[rg + (int64_t)(ci + col) * lds];
        if (cj + col < m) vb = S[rg + (int64_t)(cj + col) * lds];
      }
      pa[q] = va;
      pb[q] = vb;
    }
  };
  if (r_begin < r_end) fetch(r_begin);
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kGK) {
    for (int q = 0; q < kPer; ++q) {
      const int e = q * kGThreads + t;
      As[e % kGK][e / kGK] = pa[q];
      Bs[e % kGK][e / kGK] = pb[q];
    }
    __syncthreads();
    if (r0 + kGK < r_end) fetch(r0 + kGK);
    for (int kk = 0; kk < kGK; kk += 4) {
      const double a0 = As[kk + lk][wr + li];
      const double a1 = As[kk + lk][wr + 16 + li];
      const double b0 = Bs[kk + lk][wc + li];
      const double b1 = Bs[kk + lk][wc + 16 + li];
      if (live[0][0]) acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      if (live[0][1]) acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      if (live[1][0]) acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      if (live[1][1]) acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  double* out = part + ((int64_t)y * npairs + p) * (kGT * kGT);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        const int i = wr + a * 16 + lk + 4 * r;
        const int j = wc + b * 16 + li;
        out[i * kGT + j] = acc[a][b][r];
      }
}

// K from the partial tiles: the slices are summed in slice order, and each
// entry of the upper triangle is written to both (i, j) and (j, i), so K is
// exactly symmetric.
__global__ void __launch_bounds__(256)
    k_gram_reduce(const double* __restrict__ part, int nsplit, const int2* __restrict__ pairs, int npairs, int m,
                  double* __restrict__ K) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)npairs * kGT * kGT) return;
  const int p = (int)(e / (kGT * kGT));
  const int loc = (int)(e % (kGT * kGT));
  const int i = loc / kGT, j = loc % kGT;
  const int2 tt = pairs[p];
  const int gi = tt.x * kGT + i, gj = tt.y * kGT + j;
  if (gi >= m || gj >= m || gi > gj) return;
  double s = 0.0;
  for (int y = 0; y < nsplit; ++y) s += part[((int64_t)y * npairs + p) * (kGT * kGT) + loc];
  K[gi + (int64_t)gj * m] = s;
  K[gj + (int64_t)gi * m] = s;
}

// Modes U[:, q] = S C[:, q]: one thread per snapshot row and kMQ columns of
// C, whose entries all lanes share (C row-major, kpad columns).
__global__ void __launch_bounds__(256)
    k_modes(const double* __restrict__ S, int64_t n, int m, int64_t lds, const double* __restrict__ C, int kpad,
            int k, double* __restrict__ U, int64_t ldu) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q0 = blockIdx.y * kMQ;
  if (i >= n) return;
  double acc[kMQ];
  for (int q = 0; q < kMQ; ++q) acc[q] = 0.0;
  for (int j = 0; j < m; ++j) {
    const double s = S[i + (int64_t)j * lds];
    const double* c = C + (int64_t)j * kpad + q0;
    for (int q = 0; q < kMQ; ++q) acc[q] = fma(s, c[q], acc[q]);
  }
  for (int q = 0; q < kMQ && q0 + q < k; ++q) U[i + (int64_t)(q0 + q) * ldu] = acc[q];
}

}  // namespace

int gram_tile() { return kGT; }
int gram_rows_step() { return kGK; }
int modes_cols_per_thread() { return kMQ; }

void launch_gram(const double* S, int64_t n, int m, int64_t lds, const double* w, int64_t rows_per_split, int nsplit,
                 const int2* pairs, int npairs, double* part, hipStream_t s) {
  k_gram<<<dim3(npairs, nsplit), kGThreads, 0, s>>>(S, n, m, lds, w, rows_per_split, pairs, npairs, part);
}

void launch_gram_reduce(const double* part, int nsplit, const int2* pairs, int npairs, int m, double* K, hipStream_t s) {
  const int64_t tot = (int64_t)npairs * kGT * kGT;
  k_gram_reduce<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(part, nsplit, pairs, npairs, m, K);
}

void launch_modes(const double* S, int64_t n, int m, int64_t lds, const double* C, int kpad, int k, double* U,
                  int64_t ldu, hipStream_t s) {
  k_modes<<<dim3((unsigned)((n + 255) / 256), (unsigned)(kpad / kMQ)), 256, 0, s>>>(S, n, m, lds, C, kpad, k, U,
                                                                                    ldu);
}

}  // namespace mbx
