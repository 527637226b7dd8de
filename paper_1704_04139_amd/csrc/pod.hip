// pod.hip — kernels of the POD of a snapshot set by the method of snapshots
// (Sec. 2.5): the Gram matrix K = S^T W S on the FP64 matrix cores and the
// modes U = S C of the kept eigenvectors.
//
// Snapshots S are n x m, column-major with leading dimension lds (one column
// per snapshot, as the state of a cell is stored).  K is a tall-skinny
// symmetric product: workgroups own one 32x32 tile of its upper triangle and
// one slice of the rows, and a second kernel sums the slices in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mbx_kernels.h"

namespace mbx {
namespace {

constexpr int kGT = 32;        // edge of a Gram tile
constexpr int kGK = 64;        // snapshot rows staged in LDS per step
constexpr int kGThreads = 256; // 4 wavefronts, each owns a 16x16 quarter of the tile
constexpr int kMQ = 32;        // modes computed per thread (one row, kMQ columns)
constexpr int kRGroups = 16;   // wavefronts that share the slices of one reduction block

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Partial Gram tile of tile pair p = (ti, tj), ti <= tj, over the rows
// [y R, min(n, (y+1) R)).  Each wave accumulates one 16x16 block with
// v_mfma_f64_16x16x4: A (16x4) is the weighted slice W S[:, ti-tile]
// transposed, B (4x16) the slice S[:, tj-tile].  Lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; it receives D[l/16 + 4r][l%16], r = 0..3
// (rows interleaved across the four lane groups).  32-column tiles with 64
// rows per stage: each column is read in 512-byte pieces, and padding past m
// costs less than with wider tiles.
// The weights (kW) are staged per row in LDS and applied to the A operand, so
// that the snapshot loads carry no dependence on them: with the weight folded
// into the fetch, the compiler waits on each load before the next.
template <bool kW>
__global__ void __launch_bounds__(kGThreads)
    k_gram(const double* __restrict__ S, int64_t n, int m, int64_t lds, const double* __restrict__ w, int64_t R,
           const int2* __restrict__ pairs, int npairs, double* __restrict__ part) {
  // one pad column: the rows written by consecutive threads spread over the banks
  __shared__ double As[kGK][kGT + 1];
  __shared__ double Bs[kGK][kGT + 1];
  __shared__ double Ws[kGK];
  constexpr int kPer = (kGK * kGT) / kGThreads;   // staged values per thread and tile
  const int p = blockIdx.x;
  const int y = blockIdx.y;
  const int2 tt = pairs[p];
  const int ci = tt.x * kGT, cj = tt.y * kGT;
  const int t = threadIdx.x;
  const int wv = t >> 6, l = t & 63;
  const int wr = (wv >> 1) * 16, wc = (wv & 1) * 16;   // the wave's block of the tile
  const int li = l & 15, lk = l >> 4;
  // a block that holds no needed entry is skipped (uniform per wave): columns
  // past m, and on a diagonal tile the block below the diagonal
  const bool live = ci + wr < m && cj + wc < m && !(tt.x == tt.y && wr > wc);
  dbl4 acc = {0.0, 0.0, 0.0, 0.0};
  const int64_t r_begin = (int64_t)y * R;
  const int64_t r_end = r_begin + R < n ? r_begin + R : n;
  // kGK consecutive threads read kGK consecutive rows of one column; the next
  // stage is fetched into registers while the matrix cores work on this one
  double pa[kPer], pb[kPer], pw = 0.0;
  auto fetch = [&](int64_t r0) {
    for (int q = 0; q < kPer; ++q) {
      const int e = q * kGThreads + t;
      const int row = e % kGK, col = e / kGK;
      const int64_t rg = r0 + row;
      double va = 0.0, vb = 0.0;
      if (rg < r_end) {
        if (ci + col < m) va = S[rg + (int64_t)(ci + col) * lds];
        if (cj + col < m) vb = S[rg + (int64_t)(cj + col) * lds];
      }
      pa[q] = va;
      pb[q] = vb;
    }
    if (kW && t < kGK) pw = r0 + t < r_end ? w[r0 + t] : 0.0;
  };
  if (r_begin < r_end) fetch(r_begin);
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kGK) {
    for (int q = 0; q < kPer; ++q) {
      const int e = q * kGThreads + t;
      As[e % kGK][e / kGK] = pa[q];
      Bs[e % kGK][e / kGK] = pb[q];
    }
    if (kW && t < kGK) Ws[t] = pw;
    __syncthreads();
    if (r0 + kGK < r_end) fetch(r0 + kGK);
    if (live)
      for (int kk = 0; kk < kGK; kk += 4) {
        double a = As[kk + lk][wr + li];
        if (kW) a *= Ws[kk + lk];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[kk + lk][wc + li], acc, 0, 0, 0);
      }
    __syncthreads();
  }
  double* out = part + ((int64_t)y * npairs + p) * (kGT * kGT);
  for (int r = 0; r < 4; ++r) out[(wr + lk + 4 * r) * kGT + wc + li] = acc[r];
}

// The same partial tiles when the whole snapshot set is at most kGAllCols
// columns wide: one workgroup per row slice stages each row chunk of all m
// columns in LDS once (two buffers: the next chunk is stored while the
// current one is consumed, one barrier per chunk) and computes every tile
// pair from it, so each snapshot entry is fetched once (the pair-per-workgroup
// kernel above fetches a column tile once for every pair that holds it).
// Wavefront v takes the NU 16x16 blocks u = v, v + 8, ... (tile pair u / 4,
// quarter u % 4), every one of them in the multiply loop (no branches there:
// blocks below the diagonal or past m read staged columns and write zeros).
// Each block is accumulated over the rows in the same order as above, so the
// reduction reads the same partial layout.
constexpr int kGAllCols = 128;                              // widest set staged whole (4 tiles, 10 pairs)
constexpr int kGAllThreads = 512;                           // 8 wavefronts
constexpr int kGAllPer = (kGK * kGAllCols) / kGAllThreads;  // staged values per thread at most

template <bool kW, int NU>
__global__ void __launch_bounds__(kGAllThreads)
    k_gram_all(const double* __restrict__ S, int64_t n, int m, int64_t lds, const double* __restrict__ w, int64_t R,
               const int2* __restrict__ pairs, int npairs, double* __restrict__ part) {
  __shared__ double Ss[2][kGK][kGAllCols + 1];
  __shared__ double Ws[2][kGK];
  const int y = blockIdx.x;
  const int t = threadIdx.x;
  const int wv = t >> 6, l = t & 63;
  const int li = l & 15, lk = l >> 4;
  const int mp = (m + kGT - 1) / kGT * kGT;   // staged columns: whole tiles
  const int nst = kGK * mp;                   // staged values per chunk
  int ca[NU], cb[NU];
  bool live[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int b = wv + 8 * u, pp = b >> 2, q = b & 3;
    const int wr = (q >> 1) * 16, wc = (q & 1) * 16;
    const int2 tt = pp < npairs ? pairs[pp] : make_int2(0, 0);
    ca[u] = tt.x * kGT + wr + li;
    cb[u] = tt.y * kGT + wc + li;
    live[u] = pp < npairs && tt.x * kGT + wr < m && tt.y * kGT + wc < m && !(tt.x == tt.y && wr > wc);
  }
  dbl4 acc[NU];
#pragma unroll
  for (int u = 0; u < NU; ++u) acc[u] = dbl4{0.0, 0.0, 0.0, 0.0};
  const int64_t r_begin = (int64_t)y * R;
  const int64_t r_end = r_begin + R < n ? r_begin + R : n;
  double pv[kGAllPer], pw = 0.0;
  auto fetch = [&](int64_t r0) {
#pragma unroll
    for (int q = 0; q < kGAllPer; ++q) {
      const int e = q * kGAllThreads + t;
      const int row = e % kGK, col = e / kGK;
      const int64_t rg = r0 + row;
      pv[q] = (e < nst && rg < r_end && col < m) ? S[rg + (int64_t)col * lds] : 0.0;
    }
    if (kW && t < kGK) pw = r0 + t < r_end ? w[r0 + t] : 0.0;
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int q = 0; q < kGAllPer; ++q) {
      const int e = q * kGAllThreads + t;
      if (e < nst) Ss[buf][e % kGK][e / kGK] = pv[q];
    }
    if (kW && t < kGK) Ws[buf][t] = pw;
  };
  if (r_begin < r_end) {
    fetch(r_begin);
    stage(0);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t r0 = r_begin; r0 < r_end; r0 += kGK, cur ^= 1) {
    const bool more = r0 + kGK < r_end;
    if (more) fetch(r0 + kGK);
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 4)
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        double a = Ss[cur][kk + lk][ca[u]];
        if (kW) a *= Ws[cur][kk + lk];
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Ss[cur][kk + lk][cb[u]], acc[u], 0, 0, 0);
      }
    if (more) stage(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < NU; ++u) {
    const int b = wv + 8 * u, pp = b >> 2, q = b & 3;
    if (pp >= npairs) break;
    const int wr = (q >> 1) * 16, wc = (q & 1) * 16;
    double* out = part + ((int64_t)y * npairs + pp) * (kGT * kGT);
    for (int r = 0; r < 4; ++r) out[(wr + lk + 4 * r) * kGT + wc + li] = live[u] ? acc[u][r] : 0.0;
  }
}

template <bool kW>
void launch_gram_all(const double* S, int64_t n, int m, int64_t lds, const double* w, int64_t R, int nsplit,
                     const int2* pairs, int npairs, double* part, hipStream_t s) {
  const int nu = (4 * npairs + 7) / 8;   // blocks per wavefront: 1, 2, 3 or 5 for 1, 3, 6 or 10 pairs
  if (nu <= 1)
    k_gram_all<kW, 1><<<nsplit, kGAllThreads, 0, s>>>(S, n, m, lds, w, R, pairs, npairs, part);
  else if (nu == 2)
    k_gram_all<kW, 2><<<nsplit, kGAllThreads, 0, s>>>(S, n, m, lds, w, R, pairs, npairs, part);
  else if (nu == 3)
    k_gram_all<kW, 3><<<nsplit, kGAllThreads, 0, s>>>(S, n, m, lds, w, R, pairs, npairs, part);
  else
    k_gram_all<kW, 5><<<nsplit, kGAllThreads, 0, s>>>(S, n, m, lds, w, R, pairs, npairs, part);
}

// K from the partial tiles.  A block of kRGroups wavefronts owns 64 entries:
// wavefront g sums the slices y = g, g + kRGroups, ... (two running sums, so
// two loads are in flight), and the group sums are added in group order, so
// the result does not depend on scheduling.  Each entry of the upper triangle
// is written to both (i, j) and (j, i): K is exactly symmetric.
__global__ void __launch_bounds__(64 * kRGroups)
    k_gram_reduce(const double* __restrict__ part, int nsplit, const int2* __restrict__ pairs, int npairs, int m,
                  double* __restrict__ K) {
  __shared__ double sh[kRGroups][64];
  const int g = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t e = (int64_t)blockIdx.x * 64 + l;
  const bool in = e < (int64_t)npairs * kGT * kGT;
  const int p = in ? (int)(e / (kGT * kGT)) : 0;
  const int loc = in ? (int)(e % (kGT * kGT)) : 0;
  double s0 = 0.0, s1 = 0.0;
  if (in) {
    int y = g;
    for (; y + kRGroups < nsplit; y += 2 * kRGroups) {
      s0 += part[((int64_t)y * npairs + p) * (kGT * kGT) + loc];
      s1 += part[((int64_t)(y + kRGroups) * npairs + p) * (kGT * kGT) + loc];
    }
    if (y < nsplit) s0 += part[((int64_t)y * npairs + p) * (kGT * kGT) + loc];
  }
  sh[g][l] = s0 + s1;
  __syncthreads();
  if (g != 0 || !in) return;
  double s = 0.0;
  for (int q = 0; q < kRGroups; ++q) s += sh[q][l];
  const int2 tt = pairs[p];
  const int gi = tt.x * kGT + loc / kGT, gj = tt.y * kGT + loc % kGT;
  if (gi >= m || gj >= m || gi > gj) return;
  K[gi + (int64_t)gj * m] = s;
  K[gj + (int64_t)gi * m] = s;
}

// Modes U[:, q] = S C[:, q]: one thread per snapshot row and kMQ columns of
// C, whose entries all lanes share (C row-major, kpad columns).  The row's
// snapshot values are loaded 8 columns at a time before their products, so
// 8 loads are in flight per thread; each sum still runs over j in order.
__global__ void __launch_bounds__(256)
    k_modes(const double* __restrict__ S, int64_t n, int m, int64_t lds, const double* __restrict__ C, int kpad,
            int k, double* __restrict__ U, int64_t ldu) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int q0 = blockIdx.y * kMQ;
  if (i >= n) return;
  double acc[kMQ];
  for (int q = 0; q < kMQ; ++q) acc[q] = 0.0;
  int j = 0;
  for (; j + 8 <= m; j += 8) {
    double s8[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) s8[u] = S[i + (int64_t)(j + u) * lds];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double* c = C + (int64_t)(j + u) * kpad + q0;
#pragma unroll
      for (int q = 0; q < kMQ; ++q) acc[q] = fma(s8[u], c[q], acc[q]);
    }
  }
  for (; j < m; ++j) {
    const double s = S[i + (int64_t)j * lds];
    const double* c = C + (int64_t)j * kpad + q0;
    for (int q = 0; q < kMQ; ++q) acc[q] = fma(s, c[q], acc[q]);
  }
  for (int q = 0; q < kMQ && q0 + q < k; ++q) U[i + (int64_t)(q0 + q) * ldu] = acc[q];
}

}  // namespace

int gram_tile() { return kGT; }
int gram_all_cols() { return kGAllCols; }
int gram_rows_step() { return kGK; }
int modes_cols_per_thread() { return kMQ; }

void launch_gram(const double* S, int64_t n, int m, int64_t lds, const double* w, int64_t rows_per_split, int nsplit,
                 const int2* pairs, int npairs, double* part, hipStream_t s) {
  if (m <= kGAllCols) {
    if (w)
      launch_gram_all<true>(S, n, m, lds, w, rows_per_split, nsplit, pairs, npairs, part, s);
    else
      launch_gram_all<false>(S, n, m, lds, w, rows_per_split, nsplit, pairs, npairs, part, s);
    return;
  }
  if (w)
    k_gram<true><<<dim3(npairs, nsplit), kGThreads, 0, s>>>(S, n, m, lds, w, rows_per_split, pairs, npairs, part);
  else
    k_gram<false><<<dim3(npairs, nsplit), kGThreads, 0, s>>>(S, n, m, lds, w, rows_per_split, pairs, npairs, part);
}

void launch_gram_reduce(const double* part, int nsplit, const int2* pairs, int npairs, int m, double* K, hipStream_t s) {
  const int64_t tot = (int64_t)npairs * kGT * kGT;
  k_gram_reduce<<<(unsigned)((tot + 63) / 64), 64 * kRGroups, 0, s>>>(part, nsplit, pairs, npairs, m, K);
}

void launch_modes(const double* S, int64_t n, int m, int64_t lds, const double* C, int kpad, int k, double* U,
                  int64_t ldu, hipStream_t s) {
  k_modes<<<dim3((unsigned)((n + 255) / 256), (unsigned)(kpad / kMQ)), 256, 0, s>>>(S, n, m, lds, C, kpad, k, U,
                                                                                    ldu);
}

}  // namespace mbx
