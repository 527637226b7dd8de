// pod.cpp — POD of a snapshot set by the method of snapshots (Sec. 2.5):
// Gram matrix on the GPU (pod.hip), its eigen-decomposition on the host
// (Householder tridiagonalisation and implicit QR), modes on the GPU.  C ABI: mbx_pod, mbx_sym_eig.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <limits>
#include <mutex>
#include <vector>

#include "../../include/mbx.h"
#include "mbx_kernels.h"
#include "prof.h"

using namespace mbx;

// Workspace of mbx_pod_noalloc, one copy per device, held until the process
// ends.  It covers the largest POD any call may ask for (m = 512 snapshots:
// 16 MiB of partial Gram tiles, 2 MiB each for K and for the eigenvector
// coefficients, and the tile pairs).  Host code never passes the array's name
// to a kernel or a copy: each device's address comes from hipGetSymbolAddress.
constexpr size_t kPodScratchBytes = size_t(21) << 20;
static __device__ __align__(256) char scratch[kPodScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of the scratch array, looked
// up once per device with that device current.
int scratch_address(char** out) {
  int dev = 0;
  if (hipError_t e = hipGetDevice(&dev); e != hipSuccess)
    return report_error(MBX_EHIP, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return report_error(MBX_EINVAL, "mbx_pod_noalloc: device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return report_error(MBX_EHIP, "mbx_pod_noalloc: hipGetSymbolAddress of the scratch array failed");
    g_scratch_ptr[dev] = (char*)p;
  }
  *out = g_scratch_ptr[dev];
  return MBX_OK;
}

// Eigen-decomposition of a symmetric m x m matrix in two stages (Golub and
// Van Loan, Matrix Computations, Sec. 8.3):
//   1. Householder reduction to tridiagonal form, A = Q T Q^T: reflector k
//      maps column k below the subdiagonal onto its first entry and is
//      applied from both sides to the trailing block as the rank-2 update
//      A <- A - v w^T - w v^T (w = p - (v^T p) v, p = 2 A v, |v| = 1);
//      Q accumulates the reflectors;
//   2. implicit symmetric QR steps with the Wilkinson shift on T: the
//      shift's first Givens rotation creates a bulge below the subdiagonal
//      that further rotations chase to the end of the unreduced block;
//      subdiagonal entries below 4u (|d_i| + |d_i+1|) are set to zero.
// Every rotation touches rows and columns k-1 .. k+2 of the banded T and
// two columns of the eigenvector matrix Q.  O(m^3) work with a small
// constant.  A is column-major and overwritten; on return lam holds the
// eigenvalues in descending order and V (column-major) the matching
// eigenvectors, each signed so that its entry of largest magnitude (the
// first on ties) is positive.  Returns false if A holds a non-finite value
// or the iteration does not converge.
bool sym_eig(int m, std::vector<double>& A, std::vector<double>& lam, std::vector<double>& V) {
  auto a = [&](int i, int j) -> double& { return A[(size_t)j * m + i]; };
  for (double x : A)
    if (!std::isfinite(x)) return false;
  std::vector<double> Q((size_t)m * m, 0.0);
  auto q = [&](int i, int j) -> double& { return Q[(size_t)j * m + i]; };
  for (int i = 0; i < m; ++i) q(i, i) = 1.0;
  // ---- 1. Householder tridiagonalisation
  std::vector<double> v(m), p(m), w(m);
  for (int k = 0; k + 2 < m; ++k) {
    const int n = m - k - 1;   // length of the column below the diagonal
    double norm2 = 0.0;
    for (int r = 0; r < n; ++r) norm2 += a(k + 1 + r, k) * a(k + 1 + r, k);
    const double x0 = a(k + 1, k);
    const double alpha = -(x0 >= 0.0 ? 1.0 : -1.0) * std::sqrt(norm2);
    // v = x - alpha e1, normalised
    for (int r = 0; r < n; ++r) v[r] = a(k + 1 + r, k);
    v[0] -= alpha;
    double vn = 0.0;
    for (int r = 0; r < n; ++r) vn += v[r] * v[r];
    if (vn == 0.0) continue;   // the column is already reduced
    vn = std::sqrt(vn);
    for (int r = 0; r < n; ++r) v[r] /= vn;
    // p = 2 A_sub v, w = p - (v^T p) v: H A H = A - v w^T - w v^T
    for (int r = 0; r < n; ++r) {
      double acc = 0.0;
      for (int c = 0; c < n; ++c) acc += a(k + 1 + r, k + 1 + c) * v[c];
      p[r] = 2.0 * acc;
    }
    double vp = 0.0;
    for (int r = 0; r < n; ++r) vp += v[r] * p[r];
    for (int r = 0; r < n; ++r) w[r] = p[r] - vp * v[r];
    for (int c = 0; c < n; ++c)
      for (int r = 0; r < n; ++r) a(k + 1 + r, k + 1 + c) -= v[r] * w[c] + w[r] * v[c];
    a(k + 1, k) = a(k, k + 1) = alpha;
    for (int r = 1; r < n; ++r) a(k + 1 + r, k) = a(k, k + 1 + r) = 0.0;
    // Q <- Q H, H = I - 2 v v^T on indices k+1 ..
    for (int r = 0; r < m; ++r) {
      double acc = 0.0;
      for (int c = 0; c < n; ++c) acc += q(r, k + 1 + c) * v[c];
      acc *= 2.0;
      for (int c = 0; c < n; ++c) q(r, k + 1 + c) -= acc * v[c];
    }
  }
  // ---- 2. implicit symmetric QR with the Wilkinson shift on the band of A
  auto rotate = [&](int k, double c, double s) {
    // A <- G^T A G with G acting on (k, k+1): G = [[c, s], [-s, c]]
    const int lo = std::max(0, k - 1), hi = std::min(m - 1, k + 2);
    for (int j = lo; j <= hi; ++j) {
      const double x = a(k, j), y = a(k + 1, j);
      a(k, j) = c * x - s * y;
      a(k + 1, j) = s * x + c * y;
    }
    for (int i = lo; i <= hi; ++i) {
      const double x = a(i, k), y = a(i, k + 1);
      a(i, k) = c * x - s * y;
      a(i, k + 1) = s * x + c * y;
    }
    for (int r = 0; r < m; ++r) {
      const double x = q(r, k), y = q(r, k + 1);
      q(r, k) = c * x - s * y;
      q(r, k + 1) = s * x + c * y;
    }
  };
  // rotation with [c s; -s c]^T [x; z] = [*; 0]
  auto givens = [](double x, double z, double& c, double& s) {
    if (z == 0.0) {
      c = 1.0;
      s = 0.0;
    } else if (std::fabs(z) > std::fabs(x)) {
      const double t = -x / z;
      s = 1.0 / std::sqrt(1.0 + t * t);
      c = s * t;
    } else {
      const double t = -z / x;
      c = 1.0 / std::sqrt(1.0 + t * t);
      s = c * t;
    }
  };
  const double u4 = 4.0 * std::numeric_limits<double>::epsilon();
  int hi = m - 1;
  for (int iter = 0; hi > 0; ++iter) {
    if (iter > 60 * m) return false;
    // deflate negligible subdiagonal entries
    for (int i = 0; i < hi; ++i)
      if (std::fabs(a(i + 1, i)) <= u4 * (std::fabs(a(i, i)) + std::fabs(a(i + 1, i + 1))))
        a(i + 1, i) = a(i, i + 1) = 0.0;
    while (hi > 0 && a(hi, hi - 1) == 0.0) --hi;
    if (hi == 0) break;
    int lo = hi - 1;
    while (lo > 0 && a(lo, lo - 1) != 0.0) --lo;
    // Wilkinson shift from the trailing 2x2 block of [lo, hi]
    const double dd = 0.5 * (a(hi - 1, hi - 1) - a(hi, hi));
    const double e2 = a(hi, hi - 1) * a(hi, hi - 1);
    const double mu = a(hi, hi) - e2 / (dd + (dd >= 0.0 ? 1.0 : -1.0) * std::sqrt(dd * dd + e2));
    double x = a(lo, lo) - mu, z = a(lo + 1, lo);
    for (int k = lo; k < hi; ++k) {
      double c, s;
      givens(x, z, c, s);
      rotate(k, c, s);
      if (k + 1 < hi) {
        x = a(k + 1, k);
        z = a(k + 2, k);
      }
    }
  }
  std::vector<int> order(m);
  for (int i = 0; i < m; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return a(x, x) > a(y, y); });
  lam.resize(m);
  V.assign((size_t)m * m, 0.0);
  for (int k = 0; k < m; ++k) {
    const int src = order[k];
    lam[k] = a(src, src);
    const double* col = &Q[(size_t)src * m];
    int big = 0;
    for (int r = 1; r < m; ++r)
      if (std::fabs(col[r]) > std::fabs(col[big])) big = r;
    const double sg = col[big] < 0.0 ? -1.0 : 1.0;
    for (int r = 0; r < m; ++r) V[(size_t)k * m + r] = sg * col[r];
  }
  return true;
}

// Workspace of one mbx_pod call.  On every exit, including an error after
// work was enqueued, the stream is drained before the buffers are freed.
struct DevBufs {
  hipStream_t s;
  void* p[4] = {nullptr, nullptr, nullptr, nullptr};
  explicit DevBufs(hipStream_t st) : s(st) {}
  ~DevBufs() {
    (void)hipStreamSynchronize(s);
    for (void* x : p)
      if (x) (void)hipFree(x);
  }
};

// Device workspace of one POD call: the tile pairs, the partial Gram tiles of
// every row slice, K and the scaled eigenvector matrix C.  part_bytes and the
// other sizes follow from (n, m, k); the offsets are 256-byte aligned.
struct PodPlan {
  std::vector<int2> pairs;
  int np = 0, nsplit = 0, tile = 0;
  int64_t R = 0;
  size_t off_pairs = 0, off_part = 0, off_K = 0, off_C = 0, total = 0;
};

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

PodPlan pod_plan(int64_t n, int m, int k_cap) {
  PodPlan P;
  P.tile = gram_tile();
  const int nt = (m + P.tile - 1) / P.tile;
  for (int ti = 0; ti < nt; ++ti)
    for (int tj = ti; tj < nt; ++tj) P.pairs.push_back(make_int2(ti, tj));
  P.np = (int)P.pairs.size();
  // row slices, each a multiple of the staging step: about 2048 workgroups in
  // all when each owns one tile pair; one per compute unit (256) when each
  // owns a slice of every pair (sets at most gram_all_cols() wide)
  const int step = gram_rows_step();
  const int64_t want = m <= gram_all_cols() ? 256 : std::max<int64_t>(1, 2048 / P.np);
  int64_t R = (n + want - 1) / want;
  P.R = (R + step - 1) / step * step;
  P.nsplit = (int)((n + P.R - 1) / P.R);
  const int q = modes_cols_per_thread();
  const int kpad = (k_cap + q - 1) / q * q;
  P.off_pairs = 0;
  P.off_part = up256(sizeof(int2) * P.np);
  P.off_K = P.off_part + up256(sizeof(double) * (size_t)P.nsplit * P.np * P.tile * P.tile);
  P.off_C = P.off_K + up256(sizeof(double) * (size_t)m * m);
  P.total = P.off_C + up256(sizeof(double) * (size_t)m * kpad);
  return P;
}

// The POD on a workspace ws of at least pod_plan(n, m, min(k_max, m)).total
// bytes (device memory).  Synchronises the stream before it returns, on
// every path that enqueued work.
int pod_run(const double* S, int64_t n, int m, int64_t lds, const double* w, double rtol, int k_max,
            double* modes, int64_t ldm, double* sigma, int* k_out, hipStream_t s, const PodPlan& P, char* ws) {
  struct Drain {
    hipStream_t s;
    ~Drain() { (void)hipStreamSynchronize(s); }
  } drain{s};
  int2* d_pairs = (int2*)(ws + P.off_pairs);
  double* d_part = (double*)(ws + P.off_part);
  double* d_K = (double*)(ws + P.off_K);
  double* d_C = (double*)(ws + P.off_C);
  std::vector<double> K((size_t)m * m);
  if (hipMemcpyAsync(d_pairs, P.pairs.data(), sizeof(int2) * P.np, hipMemcpyHostToDevice, s) != hipSuccess)
    return report_error(MBX_EHIP, "mbx_pod: copy of the tile pairs failed");
  prof_begin(PK_GRAM, s);
  launch_gram(S, n, m, lds, w, P.R, P.nsplit, d_pairs, P.np, d_part, s);
  // algorithmic bytes: every snapshot entry (and weight) read once
  prof_end(PK_GRAM, s, 8.0 * (double)n * m + (w ? 8.0 * (double)n : 0.0));
  launch_gram_reduce(d_part, P.nsplit, d_pairs, P.np, m, d_K, s);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(K.data(), d_K, sizeof(double) * K.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return report_error(MBX_EHIP, hipGetErrorString(e));
  std::vector<double> lam, V;
  if (!sym_eig(m, K, lam, V)) return report_error(MBX_ENAN, "mbx_pod: non-finite Gram matrix or no convergence");
  for (int i = 0; i < m; ++i) sigma[i] = std::sqrt(std::max(lam[i], 0.0));
  int k = 0;
  while (k < std::min(k_max, m) && sigma[k] > rtol * sigma[0] && sigma[k] > 0.0) ++k;
  if (k == 0) return MBX_OK;
  const int q = modes_cols_per_thread();
  const int kpad = (k + q - 1) / q * q;
  std::vector<double> C((size_t)m * kpad, 0.0);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < k; ++i) C[(size_t)j * kpad + i] = V[(size_t)i * m + j] / sigma[i];
  e = hipMemcpyAsync(d_C, C.data(), sizeof(double) * C.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) {
    launch_modes(S, n, m, lds, d_C, kpad, k, modes, ldm, s);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return report_error(MBX_EHIP, hipGetErrorString(e));
  *k_out = k;
  return MBX_OK;
}

int pod_check(const double* S, int64_t n, int m, int64_t lds, double rtol, int k_max, double* modes, int64_t ldm,
              double* sigma, int* k_out) {
  if (!S || !modes || !sigma || !k_out) return report_error(MBX_EINVAL, "mbx_pod: null pointer");
  if (n < 1 || m < 1 || m > MBX_POD_MAX_SNAPSHOTS || lds < n || ldm < n || k_max < 1 || !(rtol >= 0.0) ||
      !std::isfinite(rtol))
    return report_error(MBX_EINVAL,
                        "mbx_pod: need n >= 1, 1 <= m <= MBX_POD_MAX_SNAPSHOTS, lds >= n, ldm >= n, k_max >= 1, "
                        "finite rtol >= 0");
  *k_out = 0;
  return MBX_OK;
}

}  // namespace

extern "C" {

int mbx_sym_eig(int m, const double* A, double* lam, double* V) {
  if (m < 1 || m > MBX_POD_MAX_SNAPSHOTS || !A || !lam || !V)
    return report_error(MBX_EINVAL, "mbx_sym_eig: need 1 <= m <= MBX_POD_MAX_SNAPSHOTS and non-null arrays");
  std::vector<double> a(A, A + (size_t)m * m), l, v;
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < j; ++i)
      if (a[(size_t)j * m + i] != a[(size_t)i * m + j])
        return report_error(MBX_EINVAL, "mbx_sym_eig: the matrix is not symmetric");
  if (!sym_eig(m, a, l, v)) return report_error(MBX_ENAN, "mbx_sym_eig: non-finite entry or no convergence");
  std::copy(l.begin(), l.end(), lam);
  std::copy(v.begin(), v.end(), V);
  return MBX_OK;
}

int mbx_pod(const double* S, int64_t n, int m, int64_t lds, const double* w, double rtol, int k_max, double* modes,
            int64_t ldm, double* sigma, int* k_out, void* stream) {
  if (int e = pod_check(S, n, m, lds, rtol, k_max, modes, ldm, sigma, k_out)) return e;
  hipStream_t s = (hipStream_t)stream;
  const PodPlan P = pod_plan(n, m, std::min(k_max, m));
  DevBufs d(s);
  if (hipError_t e = hipMalloc(&d.p[0], P.total); e != hipSuccess) return report_error(MBX_ENOMEM, hipGetErrorString(e));
  return pod_run(S, n, m, lds, w, rtol, k_max, modes, ldm, sigma, k_out, s, P, (char*)d.p[0]);
}

int mbx_pod_noalloc(const double* S, int64_t n, int m, int64_t lds, const double* w, double rtol, int k_max,
                    double* modes, int64_t ldm, double* sigma, int* k_out, void* stream) {
  if (int e = pod_check(S, n, m, lds, rtol, k_max, modes, ldm, sigma, k_out)) return e;
  const PodPlan P = pod_plan(n, m, std::min(k_max, m));
  if (P.total > kPodScratchBytes) {
    char msg[160];
    snprintf(msg, sizeof msg, "mbx_pod_noalloc: the POD needs %zu workspace bytes, more than the %zu of the scratch array",
             P.total, kPodScratchBytes);
    return report_error(MBX_EINVAL, msg);
  }
  char* ws = nullptr;
  if (int e = scratch_address(&ws)) return e;
  return pod_run(S, n, m, lds, w, rtol, k_max, modes, ldm, sigma, k_out, (hipStream_t)stream, P, ws);
}

}  // extern "C"
