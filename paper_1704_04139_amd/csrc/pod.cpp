// pod.cpp — POD of a snapshot set by the method of snapshots (Sec. 2.5):
// Gram matrix on the GPU (pod.hip), its eigen-decomposition on the host
// (cyclic Jacobi), modes on the GPU.  C ABI: mbx_pod, mbx_sym_eig.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/mbx.h"
#include "mbx_kernels.h"
#include "prof.h"

using namespace mbx;

namespace {

// Eigen-decomposition of a symmetric m x m matrix by cyclic Jacobi rotations
// (Jacobi 1846; the rotation that zeroes a_pq is chosen with |angle| <= pi/4,
// t = sgn(tau) / (|tau| + sqrt(1 + tau^2)), tau = (a_qq - a_pp) / (2 a_pq)).
// A is column-major and overwritten; on return lam holds the eigenvalues in
// descending order and V (column-major) the matching eigenvectors, each
// signed so that its entry of largest magnitude (the first on ties) is
// positive.  Returns false if A holds a non-finite value.
bool jacobi_eig(int m, std::vector<double>& A, std::vector<double>& lam, std::vector<double>& V) {
  auto a = [&](int i, int j) -> double& { return A[(size_t)j * m + i]; };
  for (double x : A)
    if (!std::isfinite(x)) return false;
  std::vector<double> W((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) W[(size_t)i * m + i] = 1.0;
  double fro = 0.0;
  for (double x : A) fro += x * x;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int q = 1; q < m; ++q)
      for (int p = 0; p < q; ++p) off += a(p, q) * a(p, q);
    if (off == 0.0 || off <= 1e-34 * fro) break;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = a(p, q);
        if (apq == 0.0) continue;
        const double app = a(p, p), aqq = a(q, q);
        // after a few sweeps an entry below the rounding of both diagonal
        // entries is set to zero without a rotation
        const double g = 100.0 * std::fabs(apq);
        if (sweep > 3 && std::fabs(app) + g == std::fabs(app) && std::fabs(aqq) + g == std::fabs(aqq)) {
          a(p, q) = a(q, p) = 0.0;
          continue;
        }
        const double tau = (aqq - app) / (2.0 * apq);
        double t;
        if (std::fabs(tau) > 1e150)
          t = 0.5 / tau;
        else
          t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int r = 0; r < m; ++r) {
          if (r == p || r == q) continue;
          const double arp = a(r, p), arq = a(r, q);
          const double np = c * arp - s * arq, nq = s * arp + c * arq;
          a(r, p) = a(p, r) = np;
          a(r, q) = a(q, r) = nq;
        }
        a(p, p) = app - t * apq;
        a(q, q) = aqq + t * apq;
        a(p, q) = a(q, p) = 0.0;
        double* vp = &W[(size_t)p * m];
        double* vq = &W[(size_t)q * m];
        for (int r = 0; r < m; ++r) {
          const double x = vp[r], y = vq[r];
          vp[r] = c * x - s * y;
          vq[r] = s * x + c * y;
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
    const double* v = &W[(size_t)src * m];
    int big = 0;
    for (int r = 1; r < m; ++r)
      if (std::fabs(v[r]) > std::fabs(v[big])) big = r;
    const double sg = v[big] < 0.0 ? -1.0 : 1.0;
    for (int r = 0; r < m; ++r) V[(size_t)k * m + r] = sg * v[r];
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
  if (!jacobi_eig(m, a, l, v)) return report_error(MBX_ENAN, "mbx_sym_eig: non-finite entry");
  std::copy(l.begin(), l.end(), lam);
  std::copy(v.begin(), v.end(), V);
  return MBX_OK;
}

int mbx_pod(const double* S, int64_t n, int m, int64_t lds, const double* w, double rtol, int k_max, double* modes,
            int64_t ldm, double* sigma, int* k_out, void* stream) {
  if (!S || !modes || !sigma || !k_out) return report_error(MBX_EINVAL, "mbx_pod: null pointer");
  if (n < 1 || m < 1 || m > MBX_POD_MAX_SNAPSHOTS || lds < n || ldm < n || k_max < 1 || !(rtol >= 0.0) ||
      !std::isfinite(rtol))
    return report_error(MBX_EINVAL,
                        "mbx_pod: need n >= 1, 1 <= m <= MBX_POD_MAX_SNAPSHOTS, lds >= n, ldm >= n, k_max >= 1, "
                        "finite rtol >= 0");
  *k_out = 0;
  hipStream_t s = (hipStream_t)stream;
  const int tile = gram_tile();
  const int nt = (m + tile - 1) / tile;
  std::vector<int2> pairs;
  for (int ti = 0; ti < nt; ++ti)
    for (int tj = ti; tj < nt; ++tj) pairs.push_back(make_int2(ti, tj));
  const int np = (int)pairs.size();
  // row slices: about 2048 workgroups in all, each slice a multiple of the
  // staging step
  const int step = gram_rows_step();
  const int64_t want = std::max<int64_t>(1, 2048 / np);
  int64_t R = (n + want - 1) / want;
  R = (R + step - 1) / step * step;
  const int nsplit = (int)((n + R - 1) / R);
  DevBufs d(s);
  const size_t part_elems = (size_t)nsplit * np * tile * tile;
  hipError_t e = hipMalloc(&d.p[0], sizeof(int2) * np);
  if (e == hipSuccess) e = hipMalloc(&d.p[1], sizeof(double) * part_elems);
  if (e == hipSuccess) e = hipMalloc(&d.p[2], sizeof(double) * (size_t)m * m);
  if (e != hipSuccess) return report_error(MBX_ENOMEM, hipGetErrorString(e));
  int2* d_pairs = (int2*)d.p[0];
  double* d_part = (double*)d.p[1];
  double* d_K = (double*)d.p[2];
  std::vector<double> K((size_t)m * m);
  if (hipMemcpyAsync(d_pairs, pairs.data(), sizeof(int2) * np, hipMemcpyHostToDevice, s) != hipSuccess)
    return report_error(MBX_EHIP, "mbx_pod: copy of the tile pairs failed");
  prof_begin(PK_GRAM, s);
  launch_gram(S, n, m, lds, w, R, nsplit, d_pairs, np, d_part, s);
  // algorithmic bytes: every snapshot entry (and weight) read once
  prof_end(PK_GRAM, s, 8.0 * (double)n * m + (w ? 8.0 * (double)n : 0.0));
  launch_gram_reduce(d_part, nsplit, d_pairs, np, m, d_K, s);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(K.data(), d_K, sizeof(double) * K.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return report_error(MBX_EHIP, hipGetErrorString(e));
  std::vector<double> lam, V;
  if (!jacobi_eig(m, K, lam, V)) return report_error(MBX_ENAN, "mbx_pod: non-finite Gram matrix");
  for (int i = 0; i < m; ++i) sigma[i] = std::sqrt(std::max(lam[i], 0.0));
  int k = 0;
  while (k < std::min(k_max, m) && sigma[k] > rtol * sigma[0] && sigma[k] > 0.0) ++k;
  if (k == 0) return MBX_OK;
  const int q = modes_cols_per_thread();
  const int kpad = (k + q - 1) / q * q;
  std::vector<double> C((size_t)m * kpad, 0.0);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < k; ++i) C[(size_t)j * kpad + i] = V[(size_t)i * m + j] / sigma[i];
  e = hipMalloc(&d.p[3], sizeof(double) * C.size());
  if (e != hipSuccess) return report_error(MBX_ENOMEM, hipGetErrorString(e));
  double* d_C = (double*)d.p[3];
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

}  // extern "C"
