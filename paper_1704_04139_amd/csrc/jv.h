// jv.h — one row of the matrix-free Newton-system product (shared by the
// Krylov kernels and the preconditioner).
#pragma once
#include "mbx_dev.h"

namespace mbx {

// Row i of the matrix-free product with the scaled, condensed Jacobian of
// the residual: same stencil as k_residual, linear in v, coefficients (type
// KT) from the last linearisation, v of type VT, accumulated in AT.  Every
// load of the row is issued before the arithmetic (absent neighbours read
// voxel i and are zeroed by select).
template <typename KT, typename VT, typename AT>
__device__ inline void jv_row(const CellDev& cd, int i, const VT* __restrict__ v, AT& yc_out, AT& yp_out) {
  const size_t N = cd.N;
  const KT* wpo = (const KT*)cd.wpore;
  const KT* can = (const KT*)cd.coef_an;
  const KT* cca = (const KT*)cd.coef_ca;
  const VoxCoord c3 = coord_of(cd, i);
  int k[6];
  bool ex[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const int kk = neighbour(cd, i, c3.x, c3.y, c3.z, d);
    ex[d] = kk >= 0;
    k[d] = ex[d] ? kk : i;
  }
  const uint32_t mi = cd.meta[i];
  const AT vc = (AT)v[i], vp = (AT)v[N + i];
  const AT wiv = (AT)wpo[i];
  uint32_t mk[6];
  AT vck[6], vpk[6], wk[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    mk[d] = cd.meta[k[d]];
    vck[d] = (AT)v[k[d]];
    vpk[d] = (AT)v[N + k[d]];
    wk[d] = (AT)wpo[k[d]];
  }
  const int L = lab_of(mi);
  const AT wi = (L == PORE) ? wiv : (AT)0;
  const AT Gk = (AT)(KT)cd.Gk, tth = (AT)(KT)cd.tth, Dh = (AT)(KT)cd.Dh, tau = (AT)(KT)cd.tau, Ke = (AT)(KT)cd.Ke;
  const AT Dsh = (AT)(KT)cd.Dsh[L == CATHODE], Gs = (AT)(KT)cd.Gs[L == CATHODE], Ks = (AT)(KT)cd.Ks[L == CATHODE];
  AT yc = vc, yp = (AT)0;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const int Lk = lab_of(mk[d]);
    const bool lo = i < k[d];
    const AT vk = vck[d], pk = vpk[d];
    // electrolyte face (oriented low index -> high index, as in the residual)
    const AT vca = lo ? vc : vk, vcb = lo ? vk : vc;
    const AT vpa = lo ? vp : pk, vpb = lo ? pk : vp;
    const AT wa = lo ? wi : wk[d], wb = lo ? wk[d] : wi;
    const AT dj = Gk * (-(vpb - vpa) + tth * (wb * vcb - wa * vca));
    const AT dN = -Dh * (vcb - vca) + tau * dj;
    // interface face: coefficients of the solid voxel's face record
    const bool pore_side = L == PORE;
    const bool iface = (L == PORE) != (Lk == PORE);
    const uint32_t f = iface ? face_rank(pore_side ? mk[d] : mi, pore_side ? (d ^ 1) : d) : 0u;
    const bool an = (pore_side ? Lk : L) == ANODE;
    const KT* co = an ? can + 5 * (size_t)f : cca + 3 * (size_t)f;
    const AT c0 = (AT)co[0], c1 = (AT)co[1], c2 = (AT)co[2];
    const AT c3v = an ? (AT)co[3] : (AT)0, c4v = an ? (AT)co[4] : (AT)0;
    const AT vs = pore_side ? vk : vc, ve = pore_side ? vc : vk;     // solid / pore values
    const AT ps = pore_side ? pk : vp, pe = pore_side ? vp : pk;
    const AT q = c0 * vs + c1 * ve + c2 * (ps - pe);
    const AT qp = c3v * ve + c4v * (ps - pe);
    AT tc, tp;
    if (L == PORE && Lk == PORE) {
      tc = lo ? dN : -dN;
      tp = lo ? dj : -dj;
    } else if (L == Lk) {
      tc = Dsh * (vc - vk);
      tp = Gs * (vp - pk);
    } else if (iface && pore_side) {
      tc = -Ke * (q + qp);
      tp = -(q + qp);
    } else if (iface) {
      tc = Ks * q;
      tp = q + qp;
    } else {
      tc = (AT)0;
      tp = (AT)0;
    }
    const AT tb = (d == 4 && L == ANODE) ? (AT)(KT)cd.Gcol * vp : (AT)0;   // anode collector
    yc += ex[d] ? tc : (AT)0;
    yp += ex[d] ? tp : tb;
  }
  yc_out = yc;
  yp_out = yp;
}

}  // namespace mbx
