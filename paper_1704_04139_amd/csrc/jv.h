// jv.h — one row of the matrix-free Newton-system product (shared by the
// Krylov kernels and the preconditioner).
#pragma once
#include "mbx_dev.h"

namespace mbx {

// Row i of the matrix-free product with the scaled, condensed Jacobian of
// the residual: same stencil as k_residual, linear in v, coefficients (type
// KT) from the last linearisation, v of type VT, accumulated in AT.  Every
// load of the row is a buffer load issued before the arithmetic; absent
// neighbours are read at element kNoIdx, past the end of every array (zero),
// and their terms are dropped by select.  The anode and cathode face records
// are read through one descriptor that starts at the anode records (the
// cathode records follow them in the cell's allocation).
template <typename KT, typename VT, typename AT>
__device__ inline void jv_row(const CellDev& cd, int i, const VT* __restrict__ v, AT& yc_out, AT& yp_out) {
  constexpr uint32_t kt = sizeof(KT), vt = sizeof(VT);
  const uint32_t N = (uint32_t)cd.N;
  const BufRes rm = buf_of(cd.meta, N * 4u);
  const BufRes rv = buf_of(v, 2u * N * vt);
  const BufRes rw = buf_of(cd.wpore, N * kt);
  const uint32_t ca_off = (uint32_t)((const char*)cd.coef_ca - (const char*)cd.coef_an);
  const BufRes rco = buf_of(cd.coef_an, ca_off + 3u * (uint32_t)(cd.F_ca > 0 ? cd.F_ca : 1) * kt);
  const VoxCoord c3 = coord_of(cd, i);
  uint32_t k[6];
  bool ex[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const int kk = neighbour(cd, i, c3.x, c3.y, c3.z, d);
    ex[d] = kk >= 0;
    k[d] = ex[d] ? (uint32_t)kk : kNoIdx;
  }
  const uint32_t ui = (uint32_t)i;
  const uint32_t mi = buf_ld<uint32_t>(rm, ui * 4u);
  const AT vc = (AT)buf_ld<VT>(rv, ui * vt), vp = (AT)buf_ld<VT>(rv, ui * vt, N * vt);
  const AT wiv = (AT)buf_ld<KT>(rw, ui * kt);
  uint32_t mk[6];
  AT vck[6], vpk[6], wk[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    mk[d] = buf_ld<uint32_t>(rm, k[d] * 4u);
    vck[d] = (AT)buf_ld<VT>(rv, k[d] * vt);
    vpk[d] = (AT)buf_ld<VT>(rv, k[d] * vt, N * vt);
    wk[d] = (AT)buf_ld<KT>(rw, k[d] * kt);
  }
  const int L = lab_of(mi);
  const AT wi = (L == PORE) ? wiv : (AT)0;
  const AT Gk = (AT)(KT)cd.Gk, tth = (AT)(KT)cd.tth, Dh = (AT)(KT)cd.Dh, tau = (AT)(KT)cd.tau, Ke = (AT)(KT)cd.Ke;
  // per-phase constants loaded as scalars, then selected per lane
  const AT Dsh0 = (AT)(KT)cd.Dsh[0], Dsh1 = (AT)(KT)cd.Dsh[1], Gs0 = (AT)(KT)cd.Gs[0], Gs1 = (AT)(KT)cd.Gs[1];
  const AT Ks0 = (AT)(KT)cd.Ks[0], Ks1 = (AT)(KT)cd.Ks[1];
  const bool cat = L == CATHODE;
  const AT Dsh = cat ? Dsh1 : Dsh0, Gs = cat ? Gs1 : Gs0, Ks = cat ? Ks1 : Ks0;
  AT yc = vc, yp = (AT)0;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const int Lk = lab_of(mk[d]);
    // the +x, +y, +z neighbours (odd d) have the higher index: the face's
    // orientation is known per direction at compile time
    const bool lo = (d & 1) != 0;
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
    // face indices are below 2^24 (checked at creation): 24-bit products
    const uint32_t co = an ? __umul24(f, 5u * kt) : ca_off + __umul24(f, 3u * kt);
    const AT c0 = (AT)buf_ld<KT>(rco, co), c1 = (AT)buf_ld<KT>(rco, co + kt), c2 = (AT)buf_ld<KT>(rco, co + 2 * kt);
    const AT c3v = (AT)buf_ld<KT>(rco, an ? co + 3 * kt : kNoOff), c4v = (AT)buf_ld<KT>(rco, an ? co + 4 * kt : kNoOff);
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
