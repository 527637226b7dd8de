// kernels.hip — HIP kernels of the implicit cell step for gfx950.
//
// Every voxel kernel is launched over the blocks of a batch of cells: block
// b works on cell blk[b].x, voxels [blk[b].y*256, +256).  One cell is a batch
// of one.  Kernels skip cells whose descriptor has active == 0, and the
// Krylov kernels also skip cells whose GMRES solve has converged.
#include <hip/hip_runtime.h>

#include "mbx_dev.h"
#include "mbx_kernels.h"
#include "jv.h"
#include "reduce.h"
#include "prof.h"

#include <rocprim/device/device_scan.hpp>

#include <algorithm>

namespace mbx {

template <typename KT>
__device__ inline KT* vec(const CellDev& cd, int sel) {
  const size_t n2 = 2 * (size_t)cd.N;
  switch (sel) {
    case VEC_Z: return (KT*)cd.z;
    case VEC_W: return (KT*)cd.w;
    case VEC_B: return (KT*)cd.b;
    default: return (KT*)cd.Vb + (size_t)sel * n2;
  }
}

__device__ inline double cref_of(const CellDev& cd, int L) { return L == PORE ? cd.c0 : cd.cmax[L - 1]; }

// ------------------------------------------------------------------ setup
// Label validation and interface masks (Sec. 2.4: each face of the voxel
// grid is either a same-phase transport face or a solid/pore interface
// carrying the Butler-Volmer flux; the paper's interface table has no
// anode/cathode interface, so such faces are rejected).
__global__ void __launch_bounds__(kBlock) k_build_meta(const uint8_t* __restrict__ lab, int nx, int ny, int nz,
                                                       uint32_t* __restrict__ meta, int* __restrict__ cnt_an,
                                                       int* __restrict__ cnt_ca, int* __restrict__ flags) {
  const int N = nx * ny * nz;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= N) return;
  const int Lraw = lab[i];
  if (Lraw > 3) {
    atomicOr(&flags[0], 1);
    meta[i] = 0;
    cnt_an[i] = cnt_ca[i] = 0;
    return;
  }
  // a half cell's Li foil (label 3, Sec. 2.2) takes the counter-electrode slot
  if (Lraw == 3) atomicOr(&flags[0], 4);
  if (Lraw == CATHODE) atomicOr(&flags[0], 8);
  const int L = Lraw == 3 ? CATHODE : Lraw;
  const int x = i % nx, y = (i / nx) % ny, z = i / (nx * ny);
  const int nb[6] = {x > 0 ? i - 1 : -1,      x < nx - 1 ? i + 1 : -1,      y > 0 ? i - nx : -1,
                     y < ny - 1 ? i + nx : -1, z > 0 ? i - nx * ny : -1, z < nz - 1 ? i + nx * ny : -1};
  uint32_t mask = 0;
  for (int d = 0; d < 6; ++d) {
    if (nb[d] < 0) continue;
    const int Lk = lab[nb[d]] == 3 ? CATHODE : lab[nb[d]];
    if ((L == PORE) != (Lk == PORE)) mask |= 1u << d;
    if ((L == ANODE && Lk == CATHODE) || (L == CATHODE && Lk == ANODE)) atomicOr(&flags[0], 2);
  }
  if (z == 0 && L == ANODE) atomicOr(&flags[1], 1);
  if (z == nz - 1 && L == CATHODE) atomicAdd(&flags[2], 1);
  meta[i] = (uint32_t)L | (mask << 2);
  const int cnt = __popc(mask);
  cnt_an[i] = (L == ANODE) ? cnt : 0;
  cnt_ca[i] = (L == CATHODE) ? cnt : 0;
}

// Stores each solid voxel's first face index (exclusive prefix sums of the
// per-voxel face counts, one scan per phase) and the compacted face lists
// (voxel index * 8 + direction) in canonical order.
__global__ void __launch_bounds__(kBlock) k_finish_meta(int N, uint32_t* __restrict__ meta,
                                                        const int* __restrict__ off_an,
                                                        const int* __restrict__ off_ca,
                                                        int* __restrict__ faces_an, int* __restrict__ faces_ca) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= N) return;
  const uint32_t m = meta[i];
  const int L = lab_of(m);
  if (L == PORE) return;
  const int base = (L == ANODE) ? off_an[i] : off_ca[i];
  meta[i] = m | ((uint32_t)base << 8);
  int* fl = (L == ANODE) ? faces_an : faces_ca;
  int r = 0;
  for (int d = 0; d < 6; ++d)
    if ((mask_of(m) >> d) & 1u) fl[base + r++] = i * 8 + d;
}

// Colour-split copy of the meta words (padding slots of odd nx stay zero
// and are never read: no voxel has them as a neighbour), label and mask
// only; cnt gets each slot's interface-face count for the base scan.
__global__ void __launch_bounds__(kBlock) k_meta_rb(CellDev cd, int* __restrict__ cnt) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= cd.N) return;
  const VoxCoord v = coord_of(cd, i);
  const uint32_t m = cd.meta[i];
  const int p = rb_index(cd, v.x, v.y, v.z);
  ((uint32_t*)cd.meta_rb)[p] = m & 0xFFu;
  cnt[p] = __popc(mask_of(m));
}

// Face-base field of the colour-split meta words: the start of the slot's
// list in its colour's part of cond_rb (off = exclusive scan of the counts
// over both colours; colour 1's part starts at off[rbH]).
__global__ void __launch_bounds__(kBlock) k_meta_rb_base(CellDev cd, const int* __restrict__ off) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= 2 * cd.rbH) return;
  uint32_t* mrb = (uint32_t*)cd.meta_rb;
  const uint32_t m = mrb[p];
  if (!mask_of(m)) return;
  const int base = off[p] - (p >= cd.rbH ? off[cd.rbH] : 0);
  mrb[p] = m | ((uint32_t)base << 8);
}

// Zero-current equilibrium (every interface current vanishes; the plated
// amount makes the plating current zero: f_pre(n) = exp(-F U_an(x0)/RT)).
__global__ void __launch_bounds__(kBlock) k_init_state(CellDev* cells, const int2* __restrict__ blk) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  const int i = bb.y * kBlock + threadIdx.x;
  if (i >= cd.N) return;
  const uint32_t m = cd.meta[i];
  const int L = lab_of(m);
  const double Uan = cd.U0[0] + cd.U1[0] * log((1.0 - cd.x0) / cd.x0);
  // a half cell's foil sits at the electrolyte potential (eta = 0 without an OCP)
  const double Uca = cd.half ? 0.0 : cd.U0[1] + cd.U1[1] * log((1.0 - cd.y0) / cd.y0);
  double c, p;
  if (L == PORE) {
    c = cd.c0;
    p = -Uan;
  } else if (L == ANODE) {
    c = cd.x0 * cd.cmax[0];
    p = 0.0;
  } else {
    c = cd.y0 * cd.cmax[1];
    p = Uca - Uan;
  }
  cd.c[i] = c;
  cd.phi[i] = p;
  if (L == ANODE) {
    const double f = exp(-kFaraday * Uan / cd.RT);
    const double neq = cd.n_c * pow(f / (1.0 - f), 0.25);
    const uint32_t cnt = __popc(mask_of(m));
    for (uint32_t r = 0; r < cnt; ++r) cd.n[base_of(m) + r] = neq;
  }
}

// --------------------------------------------------------------- residual
// FP64 residual of the implicit Euler system (eq. 2.13) at the trial state,
// in two passes.
//
// Interface pass (k_iface): one thread per solid/pore face of the compacted
// per-phase face lists (anode faces, then cathode faces, each in canonical
// order).  It evaluates the face's Butler-Volmer intercalation (eq. 2.5) and,
// on anode faces, plating/stripping (eq. 2.8) with the plated amount
// eliminated by its own balance (plated_root) -- once per face -- and stores
// the intercalation and the total current of the face, the plated-amount row
// R^n, and with LIN the scaled face coefficients of the linearisation
// (plating condensed onto the voxel unknowns) and the potential-operator
// conductance of the face.
//
// Voxel pass (k_residual): one thread per voxel; every same-phase face flux
// is evaluated from the two adjacent voxels in the same orientation on both
// sides, every interface face's current is read from the face pass, so the
// scatter conserves Li to rounding:
//   pore/pore   j = -kappa dphi/h + kappa (1-t+) theta RT/F dln c/h,
//               N = -De dc/h + t+/F j                     (eqs. 2.3-2.4, 2.6)
//   solid/solid N = -Ds dc/h, j = -sigma dphi/h            (eqs. 2.1-2.2)
//   solid/pore  the face current as the numerical flux (eq. 2.4)
//   collectors  anode at phi = 0 across h/2; cathode galvanostatic.
// With LIN it also writes the pore 1/c coefficient.
__device__ inline int face_neighbour(const CellDev& cd, int s, int d) {
  switch (d) {
    case 0: return s - 1;
    case 1: return s + 1;
    case 2: return s - cd.nx;
    case 3: return s + cd.nx;
    case 4: return s - cd.nx * cd.ny;
    default: return s + cd.nx * cd.ny;
  }
}

// grid_stride: blocks per cell of the launch (the launch covers the cell's
// faces in strides of grid_stride * kBlock); 0 = the cell's voxel block count.
template <bool LIN, typename KT>
__global__ void __launch_bounds__(kBlock) k_iface(CellDev* cells, const int2* __restrict__ blk, int grid_stride) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active) return;
  const int Fa = cd.F_an, F = cd.F_an + cd.F_ca;
  const int stride = (grid_stride > 0 ? grid_stride : cd.nblk) * kBlock;
  const bool plate = cd.plating != 0;
  const double A = cd.A, dt = cd.dt, mu = cd.mu_ref;
  for (int g = bb.y * kBlock + (int)threadIdx.x; g < F; g += stride) {
    const bool an = g < Fa;
    const int f = an ? g : g - Fa;
    const int e = an ? cd.faces_an[f] : cd.faces_ca[f];
    const int sv = e >> 3, d = e & 7;
    const int pv = face_neighbour(cd, sv, d);
    const double cs = cd.c_try[sv], ce = cd.c_try[pv], ps = cd.phi_try[sv], pe = cd.phi_try[pv];
    double nf = 0.0;
    if (an) {
      nf = cd.n_try[f];
      if (cd.elim_n) {
        nf = plate ? plated_root(cd, ce, ps, pe, cd.n_old[f], cd.n[f]) : cd.n_old[f];
        cd.n_try[f] = nf;
      }
    }
    const Kin q = interface_kinetics(cd, an ? ANODE : CATHODE, cs, ce, ps, pe, nf, an && plate, LIN);
    cd.fres[g] = q.ii;
    cd.fres[(size_t)F + g] = q.ii + q.ip;
    if (an) {
      const double Rn = A * (nf - cd.n_old[f]) / dt + A * q.ip / kFaraday;
      cd.Rn[f] = Rn;
      if (LIN) {
        const double jnn = A / dt + A * q.p_n / kFaraday;
        const double kap = (A / dt) / jnn;
        KT* co = (KT*)cd.coef_an + 5 * (size_t)f;
        co[0] = (KT)(q.d_cs * cd.cmax[0] / mu);
        co[1] = (KT)(q.d_ce * cd.c0 / mu);
        co[2] = (KT)(q.g * cd.VT / mu);
        co[3] = (KT)(kap * q.p_ce * cd.c0 / mu);
        co[4] = (KT)(kap * q.g_p * cd.VT / mu);
        cd.rn_jnn[f] = Rn / jnn;
        cd.sq[f] = q.p_n * Rn / (jnn * mu);
        ((KT*)cd.cond_an)[f] = (KT)((q.g + kap * q.g_p) * cd.VT / mu);
      }
    } else if (LIN) {
      KT* co = (KT*)cd.coef_ca + 3 * (size_t)f;
      co[0] = (KT)(q.d_cs * cd.cmax[1] / mu);
      co[1] = (KT)(q.d_ce * cd.c0 / mu);
      co[2] = (KT)(q.g * cd.VT / mu);
      ((KT*)cd.cond_ca)[f] = co[2];
    }
  }
}

template <bool LIN, typename KT>
__global__ void __launch_bounds__(kBlock) k_residual(CellDev* cells, const int2* __restrict__ blk) {
  const int2 bb = block_of(blk);
  CellDev* cdp = cells + bb.x;
  const CellDev& cd = *cdp;
  if (!cd.active) return;
  const int i = bb.y * kBlock + threadIdx.x;
  double rsq = 0.0, rmax = 0.0, msq = 0.0, dnmax = 0.0;
  if (i < cd.N) {
    const VoxCoord v = coord_of(cd, i);
    const uint32_t mi = cd.meta[i];
    const int L = lab_of(mi);
    const double ci = cd.c_try[i], pi = cd.phi_try[i], cold = cd.c_old[i];
    const double A = cd.A, h = cd.h, dt = cd.dt;
    const size_t F = (size_t)cd.F_an + cd.F_ca;
    // every load of the row issued before the arithmetic: the neighbours'
    // meta words and states (absent neighbours read voxel i), then the
    // interface faces' results, whose indices need the meta words
    int kk[6];
    bool ex[6];
    uint32_t mk[6];
    double ck[6], pk[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const int k = neighbour(cd, i, v.x, v.y, v.z, d);
      ex[d] = k >= 0;
      kk[d] = ex[d] ? k : i;
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      mk[d] = cd.meta[kk[d]];
      ck[d] = cd.c_try[kk[d]];
      pk[d] = cd.phi_try[kk[d]];
    }
    double fi[6], ft[6], rnf[6], dnf[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const int Lk = lab_of(mk[d]);
      const bool iface = ex[d] && ((L == PORE) != (Lk == PORE));
      const bool pore_side = L == PORE;
      const bool an = (pore_side ? Lk : L) == ANODE;
      const uint32_t fr = iface ? face_rank(pore_side ? mk[d] : mi, pore_side ? (d ^ 1) : d) : 0u;
      const uint32_t f = fr + (an ? 0u : (uint32_t)cd.F_an);
      const double t = cd.fres[F + (iface ? f : 0u)];
      const double s1 = cd.fres[iface ? f : 0u];
      ft[d] = t;
      fi[d] = s1;
      // plated-amount row and update of an anode face, read on the solid side
      const bool own_an = iface && !pore_side && L == ANODE;
      const uint32_t fa = own_an ? fr : 0u;
      rnf[d] = own_an ? cd.Rn[fa] : 0.0;
      dnf[d] = (own_an && cd.elim_n) ? fabs(cd.n_try[fa] - cd.n[fa]) / cd.n_c : 0.0;
    }
    double Rc = cd.Vol * (ci - cold) / dt;
    double Rp = 0.0;
    const bool foil = cd.half && L == CATHODE;
    const double lci = (L == PORE) ? log(ci) : 0.0;   // ln c of this voxel, shared by its pore faces
    double wc = 1.0, wp = 0.0;   // state-independent diagonal of the scaled rows (merit weights)
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      if (!ex[d]) {
        if (d == 4 && L == ANODE) {
          Rp += 2.0 * A * cd.sigma[0] * pi / h;
        } else if (d == 5 && L == CATHODE) {
          Rp += -cd.I_app / cd.n_top;
        }
        continue;
      }
      const int Lk = lab_of(mk[d]);
      const bool lo = (d & 1) != 0;   // the +x, +y, +z neighbours (odd d) have the higher index
      const double sgn = lo ? 1.0 : -1.0;
      weight_add(cd, L, Lk, wc, wp);
      if (L == PORE && Lk == PORE) {
        const double ca = lo ? ci : ck[d], cb = lo ? ck[d] : ci;
        const double pa = lo ? pi : pk[d], pb = lo ? pk[d] : pi;
        const double lck = log(ck[d]);
        const double lca = lo ? lci : lck, lcb = lo ? lck : lci;
        const double j = -cd.kappa * (pb - pa) / h + cd.Kd * (lcb - lca);
        const double Nf = -cd.De * (cb - ca) / h + cd.tplus / kFaraday * j;
        Rc += sgn * (A * Nf);
        Rp += sgn * (A * j);
      } else if (L == Lk) {
        const double ca = lo ? ci : ck[d], cb = lo ? ck[d] : ci;
        const double pa = lo ? pi : pk[d], pb = lo ? pk[d] : pi;
        const int s = L - 1;
        const double Nf = -cd.Ds[s] * (cb - ca) / h;
        const double j = -cd.sigma[s] * (pb - pa) / h;
        Rc += sgn * (A * Nf);
        Rp += sgn * (A * j);
      } else if (L == PORE) {
        // interface face seen from the pore: its total current leaves the solid
        Rc -= A * ft[d] / kFaraday;
        Rp -= A * ft[d];
      } else {
        if (!foil) Rc += A * fi[d] / kFaraday;   // the Li foil has no concentration equation
        Rp += A * ft[d];
        if (L == ANODE) {
          const double rs = rnf[d] * dt / (A * cd.n_c);
          rsq += rs * rs;
          rmax = fmax(rmax, fabs(rs));
          dnmax = fmax(dnmax, dnf[d]);
        }
      }
    }
    cd.Rc[i] = Rc;
    cd.Rp[i] = Rp;
    const double cref = cref_of(cd, L);
    const double sc = dt / (cd.Vol * cref), sp = 1.0 / (A * cd.mu_ref);
    const double rc = Rc * sc, rp = Rp * sp;
    rsq += rc * rc + rp * rp;
    rmax = fmax(rmax, fmax(fabs(rc), fabs(rp)));
    if (L == ANODE && v.z == 0) wp += cd.Gcol;
    const double mc = rc / wc, mp = rp / fmax(wp, 1.0);
    msq += mc * mc + mp * mp;
    if (LIN) {
      ((KT*)cd.wpore)[i] = (KT)(L == PORE ? cd.c0 / ci : 0.0);
    }
  }
  const double vals[4] = {rsq, rmax, msq, dnmax};
  reduce_block<4>(cd, bb.y, vals, 0xAu);
}

// Right-hand side of the condensed, scaled Newton system:
//   b = D_r (-R_u + J_un J_nn^-1 R_n),
// also copied to w (the first GMRES residual, x = 0), with ||b||^2.
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_rhs(CellDev* cells, const int2* __restrict__ blk) {
  const int2 bb = block_of(blk);
  CellDev* cdp = cells + bb.x;
  const CellDev& cd = *cdp;
  if (!cd.active) return;
  const int i = bb.y * kBlock + threadIdx.x;
  double ss = 0.0;
  if (i < cd.N) {
    const VoxCoord v = coord_of(cd, i);
    const uint32_t mi = cd.meta[i];
    const int L = lab_of(mi);
    const double cref = cref_of(cd, L);
    double bc = -cd.Rc[i] * cd.dt / (cd.Vol * cref);
    double bp = -cd.Rp[i] / (cd.A * cd.mu_ref);
    if (cd.plating) {
      const uint32_t msk = mask_of(mi);
      if (L == ANODE) {
        for (int d = 0; d < 6; ++d)
          if ((msk >> d) & 1u) bp += cd.sq[face_rank(mi, d)];
      } else if (L == PORE && msk) {
        for (int d = 0; d < 6; ++d) {
          if (!((msk >> d) & 1u)) continue;
          const int k = neighbour(cd, i, v.x, v.y, v.z, d);
          const uint32_t mk = cd.meta[k];
          if (lab_of(mk) != ANODE) continue;
          const double s = cd.sq[face_rank(mk, d ^ 1)];
          bc -= cd.Ke * s;
          bp -= s;
        }
      }
    }
    const size_t N = cd.N;
    KT* b = (KT*)cd.b;
    KT* w = (KT*)cd.w;
    double* x = cd.x;
    b[i] = (KT)bc;
    b[N + i] = (KT)bp;
    w[i] = (KT)bc;
    w[N + i] = (KT)bp;
    x[i] = 0.0;
    x[N + i] = 0.0;
    const double bcr = (double)(KT)bc, bpr = (double)(KT)bp;
    ss = bcr * bcr + bpr * bpr;
  }
  const double vals[1] = {ss};
  reduce_block<1>(cd, bb.y, vals, 0u);
}

// ----------------------------------------------------------------- J * v
// y = J v with the row sums accumulated in FP64 in both modes: in an FP32
// vector the differences of neighbouring potentials in high-conductance
// regions would otherwise cancel away.  keep >= 0 also stores the operand
// as preconditioned basis vector `keep` of the flexible GMRES (the exact
// values the product was applied to).
// BS threads per workgroup (kBlock in table launches; a single-cell launch
// takes the size the tuner picked for the cell).
template <typename KT, int BS>
__global__ void __launch_bounds__(BS) k_matvec(CellDev* cells, const int2* __restrict__ blk, int src, int dst,
                                               int need, int keep) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active) return;
  const int i = bb.y * BS + threadIdx.x;
  if (i >= cd.N) return;
  const KT* v = vec<KT>(cd, src);
  double yc, yp;
  jv_row<KT, KT, double>(cd, i, v, yc, yp);
  if (cd.ictl[CTL_DONE] != need) return;
  const size_t N = cd.N;
  KT* y = vec<KT>(cd, dst);
  y[i] = (KT)yc;
  y[N + i] = (KT)yp;
  if (keep >= 0) {
    KT* zk = (KT*)cd.Zb + (size_t)keep * 2 * N;
    zk[i] = v[i];
    zk[N + i] = v[N + i];
  }
}

// ------------------------------------------------------------------- GMRES
// Basis vector j as a buffer of 2N entries: a lane reads its concentration
// entry at its byte offset and its potential entry through the uniform
// offset N * sizeof(KT), so a basis load needs no address arithmetic.
// Block partials of up to eight dot products: t[jj] is this thread's term
// for basis vector c + jj; partials go to part[(c + jj) * nblk + blk] for
// c + jj <= k.  The terms are transposed through LDS, so no cross-lane
// shuffles are needed: lane group g of 32 threads sums vector g's 256 terms
// eight at a time (strided by 32, fixed order), then one thread per vector
// adds the group's 32 sums in lane order.
__device__ inline void block_dots8(const CellDev& cd, int blk, int c, int k, const double (&t)[8], double* lds) {
  double* s1 = lds;                // [8][kBlock]
  double* s2 = lds + 8 * kBlock;   // [8][32]
  __syncthreads();                 // the previous chunk is done with the buffers
#pragma unroll
  for (int jj = 0; jj < 8; ++jj) s1[jj * kBlock + threadIdx.x] = t[jj];
  __syncthreads();
  {
    const int jj = threadIdx.x >> 5, l = threadIdx.x & 31;
    double a = 0.0;
#pragma unroll
    for (int r = 0; r < kBlock / 32; ++r) a += s1[jj * kBlock + l + 32 * r];
    s2[jj * 32 + l] = a;
  }
  __syncthreads();
  if (threadIdx.x < 8 && c + (int)threadIdx.x <= k) {
    const int jj = threadIdx.x;
    double a = 0.0;
#pragma unroll
    for (int l = 0; l < 32; ++l) a += s2[jj * 32 + l];
    cd.part[(size_t)(c + jj) * cd.nblk + blk] = a;
  }
}
constexpr int kDotsLds = 8 * kBlock + 8 * 32;   // doubles of LDS for block_dots8

template <typename KT>
__device__ inline BufRes basis_buf(const CellDev& cd, int j) {
  const size_t n2 = 2 * (size_t)cd.N;
  return buf_of((const KT*)cd.Vb + (size_t)j * n2, (uint32_t)(n2 * sizeof(KT)));
}

// Dots of w with basis vectors 0..k: block partials (first pass).  The
// basis loads are issued eight vectors at a time (indices past k clamp to k
// and are not used), then the eight products are reduced through LDS.
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_multidot(CellDev* cells, const int2* __restrict__ blk, int k) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active || cd.ictl[CTL_DONE]) return;
  __shared__ double lds[kDotsLds];
  const int i = bb.y * kBlock + threadIdx.x;
  const size_t N = cd.N;
  const bool in = i < cd.N;
  double wc = 0.0, wp = 0.0;
  if (in) {
    const KT* w = (const KT*)cd.w;
    wc = (double)w[i];
    wp = (double)w[N + i];
  }
  const uint32_t off = in ? (uint32_t)i * (uint32_t)sizeof(KT) : kNoOff, soff = (uint32_t)(N * sizeof(KT));
  for (int c = 0; c <= k; c += 8) {
    KT vc[8], vp[8];
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const BufRes r = basis_buf<KT>(cd, c + jj < k ? c + jj : k);
      vc[jj] = buf_ld<KT>(r, off);
      vp[jj] = buf_ld<KT>(r, off, soff);
    }
    double t[8];
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) t[jj] = (double)vc[jj] * wc + (double)vp[jj] * wp;
    block_dots8(cd, bb.y, c, k, t, lds);
  }
}

// Second pass of the dot products: column j = blockIdx.x of cell blockIdx.y
// into H(j,k) (tgt = 0) or tmp(j) (tgt = 1).
__global__ void __launch_bounds__(kBlock) k_finalize_dots(CellDev* cells, int ncell, int k, int tgt) {
  const int j = blockIdx.x, ci = blockIdx.y;
  if (ci >= ncell || j > k) return;
  const CellDev& cd = cells[ci];
  if (!cd.active || cd.ictl[CTL_DONE]) return;
  __shared__ double lds4[4];
  __shared__ double res;
  const int m = cd.m;
  double* out = tgt == 0 ? cd.gm + gm_H(m) + (size_t)(m + 1) * k : cd.gm + gm_tmp(m);
  const double r = finalize_column(cd, j, false, lds4, &res);
  if (threadIdx.x == 0) out[j] = r;
}

// First Gram-Schmidt pass and the second pass's dot products in one kernel:
// w -= sum_j H(j,k) V_j, then block partials of V_j . w for j <= k.  The
// thread's basis entries (at most kMaxRestart pairs) stay in registers
// between the two, so the basis is read once (FP32: 96 VGPRs; FP64: 172, two
// waves per SIMD, still faster than reading the basis twice).  The dots come
// from registers, which makes their reduction the critical path: it goes
// through LDS (block_dots8) rather than per-wave shuffles.
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_orth_dots(CellDev* cells, const int2* __restrict__ blk, int k) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active || cd.ictl[CTL_DONE]) return;
  __shared__ double lds[kDotsLds];
  const int m = cd.m;
  const double* hc = cd.gm + gm_H(m) + (size_t)(m + 1) * k;
  const int i = bb.y * kBlock + threadIdx.x;
  const size_t N = cd.N;
  const bool in = i < cd.N;
  KT* w = (KT*)cd.w;
  KT wc = (KT)0, wp = (KT)0;
  if (in) {
    wc = w[i];
    wp = w[N + i];
  }
  const uint32_t off = in ? (uint32_t)i * (uint32_t)sizeof(KT) : kNoOff, soff = (uint32_t)(N * sizeof(KT));
  constexpr int kCh = kMaxRestart / 8;
  KT vc[kCh][8], vp[kCh][8];
#pragma unroll
  for (int ch = 0; ch < kCh; ++ch)
    if (8 * ch <= k) {
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {   // indices past k clamp to k (loaded, not used)
        const BufRes r = basis_buf<KT>(cd, 8 * ch + jj < k ? 8 * ch + jj : k);
        vc[ch][jj] = buf_ld<KT>(r, off);
        vp[ch][jj] = buf_ld<KT>(r, off, soff);
      }
    }
#pragma unroll
  for (int ch = 0; ch < kCh; ++ch)
    if (8 * ch <= k) {
#pragma unroll
      for (int jj = 0; jj < 8; ++jj)
        if (8 * ch + jj <= k) {
          const KT hj = (KT)hc[8 * ch + jj];
          wc -= hj * vc[ch][jj];
          wp -= hj * vp[ch][jj];
        }
    }
  if (in) {
    w[i] = wc;
    w[N + i] = wp;
  } else {
    wc = (KT)0;
    wp = (KT)0;
  }
  const double dwc = (double)wc, dwp = (double)wp;
#pragma unroll
  for (int ch = 0; ch < kCh; ++ch)
    if (8 * ch <= k) {
      double t[8];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) t[jj] = (double)vc[ch][jj] * dwc + (double)vp[ch][jj] * dwp;
      block_dots8(cd, bb.y, 8 * ch, k, t, lds);
    }
}

// w -= sum_j h_j V_j with h = H(:,k) (src = 0) or tmp (src = 1); block
// partials of ||w||^2 (first pass).
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_orth(CellDev* cells, const int2* __restrict__ blk, int k, int src) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active || cd.ictl[CTL_DONE]) return;
  const int m = cd.m;
  const double* hc = src == 0 ? cd.gm + gm_H(m) + (size_t)(m + 1) * k : cd.gm + gm_tmp(m);
  const int i = bb.y * kBlock + threadIdx.x;
  const size_t N = cd.N;
  double ss = 0.0;
  if (i < cd.N) {
    KT* w = (KT*)cd.w;
    KT wc = w[i], wp = w[N + i];
    const uint32_t off = (uint32_t)i * (uint32_t)sizeof(KT), soff = (uint32_t)(N * sizeof(KT));
    for (int c = 0; c <= k; c += 8) {
      KT vc[8], vp[8];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const BufRes r = basis_buf<KT>(cd, c + jj < k ? c + jj : k);
        vc[jj] = buf_ld<KT>(r, off);
        vp[jj] = buf_ld<KT>(r, off, soff);
      }
#pragma unroll
      for (int jj = 0; jj < 8; ++jj)
        if (c + jj <= k) {
          const KT hj = (KT)hc[c + jj];
          wc -= hj * vc[jj];
          wp -= hj * vp[jj];
        }
    }
    w[i] = wc;
    w[N + i] = wp;
    ss = (double)wc * (double)wc + (double)wp * (double)wp;
  }
  const double vals[1] = {ss};
  reduce_block<1>(cd, bb.y, vals, 0u);
}

// Givens rotations of the Hessenberg column k of one cell (one thread), and
// the cell's GMRES state after iteration k.
__device__ inline void givens_column(const CellDev& cd, int k) {
  const int m = cd.m;
  double* H = cd.gm + gm_H(m) + (size_t)(m + 1) * k;
  double* g = cd.gm + gm_g(m);
  double* cs = cd.gm + gm_cs(m);
  double* sn = cd.gm + gm_sn(m);
  for (int j = 0; j < k; ++j) {
    const double t = cs[j] * H[j] + sn[j] * H[j + 1];
    H[j + 1] = -sn[j] * H[j] + cs[j] * H[j + 1];
    H[j] = t;
  }
  const double a = H[k], b = H[k + 1];
  const double r = hypot(a, b);
  double c = 1.0, s = 0.0;
  if (r > 0.0) {
    c = a / r;
    s = b / r;
  }
  cs[k] = c;
  sn[k] = s;
  H[k] = r;
  H[k + 1] = 0.0;
  g[k + 1] = -s * g[k];
  g[k] = c * g[k];
  cd.ictl[CTL_K] = k + 1;
  cd.ictl[CTL_ITERS] += 1;
  if (fabs(g[k + 1]) <= cd.red[RED_TOL] || b == 0.0)
    cd.ictl[CTL_DONE] = 1;          // converged (or exact breakdown)
  else if (k + 1 >= m)
    cd.ictl[CTL_DONE] = 2;          // cycle full: restart needed
}

// Second pass of k_orth: H(k+1,k) = ||w|| (src = 1 also adds tmp to H(:,k)),
// kept in red[RED_HNORM] for k_scale_next; then the Givens step of column k
// (one thread: givens_column).
__global__ void __launch_bounds__(kBlock) k_finalize_norm(CellDev* cells, int ncell, int k, int src) {
  const int ci = blockIdx.x;
  if (ci >= ncell) return;
  CellDev& cd = cells[ci];
  if (!cd.active || cd.ictl[CTL_DONE]) return;
  __shared__ double lds4[4];
  __shared__ double res;
  const double acc = finalize_column(cd, 0, false, lds4, &res);
  if (threadIdx.x == 0) {
    const int m = cd.m;
    double* H = cd.gm + gm_H(m) + (size_t)(m + 1) * k;
    if (src == 1) {
      const double* tmp = cd.gm + gm_tmp(m);
      for (int j = 0; j <= k; ++j) H[j] += tmp[j];
    }
    H[k + 1] = sqrt(acc);
    cd.red[RED_HNORM] = H[k + 1];
    givens_column(cd, k);
  }
}

// Second pass of the voxel-block reductions: partial columns 0..K-1 into
// red[slot..slot+K) (bit j of maxmask: max, else sum).  need: -3 any active
// cell, -4 cells whose GMRES cycle just closed (state 1 or 2), otherwise only
// cells whose GMRES state equals need.
__global__ void __launch_bounds__(kBlock) k_finalize_red(CellDev* cells, int ncell, int slot, int K, unsigned maxmask,
                                                         int need) {
  const int ci = blockIdx.x;
  if (ci >= ncell) return;
  const CellDev& cd = cells[ci];
  if (!cd.active) return;
  const int st = cd.ictl[CTL_DONE];
  if (need == -4 ? (st != 1 && st != 2) : (need != -3 && st != need)) return;
  __shared__ double lds4[4];
  __shared__ double res;
  for (int j = 0; j < K; ++j) {
    const double r = finalize_column(cd, j, (maxmask >> j) & 1u, lds4, &res);
    if (threadIdx.x == 0) cd.red[slot + j] = r;
  }
}

// V_{k+1} = w / ||w|| (red[RED_HNORM]).  Cells whose GMRES cycle ended at
// iteration k (converged or full) skip it: their V_{k+1} is not used.
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_scale_next(CellDev* cells, const int2* __restrict__ blk, int k) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active || cd.ictl[CTL_DONE]) return;
  const int i = bb.y * kBlock + threadIdx.x;
  if (i >= cd.N) return;
  const double hn = cd.red[RED_HNORM];
  const KT inv = hn > 0.0 ? (KT)(1.0 / hn) : (KT)0;
  const size_t N = cd.N;
  const KT* w = (const KT*)cd.w;
  KT* vn = vec<KT>(cd, k + 1);
  vn[i] = w[i] * inv;
  vn[N + i] = w[N + i] * inv;
}

// Back substitution R y = g for the iterations of the current cycle.
__global__ void k_backsolve(CellDev* cells, int ncell) {
  const int ci = blockIdx.x * blockDim.x + threadIdx.x;
  if (ci >= ncell) return;
  const CellDev& cd = cells[ci];
  if (!cd.active) return;
  const int st = cd.ictl[CTL_DONE];
  if (st != 1 && st != 2) return;
  const int m = cd.m;
  const int kk = cd.ictl[CTL_K];
  const double* H = cd.gm + gm_H(m);
  const double* g = cd.gm + gm_g(m);
  double* y = cd.gm + gm_y(m);
  for (int r = kk - 1; r >= 0; --r) {
    double s = g[r];
    for (int j = r + 1; j < kk; ++j) s -= H[r + (size_t)(m + 1) * j] * y[j];
    const double dgl = H[r + (size_t)(m + 1) * r];
    y[r] = dgl != 0.0 ? s / dgl : 0.0;
  }
}

// w = sum_{j<k} y_j V_j (cycle end; runs for converged cells too)
// End of a cycle (flexible GMRES): x += sum_j y_j Z_j over the cycle's
// preconditioned basis vectors, accumulated in FP64.
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_update_x(CellDev* cells, const int2* __restrict__ blk) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active) return;
  {
    const int st = cd.ictl[CTL_DONE];
    if (st != 1 && st != 2) return;
  }
  const int i = bb.y * kBlock + threadIdx.x;
  if (i >= cd.N) return;
  const int m = cd.m;
  const int kk = cd.ictl[CTL_K];
  const double* y = cd.gm + gm_y(m);
  const size_t N = cd.N;
  const KT* Z = (const KT*)cd.Zb;
  double ac = 0.0, ap = 0.0;
  for (int j = 0; j < kk; ++j) {
    const KT* zj = Z + (size_t)j * 2 * N;
    ac += y[j] * (double)zj[i];
    ap += y[j] * (double)zj[N + i];
  }
  cd.x[i] += ac;
  cd.x[N + i] += ap;
}

// Restart: w = b - J x with ||w||^2.  The iterate x is kept in FP64 and the
// product is accumulated in FP64 in both precision modes: in the mixed mode
// the rows with large conductance would otherwise turn the FP32 rounding of
// a large common potential shift into a residual floor far above the
// tolerance (restarted GMRES then acts as iterative refinement).
// With an FP32 basis (the mixed mode) a cycle that converged by the Givens
// estimate (state 1) also computes its true residual: the FP32 rounding of
// the preconditioned correction can leave the true residual above the
// tolerance, and such a cell then restarts from it (iterative refinement).
template <typename KT>
__device__ constexpr bool refine_on_convergence() { return sizeof(KT) < sizeof(double); }
template <typename KT>
__device__ inline bool needs_true_residual(int st) {
  return st == 2 || (refine_on_convergence<KT>() && st == 1);
}

template <typename KT>
__global__ void __launch_bounds__(kBlock) k_true_residual(CellDev* cells, const int2* __restrict__ blk) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active || !needs_true_residual<KT>(cd.ictl[CTL_DONE])) return;
  const int i = bb.y * kBlock + threadIdx.x;
  double ss = 0.0;
  if (i < cd.N) {
    const size_t N = cd.N;
    double yc, yp;
    jv_row<KT, double, double>(cd, i, (const double*)cd.x, yc, yp);
    const KT* b = (const KT*)cd.b;
    KT* w = (KT*)cd.w;
    const KT rc = (KT)((double)b[i] - yc), rp = (KT)((double)b[N + i] - yp);
    w[i] = rc;
    w[N + i] = rp;
    ss = (double)rc * (double)rc + (double)rp * (double)rp;
  }
  const double vals[1] = {ss};
  reduce_block<1>(cd, bb.y, vals, 0u);
}

// Start a GMRES cycle from the residual in w: V_0 = w/beta (all cells on
// the first cycle of a solve, otherwise only cells that must restart).
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_gm_start(CellDev* cells, const int2* __restrict__ blk, int first) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active) return;
  if (!first && !needs_true_residual<KT>(cd.ictl[CTL_DONE])) return;
  const double beta = sqrt(cd.red[RED_BSQ]);
  const int i = bb.y * kBlock + threadIdx.x;
  if (i >= cd.N) return;
  const size_t N = cd.N;
  const KT inv = beta > 0.0 ? (KT)(1.0 / beta) : (KT)0;
  const KT* w = (const KT*)cd.w;
  KT* v0 = vec<KT>(cd, 0);
  v0[i] = w[i] * inv;
  v0[N + i] = w[N + i] * inv;
}

// Per-cell GMRES bookkeeping after k_gm_start (one thread per cell):
// first cycle: tolerance = rtol * beta0; later: a cell that converged in the
// cycle just closed is finished (state 3) -- with refine, only if its true
// residual meets the tolerance, else it restarts from it -- and a cell that
// ran out of basis restarts from the true residual.
__global__ void k_gm_flags(CellDev* cells, int ncell, int first, int refine) {
  const int ci = blockIdx.x * blockDim.x + threadIdx.x;
  if (ci >= ncell) return;
  const CellDev& cd = cells[ci];
  if (!cd.active) return;
  const int m = cd.m;
  const double beta = sqrt(cd.red[RED_BSQ]);
  double* g = cd.gm + gm_g(m);
  if (first) {
    cd.red[RED_BETA0] = beta;
    cd.red[RED_TOL] = cd.rtol * beta;
    cd.ictl[CTL_ITERS] = 0;
  } else {
    const int st = cd.ictl[CTL_DONE];
    if (st == 3 || (st == 1 && (!refine || beta <= cd.red[RED_TOL]))) {
      cd.ictl[CTL_DONE] = 3;
      return;
    }
    if (st != 1 && st != 2) return;
  }
  for (int j = 0; j <= m; ++j) g[j] = 0.0;
  g[0] = beta;
  cd.ictl[CTL_K] = 0;
  cd.ictl[CTL_DONE] = (beta <= cd.red[RED_TOL]) ? 1 : 0;
}

// Gathers every cell's reduction slots and flags for one host read.
__global__ void k_gather_ctl(CellDev* cells, int ncell, double* out) {
  const int ci = blockIdx.x * blockDim.x + threadIdx.x;
  if (ci >= ncell) return;
  const CellDev& cd = cells[ci];
  double* o = out + (size_t)ci * (RED_NSLOT + CTL_NSLOT);
  for (int j = 0; j < RED_NSLOT; ++j) o[j] = cd.red[j];
  for (int j = 0; j < CTL_NSLOT; ++j) o[RED_NSLOT + j] = (double)cd.ictl[j];
}

// ------------------------------------------------------------------ Newton
// Raw Newton direction from the Krylov solution x: dc = c_ref x_c,
// dphi = (RT/F) x_phi, and the condensed plated unknowns
// dn = -R^n/J_nn - (dt/F) (d i_pl, condensed).
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_direction(CellDev* cells, const int2* __restrict__ blk) {
  const int2 bb = block_of(blk);
  CellDev* cdp = cells + bb.x;
  const CellDev& cd = *cdp;
  if (!cd.active) return;
  const int i = bb.y * kBlock + threadIdx.x;
  double dmax = 0.0;
  if (i < cd.N) {
  const size_t N = cd.N;
  const double* x = cd.x;
  const uint32_t mi = cd.meta[i];
  const int L = lab_of(mi);
  const double xc = x[i], xp = x[N + i];
  cd.dc[i] = cref_of(cd, L) * xc;
  cd.dp[i] = cd.VT * xp;
  dmax = fmax(fabs(xc), fabs(xp));
  if (!isfinite(dmax)) dmax = INFINITY;
  if (L == ANODE && !cd.elim_n) {
    const VoxCoord v = coord_of(cd, i);
    const uint32_t msk = mask_of(mi);
    const KT* can = (const KT*)cd.coef_an;
    for (int d = 0; d < 6; ++d) {
      if (!((msk >> d) & 1u)) continue;
      const int k = neighbour(cd, i, v.x, v.y, v.z, d);
      const uint32_t f = face_rank(mi, d);
      double dn = -cd.rn_jnn[f];
      if (cd.plating) {
        const KT* co = can + 5 * (size_t)f;
        const double qp = (double)co[3] * (double)x[k] + (double)co[4] * (xp - (double)x[N + k]);
        dn -= cd.dt * cd.mu_ref / kFaraday * qp;
      }
      cd.dn[f] = dn;
      dmax = fmax(dmax, fabs(dn) / cd.n_c);
    }
  }
  }
  // scaled max-norm of the full Newton step (step-length limiter)
  const double vals[1] = {dmax};
  reduce_block<1>(cd, bb.y, vals, 0x1u);
}

// Trial state u + lam du; counts inadmissible entries (c <= 0, c_s >= c_max,
// n < 0, non-finite) and the scaled max-norm of the step.
__global__ void __launch_bounds__(kBlock) k_trial(CellDev* cells, const int2* __restrict__ blk) {
  const int2 bb = block_of(blk);
  CellDev* cdp = cells + bb.x;
  const CellDev& cd = *cdp;
  if (!cd.active) return;
  const int i = bb.y * kBlock + threadIdx.x;
  double bad = 0.0, dmax = 0.0;
  if (i < cd.N) {
    const uint32_t mi = cd.meta[i];
    const int L = lab_of(mi);
    const double lam = cd.lam;
    const double c0 = cd.c[i];
    const double cref = cref_of(cd, L);
    // fraction to the boundary, per voxel: a concentration moves at most 90%
    // of the way to 0 (or, in a solid, to c_max) in one iteration, so that a
    // few voxels near depletion do not shrink the whole step
    double c = c0 + lam * cd.dc[i];
    c = fmax(c, kToBoundary * c0);
    if (L != PORE) c = fmin(c, cref - kToBoundary * (cref - c0));
    const double p = cd.phi[i] + lam * cd.dp[i];
    cd.c_try[i] = c;
    cd.phi_try[i] = p;
    if (!(c > 0.0) || !isfinite(p) || (L != PORE && !(c < cref))) bad += 1.0;
    dmax = fmax(fabs(c - c0) / cref, fabs(lam * cd.dp[i]) / cd.VT);
    if (!isfinite(dmax)) bad += 1.0;
    if (L == ANODE && !cd.elim_n) {
      const uint32_t cnt = __popc(mask_of(mi));
      for (uint32_t r = 0; r < cnt; ++r) {
        const uint32_t f = base_of(mi) + r;
        const double nn = cd.n[f] + lam * cd.dn[f];
        cd.n_try[f] = nn;
        if (!(nn >= 0.0)) bad += 1.0;
        dmax = fmax(dmax, fabs(lam * cd.dn[f]) / cd.n_c);
      }
    }
  }
  const double vals[2] = {bad, dmax};
  reduce_block<2>(cd, bb.y, vals, 0x2u);
}

// Local-error indicator of an adaptive step (differential unknowns only):
// max |u - (u_old + w (u_old - u_prev))| over the concentrations (relative to
// c0 / c_max) and the plated amounts (relative to n_c), w = dt / dt_prev.
__global__ void __launch_bounds__(kBlock) k_lte(CellDev* cells, const int2* __restrict__ blk, double w) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active) return;
  const int i = bb.y * kBlock + threadIdx.x;
  double e = 0.0;
  if (i < cd.N) {
    const uint32_t mi = cd.meta[i];
    const int L = lab_of(mi);
    const double co = cd.c_old[i];
    e = fabs(cd.c[i] - (co + w * (co - cd.c_prev[i]))) / cref_of(cd, L);
    if (L == ANODE) {
      const uint32_t cnt = __popc(mask_of(mi));
      for (uint32_t r = 0; r < cnt; ++r) {
        const uint32_t f = base_of(mi) + r;
        const double no = cd.n_old[f];
        e = fmax(e, fabs(cd.n[f] - (no + w * (no - cd.n_prev[f]))) / cd.n_c);
      }
    }
  }
  const double vals[1] = {e};
  reduce_block<1>(cd, bb.y, vals, 0x1u);
}

// State copies: 0 try -> iterate, 1 iterate -> try, 2 iterate -> old (step
// start), 3 old -> iterate and try (rollback), 4 old -> try (step start),
// 5 old -> previous (an adaptive run's history; concentrations and plated
// amounts).
__global__ void __launch_bounds__(kBlock) k_copy_state(CellDev* cells, const int2* __restrict__ blk, int mode) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active) return;
  const int i = bb.y * kBlock + threadIdx.x;
  if (i >= cd.N) return;
  const uint32_t mi = cd.meta[i];
  const int L = lab_of(mi);
  const uint32_t cnt = (L == ANODE) ? __popc(mask_of(mi)) : 0u;
  const uint32_t f0 = base_of(mi);
  const double *sc, *sp, *sn;
  double *dc, *dp, *dn;
  double *dc2 = nullptr, *dp2 = nullptr, *dn2 = nullptr;
  switch (mode) {
    case 0: sc = cd.c_try; sp = cd.phi_try; sn = cd.n_try; dc = cd.c; dp = cd.phi; dn = cd.n; break;
    case 1: sc = cd.c; sp = cd.phi; sn = cd.n; dc = cd.c_try; dp = cd.phi_try; dn = cd.n_try; break;
    case 2: sc = cd.c; sp = cd.phi; sn = cd.n; dc = cd.c_old; dp = cd.phi_old; dn = cd.n_old; break;
    case 3:
      sc = cd.c_old; sp = cd.phi_old; sn = cd.n_old; dc = cd.c; dp = cd.phi; dn = cd.n;
      dc2 = cd.c_try; dp2 = cd.phi_try; dn2 = cd.n_try;
      break;
    case 5: {
      cd.c_prev[i] = cd.c_old[i];
      for (uint32_t r = 0; r < cnt; ++r) cd.n_prev[f0 + r] = cd.n_old[f0 + r];
      return;
    }
    default: sc = cd.c_old; sp = cd.phi_old; sn = cd.n_old; dc = cd.c_try; dp = cd.phi_try; dn = cd.n_try; break;
  }
  dc[i] = sc[i];
  dp[i] = sp[i];
  if (dc2) {
    dc2[i] = sc[i];
    dp2[i] = sp[i];
  }
  for (uint32_t r = 0; r < cnt; ++r) {
    dn[f0 + r] = sn[f0 + r];
    if (dn2) dn2[f0 + r] = sn[f0 + r];
  }
}

// Output functionals of the iterate (Sec. 2.5: linear functionals of the
// state): Li inventories per phase and the plated layer, and the sum over
// cathode collector faces of the extrapolated collector potential.
__global__ void __launch_bounds__(kBlock) k_outputs(CellDev* cells, const int2* __restrict__ blk) {
  const int2 bb = block_of(blk);
  CellDev* cdp = cells + bb.x;
  const CellDev& cd = *cdp;
  if (!cd.active) return;
  const int i = bb.y * kBlock + threadIdx.x;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (i < cd.N) {
    const uint32_t mi = cd.meta[i];
    const int L = lab_of(mi);
    v[L] = cd.c[i] * cd.Vol;
    if (L == ANODE) {
      const uint32_t cnt = __popc(mask_of(mi));
      double s = 0.0;
      for (uint32_t r = 0; r < cnt; ++r) s += cd.n[base_of(mi) + r];
      v[3] = s * cd.A;
    }
    const int z = i / (cd.nx * cd.ny);
    if (L == CATHODE && z == cd.nz - 1) {
      const double jout = -cd.I_app / (cd.n_top * cd.A);
      v[4] = cd.phi[i] - jout * cd.h / (2.0 * cd.sigma[1]);
    }
  }
  reduce_block<5>(cd, bb.y, v, 0u);
}

// Conversions between the raw FP64 scratch pair (dc, dp: 2N contiguous
// doubles) and a Krylov vector: dir 0 doubles -> KT vector, 1 KT -> doubles.
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_convert(CellDev* cells, const int2* __restrict__ blk, int sel, int dir) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  const int i = bb.y * kBlock + threadIdx.x;
  if (i >= cd.N) return;
  const size_t N = cd.N;
  if (sel == VEC_X) {   // the iterate is FP64 in both modes
    if (dir == 0) {
      cd.x[i] = cd.dc[i];
      cd.x[N + i] = cd.dp[i];
    } else {
      cd.dc[i] = cd.x[i];
      cd.dp[i] = cd.x[N + i];
    }
    return;
  }
  KT* v = vec<KT>(cd, sel);
  if (dir == 0) {
    v[i] = (KT)cd.dc[i];
    v[N + i] = (KT)cd.dp[i];
  } else {
    cd.dc[i] = (double)v[i];
    cd.dp[i] = (double)v[N + i];
  }
}

// x = 0 (start of a solve from a given right-hand side)
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_zero_x(CellDev* cells, const int2* __restrict__ blk) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active) return;
  const int i = bb.y * kBlock + threadIdx.x;
  if (i >= cd.N) return;
  double* x = cd.x;
  x[i] = 0.0;
  x[(size_t)cd.N + i] = 0.0;
}

// ||w||^2 into RED_BSQ
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_norm_w(CellDev* cells, const int2* __restrict__ blk) {
  const int2 bb = block_of(blk);
  CellDev* cdp = cells + bb.x;
  const CellDev& cd = *cdp;
  if (!cd.active) return;
  const int i = bb.y * kBlock + threadIdx.x;
  double ss = 0.0;
  if (i < cd.N) {
    const KT* w = (const KT*)cd.w;
    const double a = (double)w[i], b = (double)w[(size_t)cd.N + i];
    ss = a * a + b * b;
  }
  const double vals[1] = {ss};
  reduce_block<1>(cd, bb.y, vals, 0u);
}

// --------------------------------------------------------------- launchers
static inline dim3 grid_of(int nblk) { return dim3((unsigned)nblk); }

void launch_build_meta(const uint8_t* lab, int nx, int ny, int nz, uint32_t* meta, int* cnt_an, int* cnt_ca,
                       int* flags, hipStream_t s) {
  const int N = nx * ny * nz;
  k_build_meta<<<(N + kBlock - 1) / kBlock, kBlock, 0, s>>>(lab, nx, ny, nz, meta, cnt_an, cnt_ca, flags);
}
void launch_finish_meta(int N, uint32_t* meta, const int* off_an, const int* off_ca, int* faces_an, int* faces_ca,
                        hipStream_t s) {
  k_finish_meta<<<(N + kBlock - 1) / kBlock, kBlock, 0, s>>>(N, meta, off_an, off_ca, faces_an, faces_ca);
}
hipError_t exclusive_scan(void* temp, size_t& temp_bytes, const int* in, int* out, int n, hipStream_t s) {
  return rocprim::exclusive_scan(temp, temp_bytes, in, out, 0, (size_t)n, rocprim::plus<int>(), s);
}
void launch_meta_rb(const CellDev& cd, int* cnt, hipStream_t s) {
  (void)hipMemsetAsync((void*)cd.meta_rb, 0, 8 * (size_t)cd.rbH, s);
  (void)hipMemsetAsync(cnt, 0, 8 * (size_t)cd.rbH, s);
  k_meta_rb<<<(cd.N + kBlock - 1) / kBlock, kBlock, 0, s>>>(cd, cnt);
}

void launch_meta_rb_base(const CellDev& cd, const int* off, hipStream_t s) {
  k_meta_rb_base<<<(2 * cd.rbH + kBlock - 1) / kBlock, kBlock, 0, s>>>(cd, off);
}
void launch_init_state(const BatchLaunch& b, hipStream_t s) {
  k_init_state<<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk);
}

template <typename KT>
void launch_residual(const BatchLaunch& b, bool lin, hipStream_t s) {
  prof_begin(PK_RESIDUAL, s);
  // a single cell launches only the blocks its faces need; a batch uses the
  // voxel block table and strides each cell's faces over its own blocks
  const int fgrid = b.blk ? b.nblk : std::max(1, std::min(b.nblk, (b.faces_single + kBlock - 1) / kBlock));
  const int stride = b.blk ? 0 : fgrid;
  if (lin) {
    k_iface<true, KT><<<grid_of(fgrid), kBlock, 0, s>>>(b.cells, b.blk, stride);
    k_residual<true, KT><<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk);
  } else {
    k_iface<false, KT><<<grid_of(fgrid), kBlock, 0, s>>>(b.cells, b.blk, stride);
    k_residual<false, KT><<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk);
  }
  if (prof_on(PK_RESIDUAL)) prof_end(PK_RESIDUAL, s, b.bytes_residual[lin ? 1 : 0]);
  k_finalize_red<<<b.ncell, kBlock, 0, s>>>(b.cells, b.ncell, RED_RSQ, 4, 0xAu, -3);
}
template <typename KT>
void launch_rhs(const BatchLaunch& b, hipStream_t s) {
  k_rhs<KT><<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk);
  k_finalize_red<<<b.ncell, kBlock, 0, s>>>(b.cells, b.ncell, RED_BSQ, 1, 0u, -3);
}
template <typename KT>
void launch_matvec(const BatchLaunch& b, int src, int dst, int need, int keep, hipStream_t s) {
  prof_begin(PK_MATVEC, s);
  const int bs = b.blk ? kBlock : b.bs_matvec;
  if (bs == 64)
    k_matvec<KT, 64><<<(b.n_single + 63) / 64, 64, 0, s>>>(b.cells, nullptr, src, dst, need, keep);
  else if (bs == 128)
    k_matvec<KT, 128><<<(b.n_single + 127) / 128, 128, 0, s>>>(b.cells, nullptr, src, dst, need, keep);
  else if (bs == 512)
    k_matvec<KT, 512><<<(b.n_single + 511) / 512, 512, 0, s>>>(b.cells, nullptr, src, dst, need, keep);
  else if (bs == 1024)
    k_matvec<KT, 1024><<<(b.n_single + 1023) / 1024, 1024, 0, s>>>(b.cells, nullptr, src, dst, need, keep);
  else
    k_matvec<KT, kBlock><<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk, src, dst, need, keep);
  if (prof_on(PK_MATVEC)) prof_end(PK_MATVEC, s, b.bytes_matvec);
}
template <typename KT>
void launch_multidot(const BatchLaunch& b, int k, int tgt, hipStream_t s) {
  k_multidot<KT><<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk, k);
  k_finalize_dots<<<dim3(k + 1, b.ncell), kBlock, 0, s>>>(b.cells, b.ncell, k, tgt);
}
template <typename KT>
void launch_orth_dots(const BatchLaunch& b, int k, hipStream_t s) {
  k_orth_dots<KT><<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk, k);
  k_finalize_dots<<<dim3(k + 1, b.ncell), kBlock, 0, s>>>(b.cells, b.ncell, k, 1);
}
template <typename KT>
void launch_orth(const BatchLaunch& b, int k, int src, hipStream_t s) {
  k_orth<KT><<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk, k, src);
  k_finalize_norm<<<b.ncell, kBlock, 0, s>>>(b.cells, b.ncell, k, src);
}
template <typename KT>
void launch_scale_next(const BatchLaunch& b, int k, hipStream_t s) {
  k_scale_next<KT><<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk, k);
}
void launch_backsolve(const BatchLaunch& b, hipStream_t s) {
  k_backsolve<<<(b.ncell + 63) / 64, 64, 0, s>>>(b.cells, b.ncell);
}
template <typename KT>
void launch_update_x(const BatchLaunch& b, hipStream_t s) {
  k_update_x<KT><<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk);
}
template <typename KT>
void launch_true_residual(const BatchLaunch& b, hipStream_t s) {
  k_true_residual<KT><<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk);
  k_finalize_red<<<b.ncell, kBlock, 0, s>>>(b.cells, b.ncell, RED_BSQ, 1, 0u, sizeof(KT) < sizeof(double) ? -4 : 2);
}
template <typename KT>
void launch_gm_start(const BatchLaunch& b, int first, hipStream_t s) {
  k_gm_start<KT><<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk, first);
}
void launch_gm_flags(const BatchLaunch& b, int first, int refine, hipStream_t s) {
  k_gm_flags<<<(b.ncell + 63) / 64, 64, 0, s>>>(b.cells, b.ncell, first, refine);
}
void launch_gather_ctl(const BatchLaunch& b, double* out, hipStream_t s) {
  k_gather_ctl<<<(b.ncell + 63) / 64, 64, 0, s>>>(b.cells, b.ncell, out);
}
template <typename KT>
void launch_zero_x(const BatchLaunch& b, hipStream_t s) {
  k_zero_x<KT><<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk);
}
template <typename KT>
void launch_norm_w(const BatchLaunch& b, hipStream_t s) {
  k_norm_w<KT><<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk);
  k_finalize_red<<<b.ncell, kBlock, 0, s>>>(b.cells, b.ncell, RED_BSQ, 1, 0u, -3);
}
template <typename KT>
void launch_convert(const BatchLaunch& b, int sel, int dir, hipStream_t s) {
  k_convert<KT><<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk, sel, dir);
}
template <typename KT>
void launch_direction(const BatchLaunch& b, hipStream_t s) {
  k_direction<KT><<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk);
  k_finalize_red<<<b.ncell, kBlock, 0, s>>>(b.cells, b.ncell, RED_DUMAX, 1, 0x1u, -3);
}
void launch_trial(const BatchLaunch& b, hipStream_t s) {
  k_trial<<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk);
  k_finalize_red<<<b.ncell, kBlock, 0, s>>>(b.cells, b.ncell, RED_BAD, 2, 0x2u, -3);
}
void launch_copy_state(const BatchLaunch& b, int mode, hipStream_t s) {
  k_copy_state<<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk, mode);
}
void launch_lte(const BatchLaunch& b, double w, hipStream_t s) {
  k_lte<<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk, w);
  k_finalize_red<<<b.ncell, kBlock, 0, s>>>(b.cells, b.ncell, RED_LTE, 1, 0x1u, -3);
}
void launch_outputs(const BatchLaunch& b, hipStream_t s) {
  k_outputs<<<grid_of(b.nblk), kBlock, 0, s>>>(b.cells, b.blk);
  k_finalize_red<<<b.ncell, kBlock, 0, s>>>(b.cells, b.ncell, RED_INV0, 5, 0u, -3);
}

#define MBX_INST(KT)                                                             \
  template void launch_residual<KT>(const BatchLaunch&, bool, hipStream_t);      \
  template void launch_rhs<KT>(const BatchLaunch&, hipStream_t);                 \
  template void launch_matvec<KT>(const BatchLaunch&, int, int, int, int, hipStream_t);  \
  template void launch_convert<KT>(const BatchLaunch&, int, int, hipStream_t);      \
  template void launch_zero_x<KT>(const BatchLaunch&, hipStream_t);                  \
  template void launch_norm_w<KT>(const BatchLaunch&, hipStream_t);                  \
  template void launch_multidot<KT>(const BatchLaunch&, int, int, hipStream_t);  \
  template void launch_orth<KT>(const BatchLaunch&, int, int, hipStream_t);      \
  template void launch_orth_dots<KT>(const BatchLaunch&, int, hipStream_t);     \
  template void launch_scale_next<KT>(const BatchLaunch&, int, hipStream_t);     \
  template void launch_update_x<KT>(const BatchLaunch&, hipStream_t);            \
  template void launch_true_residual<KT>(const BatchLaunch&, hipStream_t);       \
  template void launch_gm_start<KT>(const BatchLaunch&, int, hipStream_t);       \
  template void launch_direction<KT>(const BatchLaunch&, hipStream_t);
MBX_INST(float)
MBX_INST(double)
#undef MBX_INST

}  // namespace mbx
