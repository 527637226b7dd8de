// mg.hip — preconditioner of the Newton correction system.
//
// The scaled Jacobian J couples concentrations and potentials.  The
// preconditioner (1) removes the migration coupling from the pore
// concentration rows with the row operation c-row -= tau * phi-row (in the
// bulk electrolyte the t+ j/F flux then cancels exactly), (2) solves the
// concentration block (mass + same-phase diffusion, symmetric positive
// definite), (3) solves the potential block (conduction in each phase plus
// Butler-Volmer and plating conductances across solid/pore faces: a
// symmetric weighted graph Laplacian, pinned by the anode collector) with
// the concentration coupling moved to the right-hand side.  Each block is
// solved approximately by one multigrid V-cycle: aggregates are 2x2x2 voxel
// blocks split by phase (a coarse cell holds up to three slots: pore, anode,
// cathode), coarse operators are Galerkin sums with piecewise-constant
// transfer, smoothing is red-black Gauss-Seidel, the coarse correction is
// scaled by alpha, and the coarsest level is solved with a dense inverse.
// Phase-respecting aggregates keep the near-null modes of the potential
// operator (a constant potential per phase, tied only by the weak interface
// conductances) exactly representable on every level.
#include <hip/hip_runtime.h>


#include <algorithm>

#include "mbx_dev.h"
#include "mbx_kernels.h"
#include "prof.h"

namespace mbx {

namespace {

__device__ inline int xidx(int s, int t) { return s + t - 1; }   // (0,1)->0 (0,2)->1 (1,2)->2

template <typename KT>
struct OpV {
  const KT* p;
  int n;
  __device__ KT E(int c, int s) const { return p[(size_t)s * n + c]; }
  __device__ KT X(int c, int k) const { return p[(size_t)(3 + k) * n + c]; }
  __device__ KT G(int c, int dir, int s, int t) const { return p[(size_t)(6 + dir * 9 + s * 3 + t) * n + c]; }
};

// run gate for preconditioner kernels: need >= 0 -> GMRES state == need;
// need == -1 -> cycle end (state 1 or 2); need == -2 -> always.
__device__ inline bool gate(const CellDev& cd, int need) {
  if (!cd.active) return false;
  if (need == -2) return true;
  const int st = cd.ictl[CTL_DONE];
  if (need == -1) return st == 1 || st == 2;
  return st == need;
}
// The GMRES-state part of the gate alone.  Hot kernels test cd.active first,
// issue their loads, and test this only before their stores, so the flag load
// overlaps the data loads instead of preceding them.
__device__ inline bool gate_state(const CellDev& cd, int need) {
  if (need == -2) return true;
  const int st = cd.ictl[CTL_DONE];
  if (need == -1) return st == 1 || st == 2;
  return st == need;
}

template <typename KT>
__device__ inline KT* vsel(const CellDev& cd, int sel) {
  const size_t n2 = 2 * (size_t)cd.N;
  switch (sel) {
    case VEC_Z: return (KT*)cd.z;
    case VEC_W: return (KT*)cd.w;
    case VEC_B: return (KT*)cd.b;
    default: return (KT*)cd.Vb + (size_t)sel * n2;
  }
}

struct C3 {
  int x, y, z;
};
__device__ inline C3 c3_of(int i, int nx, int ny, double inv_nx, double inv_ny) {
  C3 c;
  c.z = divmod(divmod(i, nx, inv_nx, c.x), ny, inv_ny, c.y);
  return c;
}

// Level-0 conductance of the face between voxel i (label L) and its
// neighbour k (label Lk) in direction d, for operator op (0 concentration,
// 1 potential).  Zero when the operator does not couple the two voxels.
template <typename KT>
__device__ inline KT fine_cond(const CellDev& cd, int op, int L, int Lk, uint32_t mi, uint32_t mk, int d) {
  if (L == Lk) {
    if (op == 0) return (KT)(L == PORE ? cd.Dh : cd.Dsh[L - 1]);
    return (KT)(L == PORE ? cd.Gk : cd.Gs[L - 1]);
  }
  if (op == 0 || (L != PORE && Lk != PORE)) return (KT)0;
  if (L == PORE) {
    const uint32_t f = face_rank(mk, d ^ 1);
    return Lk == ANODE ? ((const KT*)cd.cond_an)[f] : ((const KT*)cd.cond_ca)[f];
  }
  const uint32_t f = face_rank(mi, d);
  return L == ANODE ? ((const KT*)cd.cond_an)[f] : ((const KT*)cd.cond_ca)[f];
}

template <typename KT>
__device__ inline KT fine_extra(const CellDev& cd, int op, int L, int z) {
  if (op == 0) return (KT)1;
  return (L == ANODE && z == 0) ? (KT)cd.Gcol : (KT)0;
}

// Interface part of the concentration operator's diagonal at voxel i, face
// (neighbour label Lk, direction d from i): the own-concentration derivative
// of the Butler-Volmer / plating molar flux through that face, in the rows of
// the preconditioned system (solid rows as they are, pore rows after the
// migration row operation, which scales them by -(1 - t+)).  Negative values
// are dropped so the block stays positive definite.  Near a depleted particle
// surface the open-circuit-potential slope makes this term dominate the row.
template <typename KT>
__device__ inline KT c_iface_term(const CellDev& cd, int L, int Lk, uint32_t mi, uint32_t mk, int d) {
  const bool iface = (L == PORE) != (Lk == PORE);
  if (!iface) return (KT)0;
  const bool pore_side = L == PORE;
  const uint32_t f = face_rank(pore_side ? mk : mi, pore_side ? (d ^ 1) : d);
  const bool an = (pore_side ? Lk : L) == ANODE;
  const KT* co = an ? (const KT*)cd.coef_an + 5 * (size_t)f : (const KT*)cd.coef_ca + 3 * (size_t)f;
  KT v;
  if (pore_side) {
    const KT d_ce = co[1] + (an ? co[3] : (KT)0);
    v = (KT)(cd.tau - cd.Ke) * d_ce;
  } else {
    v = (KT)cd.Ks[L == CATHODE] * co[0];
  }
  return v > (KT)0 ? v : (KT)0;
}

__device__ inline int fine_nbr(int i, const C3& c, int nx, int ny, int nz, int d) {
  switch (d) {
    case 0: return c.x > 0 ? i - 1 : -1;
    case 1: return c.x < nx - 1 ? i + 1 : -1;
    case 2: return c.y > 0 ? i - nx : -1;
    case 3: return c.y < ny - 1 ? i + nx : -1;
    case 4: return c.z > 0 ? i - nx * ny : -1;
    default: return c.z < nz - 1 ? i + nx * ny : -1;
  }
}

// Storage order of a coarse level (l >= 1): rows of nx cells ((y, z) in
// row-major order), and inside each row the even-x cells first, then the
// odd-x cells.  A red-black half sweep visits one x-parity per row, whose
// cells are then contiguous (whole cache lines instead of every other
// element); the +-y and +-z neighbours keep the strides nx and nx*ny.
__device__ inline int xperm(int x, int nx) { return (x >> 1) + (x & 1) * ((nx + 1) >> 1); }
// (non-negative coordinates inside the level; the products fit the 24-bit
// multiplier under the grid limits nx, ny <= 2^21 and ny*nz <= 2^23)
__device__ inline int lvl_index(int x, int y, int z, int nx, int ny) {
  return xperm(x, nx) + (int)__umul24((unsigned)nx, (unsigned)(y + (int)__umul24((unsigned)ny, (unsigned)z)));
}
__device__ inline int lvl_cell(const MGLevel& L, int x, int y, int z) { return lvl_index(x, y, z, L.nx, L.ny); }
// coordinates of the cell stored at index c
__device__ inline C3 lvl_coords(int c, const MGLevel& G) {
  C3 q = c3_of(c, G.nx, G.ny, G.inv_nx, G.inv_ny);   // q.x: position in the row
  const int he = (G.nx + 1) >> 1;
  q.x = q.x < he ? 2 * q.x : 2 * (q.x - he) + 1;
  return q;
}
// index of the cell dx in {-1, 0, 1} cells along x from cell c at x
__device__ inline int lvl_xstep(int c, int x, int dx, int nx) { return c - xperm(x, nx) + xperm(x + dx, nx); }

// Smoothing modes: which values stand for the cell's own slots and for its
// neighbours.  "corrected" adds alpha times the parent's level l+1 solution
// (the coarse-grid correction applied lazily on the first post-sweeps).
enum { SM_PLAIN = 0, SM_ZERO = 1, SM_CORR = 2, SM_OWNZERO = 3, SM_OWNCORR = 4 };
__device__ inline bool own_zero(int m) { return m == SM_ZERO || m == SM_OWNZERO; }
__device__ inline bool own_corr(int m) { return m == SM_CORR || m == SM_OWNCORR; }
__device__ inline bool nbr_zero(int m) { return m == SM_ZERO; }
__device__ inline bool nbr_corr(int m) { return m == SM_CORR; }

// Red-black thread mapping: thread t of a level with extents (nx, ny, nz)
// handles the t-th cell of colour `color` ((x + y + z) & 1 == color) in
// row-major order; false when t is past the end.
__device__ inline bool color_cell(int t, int color, int nx, int ny, int nz, double inv_hx, double inv_ny, C3& q) {
  const int hx = (nx + 1) >> 1;
  int j;
  const int row = divmod(t, hx, inv_hx, j);
  q.z = divmod(row, ny, inv_ny, q.y);
  q.x = 2 * j + ((color + q.y + q.z) & 1);
  return q.z < nz && q.x < nx;
}
__device__ inline bool color_cell(int t, int color, const MGLevel& L, C3& q) {
  return color_cell(t, color, L.nx, L.ny, L.nz, L.inv_hx, L.inv_ny, q);
}

// Neighbour cells (+x, -x, +y, -y, +z, -z) of cell c at q; absent neighbours
// are replaced by c itself and flagged false (their couplings are zeroed, so
// every load stays in bounds and can be issued without a branch).  Natural
// order (the voxel grid).
__device__ inline void neighbours6(int c, const C3& q, int nx, int ny, int nz, int (&nb)[6], bool (&ex)[6]) {
  const int sx = 1, sy = nx, sz = nx * ny;
  ex[0] = q.x + 1 < nx; ex[1] = q.x > 0;
  ex[2] = q.y + 1 < ny; ex[3] = q.y > 0;
  ex[4] = q.z + 1 < nz; ex[5] = q.z > 0;
  nb[0] = ex[0] ? c + sx : c; nb[1] = ex[1] ? c - sx : c;
  nb[2] = ex[2] ? c + sy : c; nb[3] = ex[3] ? c - sy : c;
  nb[4] = ex[4] ? c + sz : c; nb[5] = ex[5] ? c - sz : c;
}
// The same for a coarse level's storage order (lvl_index).
__device__ inline void lvl_neighbours6(int c, const C3& q, int nx, int ny, int nz, int (&nb)[6], bool (&ex)[6]) {
  const int sy = nx, sz = nx * ny;
  ex[0] = q.x + 1 < nx; ex[1] = q.x > 0;
  ex[2] = q.y + 1 < ny; ex[3] = q.y > 0;
  ex[4] = q.z + 1 < nz; ex[5] = q.z > 0;
  nb[0] = ex[0] ? lvl_xstep(c, q.x, 1, nx) : c; nb[1] = ex[1] ? lvl_xstep(c, q.x, -1, nx) : c;
  nb[2] = ex[2] ? c + sy : c; nb[3] = ex[3] ? c - sy : c;
  nb[4] = ex[4] ? c + sz : c; nb[5] = ex[5] ? c - sz : c;
}

// Row of the level-0 operator OP at voxel c (colour-split index p, colour
// `color`): diagonal D (extra term plus all couplings) and
// S = sum_k g_ik x_k over the neighbours (x_k read from the colour-split
// iterate xsrc, plus alpha times the level-1 solution of k's slot when corr).
// The voxel's own interface mask tells same-phase neighbours from interface
// ones (anode and cathode never touch); the potential operator's interface
// conductances come from the voxel's own list in cond_rb, whose sign also
// gives a pore voxel its solid neighbour's phase.  Every load is a buffer
// load issued before any arithmetic depends on it; absent neighbours and
// faces the voxel does not have are read at kNoOff (zero).
template <typename KT, int OP>
__device__ inline void voxel_row(const CellDev& cd, int color, int p, const C3& c, uint32_t mi,
                                 const KT* __restrict__ xsrc, bool zero, bool corr, KT& D, KT& S) {
  constexpr uint32_t kt = sizeof(KT);
  // colour-split neighbours (+x, -x, +y, -y, +z, -z): the other colour, at
  // q0 = the slot of (x, y, z) in that colour's rows (p's slot, moved by
  // one colour block: both colours index rows and columns alike)
  const int hx = cd.rbhx;
  const int q0 = p + (1 - 2 * color) * cd.rbH;
  const int odd = c.x & 1;
  bool ex[6];
  ex[0] = c.x + 1 < cd.nx; ex[1] = c.x > 0;
  ex[2] = c.y + 1 < cd.ny; ex[3] = c.y > 0;
  ex[4] = c.z + 1 < cd.nz; ex[5] = c.z > 0;
  const int kq[6] = {q0 + odd, q0 + odd - 1, q0 + hx, q0 - hx, q0 + cd.ny * hx, q0 - cd.ny * hx};
  const int dmap[6] = {1, 0, 3, 2, 5, 4};   // neighbour slot -> face direction (0:-x 1:+x ...)
  const int L = lab_of(mi);
  const bool pore = L == PORE;
  const uint32_t msk = mask_of(mi);
  bool ifc[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) ifc[j] = (msk >> dmap[j]) & 1u;   // set only for existing neighbours
  KT xk[6], gf[6];
  if (!zero) {
    const BufRes rx = buf_of(xsrc, 2u * (uint32_t)cd.rbH * kt);
#pragma unroll
    for (int j = 0; j < 6; ++j) xk[j] = buf_ld<KT>(rx, ex[j] ? (uint32_t)kq[j] * kt : kNoOff);
  } else {
#pragma unroll
    for (int j = 0; j < 6; ++j) xk[j] = (KT)0;
  }
  if (OP != 0) {
    const uint32_t F = (uint32_t)(cd.F_an + cd.F_ca);
    const BufRes rc = buf_of((const KT*)cd.cond_rb + (size_t)color * F, F * kt);
    const uint32_t fb = base_of(mi);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const uint32_t r = (uint32_t)__popc(msk & ((1u << dmap[j]) - 1u));
      gf[j] = buf_ld<KT>(rc, ifc[j] ? (fb + r) * kt : kNoOff);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 6; ++j) gf[j] = (KT)0;
  }
  // interface part of the concentration diagonal (per voxel, from the setup)
  const KT dint = OP == 0 ? buf_ld<KT>(buf_of(cd.dint, 2u * (uint32_t)cd.rbH * kt), (uint32_t)p * kt) : (KT)0;
  // same-phase coupling (per-cell constants in the Krylov type, selected by label)
  const Gsame<KT> gs = gsame_of<KT>(cd, OP);
  const KT gsame = pore ? gs.pore : (L == CATHODE ? gs.ca : gs.an);
  KT g[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const KT v = ifc[j] ? (OP == 0 ? (KT)0 : (KT)fabs(gf[j])) : gsame;
    g[j] = ex[j] ? v : (KT)0;
  }
  if (corr) {
    const MGLevel& L1 = cd.lv[1];
    const KT alpha = (KT)cd.alpha;
    const BufRes r1 = buf_of(L1.x, 3u * (uint32_t)L1.ncell * kt);
    const int px = c.x >> 1, py = c.y >> 1, pz = c.z >> 1;
    const int pq[6] = {((c.x + 1) >> 1) - px, ((c.x - 1) >> 1) - px, ((c.y + 1) >> 1) - py,
                       ((c.y - 1) >> 1) - py, ((c.z + 1) >> 1) - pz, ((c.z - 1) >> 1) - pz};
    const int pc = lvl_cell(L1, px, py, pz);
    const int pst[6] = {0, 0, L1.nx, L1.nx, L1.nx * L1.ny, L1.nx * L1.ny};   // x steps: lvl_xstep
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      // the neighbour's phase slot (an interface neighbour of the
      // concentration operator has a zero coupling: its own slot serves)
      const int ns = pore ? (__builtin_signbit(gf[j]) ? CATHODE : ANODE) : PORE;
      const int slot = (OP != 0 && ifc[j]) ? ns : L;
      const int pcj = j < 2 ? lvl_xstep(pc, px, pq[j], L1.nx) : pc + pq[j] * pst[j];
      const uint32_t off = (uint32_t)(slot * L1.ncell + pcj) * kt;
      const KT cv = alpha * buf_ld<KT>(r1, ex[j] ? off : kNoOff);   // rounded before the sum (no fused form)
      xk[j] += cv;
    }
  }
  D = OP == 0 ? (KT)1 + dint : ((L == ANODE && c.z == 0) ? (KT)cd.Gcol : (KT)0);
  S = (KT)0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    D += g[j];
    S += g[j] * xk[j];   // xk = 0 from a zero iterate: S stays +0 (the couplings are finite)
  }
}

// Gathered row block of coarse cell C at level l: the 3x3 in-cell couplings,
// the couplings to the six neighbours and the neighbour values, loaded
// without branches (absent neighbours read cell C with zero couplings).
// A coarse level as the smoother sees it: extents, the vectors and the
// operator being solved (typed pointers, in device memory or in LDS).
template <typename KT>
struct LV {
  int nx, ny, nz, ncell;
  KT* x;
  KT* b;
  const KT* A;
  int op;   // 0: concentration operator (same-slot couplings only), 1: potential operator
};
template <typename KT>
__device__ inline LV<KT> view(const MGLevel& L, int op) {
  return LV<KT>{L.nx, L.ny, L.nz, L.ncell, (KT*)L.x, (KT*)L.b, (const KT*)L.op[op], op};
}

// Couplings that are zero by construction and never loaded: the
// concentration operator couples only equal slots (no cross-phase transport);
// anode and cathode never share a face, so slots 1 and 2 are never coupled.
__host__ __device__ constexpr bool cross_zero(int s, int t) { return (s == 1 && t == 2) || (s == 2 && t == 1); }

template <typename KT>
struct CoarseRow {
  KT E[3], X[3], b[3], xo[3];
  KT Gp[3][9], Gm[3][9];   // Gp[dir][s*3+t]: own slot s to slot t of the +dir neighbour; Gm from -dir neighbour
  KT xn[6][3];
};

// L: the level, Lp: the next coarser level (read in the corrected modes),
// alpha: the coarse-correction factor.  The level descriptors may point into
// device memory or into LDS.
template <typename KT, int OP>
__device__ inline void gather_coarse(const LV<KT>& L, const LV<KT>& Lp, KT alpha, int C, const C3& q, int mode,
                                     CoarseRow<KT>& R) {
  const size_t n = L.ncell;
  const KT* A = L.A;
  const KT* b = L.b;
  const KT* x = L.x;
  int nb[6];
  bool ex[6];
  lvl_neighbours6(C, q, L.nx, L.ny, L.nz, nb, ex);
  constexpr bool cross = OP != 0;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    R.E[s] = A[s * n + C];
    R.X[s] = (cross && s != 2) ? A[(3 + s) * n + C] : (KT)0;   // X pairs (0,1) (0,2) (1,2)
    R.b[s] = b[s * n + C];
  }
#pragma unroll
  for (int dir = 0; dir < 3; ++dir)
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int s = k / 3, t = k % 3;
      KT gp = (KT)0, gm = (KT)0;
      if (s == t || (cross && !cross_zero(s, t))) {
        gp = A[(6 + dir * 9 + k) * n + C];
        gm = A[(6 + dir * 9 + k) * n + nb[2 * dir + 1]];
      }
      R.Gp[dir][k] = ex[2 * dir] ? gp : (KT)0;
      R.Gm[dir][k] = ex[2 * dir + 1] ? gm : (KT)0;
    }
#pragma unroll
  for (int t = 0; t < 3; ++t) R.xo[t] = own_zero(mode) ? (KT)0 : x[t * n + C];
#pragma unroll
  for (int j = 0; j < 6; ++j)
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      // absent neighbours read cell C itself (possibly unwritten): select zero
      const KT v = nbr_zero(mode) ? (KT)0 : x[t * n + nb[j]];
      R.xn[j][t] = ex[j] ? v : (KT)0;
    }
  if (own_corr(mode) || nbr_corr(mode)) {
    const size_t np = Lp.ncell;
    const KT* xp = Lp.x;
    const int px = q.x >> 1, py = q.y >> 1, pz = q.z >> 1;
    const int pc = lvl_index(px, py, pz, Lp.nx, Lp.ny);
    if (own_corr(mode))
#pragma unroll
      for (int t = 0; t < 3; ++t) R.xo[t] += alpha * xp[t * np + pc];
    if (nbr_corr(mode)) {
      const int pq[6] = {((q.x + 1) >> 1) - px, ((q.x - 1) >> 1) - px, ((q.y + 1) >> 1) - py,
                         ((q.y - 1) >> 1) - py, ((q.z + 1) >> 1) - pz, ((q.z - 1) >> 1) - pz};
      const int pst[6] = {0, 0, Lp.nx, Lp.nx, Lp.nx * Lp.ny, Lp.nx * Lp.ny};   // x steps: lvl_xstep
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        const int pcj = !ex[j] ? pc : j < 2 ? lvl_xstep(pc, px, pq[j], Lp.nx) : pc + pq[j] * pst[j];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const KT v = xp[t * np + pcj];
          R.xn[j][t] += ex[j] ? alpha * v : (KT)0;
        }
      }
    }
  }
}

}  // namespace

// ---------------------------------------------------------------- assembly
// The potential operator's interface conductances in the order the level-0
// smoother reads them (cond_rb): voxel i's interface faces in direction
// order at the start of its list, from whichever side i is on, negated for
// cathode (or foil) faces.  One thread per voxel; run after every
// linearisation, which rewrites cond_an and cond_ca.
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_cond_rb(CellDev* cells, const int2* __restrict__ blk) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active) return;
  const int i = bb.y * kBlock + threadIdx.x;
  if (i >= cd.N) return;
  const uint32_t mi = cd.meta[i];
  const uint32_t msk = mask_of(mi);
  if (!msk) return;
  const C3 c = c3_of(i, cd.nx, cd.ny, cd.inv_nx, cd.inv_ny);
  const int color = (c.x + c.y + c.z) & 1;
  KT* out = (KT*)cd.cond_rb + (size_t)color * (cd.F_an + cd.F_ca) + base_of(cd.meta_rb[rb_index(cd, c.x, c.y, c.z)]);
  const int L = lab_of(mi);
  int r = 0;
  for (int d = 0; d < 6; ++d) {
    if (!((msk >> d) & 1u)) continue;
    int Ls = L;
    uint32_t f;
    if (L == PORE) {   // the face record sits with the solid neighbour (the mask marks existing neighbours only)
      const int k = fine_nbr(i, c, cd.nx, cd.ny, cd.nz, d);
      const uint32_t mk = cd.meta[k >= 0 ? k : i];
      Ls = lab_of(mk);
      f = face_rank(mk, d ^ 1);
    } else {
      f = face_rank(mi, d);
    }
    const KT g = Ls == CATHODE ? ((const KT*)cd.cond_ca)[f] : ((const KT*)cd.cond_an)[f];
    out[r++] = Ls == CATHODE ? -g : g;
  }
}

// Level-1 operator from the voxel level: extras summed per slot; faces inside
// the cell between different slots -> X; faces to the +dir neighbour cell -> G.
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_mg_assemble0(CellDev* cells, const int2* __restrict__ blk, int op) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active || cd.nlev < 2) return;
  const MGLevel& L1 = cd.lv[1];
  const int C = bb.y * kBlock + threadIdx.x;
  if (C >= L1.ncell) return;
  const C3 q = lvl_coords(C, L1);
  KT E[3] = {0, 0, 0}, X[3] = {0, 0, 0}, G[27];
  for (int k = 0; k < 27; ++k) G[k] = (KT)0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int fx = 2 * q.x + dx, fy = 2 * q.y + dy, fz = 2 * q.z + dz;
        if (fx >= cd.nx || fy >= cd.ny || fz >= cd.nz) continue;
        const int i = fx + cd.nx * (fy + cd.ny * fz);
        const uint32_t mi = cd.meta[i];
        const int Li = lab_of(mi);
        const C3 fc{fx, fy, fz};
        E[Li] += fine_extra<KT>(cd, op, Li, fz);
        if (op == 0) {   // interface part of the concentration diagonal, all six faces
          KT di = (KT)0;
          for (int d = 0; d < 6; ++d) {
            const int k = fine_nbr(i, fc, cd.nx, cd.ny, cd.nz, d);
            if (k >= 0) {
              const uint32_t mk = cd.meta[k];
              di += c_iface_term<KT>(cd, Li, lab_of(mk), mi, mk, d);
            }
          }
          E[Li] += di;
          ((KT*)cd.dint)[rb_index(cd, fx, fy, fz)] = di;   // for the level-0 smoother and restriction
        }
        for (int d = 1; d < 6; d += 2) {   // + directions only: each face counted once
          const int k = fine_nbr(i, fc, cd.nx, cd.ny, cd.nz, d);
          if (k < 0) continue;
          const uint32_t mk = cd.meta[k];
          const int Lk = lab_of(mk);
          const KT g = fine_cond<KT>(cd, op, Li, Lk, mi, mk, d);
          if (g == (KT)0) continue;
          const int dir = d >> 1;
          const bool inside = (dir == 0 ? dx : dir == 1 ? dy : dz) == 0;
          if (inside) {
            if (Li != Lk) X[xidx(Li, Lk)] += g;
          } else {
            G[dir * 9 + Li * 3 + Lk] += g;
          }
        }
      }
  KT* o = (KT*)L1.op[op];
  const size_t n = L1.ncell;
  for (int s = 0; s < 3; ++s) o[s * n + C] = E[s];
  for (int k = 0; k < 3; ++k) o[(3 + k) * n + C] = X[k];
  for (int k = 0; k < 27; ++k) o[(6 + k) * n + C] = G[k];
}

// Level l+1 operator from level l (Galerkin sum with piecewise-constant
// transfer; same-slot couplings inside an aggregate cancel).
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_mg_assemble(CellDev* cells, const int2* __restrict__ blk, int l, int op) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active || l + 1 >= cd.nlev) return;
  const MGLevel& Lc = cd.lv[l];
  const MGLevel& Lp = cd.lv[l + 1];
  const int P = bb.y * kBlock + threadIdx.x;
  if (P >= Lp.ncell) return;
  const C3 q = lvl_coords(P, Lp);
  const OpV<KT> A{(const KT*)Lc.op[op], Lc.ncell};
  KT E[3] = {0, 0, 0}, X[3] = {0, 0, 0}, G[27];
  for (int k = 0; k < 27; ++k) G[k] = (KT)0;
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int cx = 2 * q.x + dx, cy = 2 * q.y + dy, cz = 2 * q.z + dz;
        if (cx >= Lc.nx || cy >= Lc.ny || cz >= Lc.nz) continue;
        const int c = lvl_cell(Lc, cx, cy, cz);
        for (int s = 0; s < 3; ++s) E[s] += A.E(c, s);
        for (int k = 0; k < 3; ++k) X[k] += A.X(c, k);
        for (int dir = 0; dir < 3; ++dir) {
          const int nxp = cx + (dir == 0), nyp = cy + (dir == 1), nzp = cz + (dir == 2);
          if (nxp >= Lc.nx || nyp >= Lc.ny || nzp >= Lc.nz) continue;
          const bool inside = (dir == 0 ? dx : dir == 1 ? dy : dz) == 0;
          for (int s = 0; s < 3; ++s)
            for (int t = 0; t < 3; ++t) {
              const KT g = A.G(c, dir, s, t);
              if (g == (KT)0) continue;
              if (inside) {
                if (s != t) X[xidx(s, t)] += g;
              } else {
                G[dir * 9 + s * 3 + t] += g;
              }
            }
        }
      }
  KT* o = (KT*)Lp.op[op];
  const size_t n = Lp.ncell;
  for (int s = 0; s < 3; ++s) o[s * n + P] = E[s];
  for (int k = 0; k < 3; ++k) o[(3 + k) * n + P] = X[k];
  for (int k = 0; k < 27; ++k) o[(6 + k) * n + P] = G[k];
}

// Dense inverse of the coarsest operator (one block per cell, FP64,
// Gauss-Jordan without pivoting: the operator is symmetric positive
// definite; empty slots get an identity row).  Matrices of up to
// kCoarseLdsDim rows are assembled and inverted in LDS and then written out.
constexpr int kCoarseLdsDim = 88;   // 88^2 doubles = 61,952 B of LDS

template <typename KT>
__device__ inline void coarse_assemble(const MGLevel& L, const OpV<KT>& A, double* M, int n) {
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) M[e] = 0.0;
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += blockDim.x) {
    const int c = r / 3, s = r % 3;
    const C3 q = lvl_coords(c, L);
    double D = (double)A.E(c, s);
    for (int t = 0; t < 3; ++t)
      if (t != s) {
        const double g = (double)A.X(c, xidx(s, t));
        D += g;
        M[(size_t)r * n + 3 * c + t] -= g;
      }
    for (int dir = 0; dir < 3; ++dir) {
      const int xp = q.x + (dir == 0), yp = q.y + (dir == 1), zp = q.z + (dir == 2);
      if (xp < L.nx && yp < L.ny && zp < L.nz) {
        const int c2 = lvl_cell(L, xp, yp, zp);
        for (int t = 0; t < 3; ++t) {
          const double g = (double)A.G(c, dir, s, t);
          D += g;
          M[(size_t)r * n + 3 * c2 + t] -= g;
        }
      }
      const int xm = q.x - (dir == 0), ym = q.y - (dir == 1), zm = q.z - (dir == 2);
      if (xm >= 0 && ym >= 0 && zm >= 0) {
        const int c2 = lvl_cell(L, xm, ym, zm);
        for (int t = 0; t < 3; ++t) {
          const double g = (double)A.G(c2, dir, t, s);
          D += g;
          M[(size_t)r * n + 3 * c2 + t] -= g;
        }
      }
    }
    M[(size_t)r * n + r] = D > 0.0 ? D : 1.0;
  }
  __syncthreads();
}

// In-place Gauss-Jordan inversion of the n x n matrix M (all threads).
__device__ inline void gauss_jordan(double* M, int n, double* piv) {
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) *piv = M[(size_t)k * n + k];
    __syncthreads();
    const double inv = 1.0 / *piv;
    for (int j = threadIdx.x; j < n; j += blockDim.x) M[(size_t)k * n + j] = (j == k ? inv : M[(size_t)k * n + j] * inv);
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int i = e / n, j = e % n;
      if (i == k || j == k) continue;   // row k and column k are read only in this pass
      M[(size_t)i * n + j] -= M[(size_t)i * n + k] * M[(size_t)k * n + j];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      if (i != k) M[(size_t)i * n + k] = -M[(size_t)i * n + k] * M[(size_t)k * n + k];
    __syncthreads();
  }
}

template <typename KT>
__global__ void __launch_bounds__(kBlock) k_mg_coarse_build(CellDev* cells, int ncells, int op) {
  __shared__ double Ms[kCoarseLdsDim * kCoarseLdsDim];
  __shared__ double piv;
  const int ci = blockIdx.x;
  if (ci >= ncells) return;
  const CellDev& cd = cells[ci];
  if (!cd.active) return;
  const int lc = cd.nlev - 1;
  const MGLevel& L = cd.lv[lc];
  const OpV<KT> A{(const KT*)L.op[op], L.ncell};
  const int n = 3 * L.ncell;
  double* M = cd.cinv[op];
  if (n <= kCoarseLdsDim) {
    coarse_assemble<KT>(L, A, Ms, n);
    gauss_jordan(Ms, n, &piv);
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) M[e] = Ms[e];
  } else {
    coarse_assemble<KT>(L, A, M, n);
    gauss_jordan(M, n, &piv);
  }
}

// ---------------------------------------------------------------- V-cycle
// Level-0 red-black Gauss-Seidel half sweep on operator op over the voxels of
// one colour (threads map to that colour only); the solution lives in the
// Krylov vector z (concentration part for op 0, potential part for op 1), the
// right-hand side in b0.  mode SM_ZERO: first sweep (x treated as zero);
// SM_CORR: neighbours corrected by alpha * (level-1 solution); else plain.
// The iterate, right-hand side and meta words are read in colour-split order
// (thread t of colour `color` is colour-split slot color*rbH + t), so a half
// sweep touches whole cache lines of each colour.  On a cell's last
// post-smoothing sweep (post, it == nu-1) the new values also go to the
// Krylov vector z in natural order: the black values of that sweep are final,
// and the red ones of the following half sweep.
// BS threads per workgroup (kBlock in table launches; a single-cell launch
// takes the size the tuner picked for the cell).
template <typename KT, int BS, int OP>
__global__ void __launch_bounds__(BS) k_mg0_smooth(CellDev* cells, const int2* __restrict__ blk, int color, int mode,
                                                   int it, int need, int post) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active || it >= cd.nu) return;   // cells that asked for fewer sweeps skip this one
  C3 c;
  const int t = bb.y * BS + threadIdx.x;
  if (!color_cell(t, color, cd.lv[0], c)) return;
  const int p = color * cd.rbH + t;
  KT* x0 = (KT*)cd.x_rb;
  const uint32_t nrb = 2u * (uint32_t)cd.rbH;
  const uint32_t mi = buf_ld<uint32_t>(buf_of(cd.meta_rb, nrb * 4u), (uint32_t)p * 4u);
  const KT bi = buf_ld<KT>(buf_of(cd.b0, nrb * (uint32_t)sizeof(KT)), (uint32_t)p * (uint32_t)sizeof(KT));
  KT D, S;
  voxel_row<KT, OP>(cd, color, p, c, mi, x0, mode == SM_ZERO, mode == SM_CORR, D, S);
  if (!gate_state(cd, need)) return;
  const KT xn = D > (KT)0 ? (bi + S) / D : (KT)0;
  buf_st(buf_of(x0, nrb * (uint32_t)sizeof(KT)), (uint32_t)p * (uint32_t)sizeof(KT), xn);
  if (post && it == cd.nu - 1)
    ((KT*)cd.z)[(size_t)OP * cd.N + c.x + __umul24((unsigned)cd.nx, (unsigned)(c.y + (int)__umul24((unsigned)cd.ny, (unsigned)c.z)))] = xn;
}

// Sum over the 4 lanes of an aligned lane group (xor butterfly: every lane
// ends with the identical value).
template <typename T>
__device__ inline T lane4_sum(T v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  return v;
}

// Child c (0..3) of a parent cell among its red children (offsets with an
// even sum: parent cells sit at even coordinates, so these are the children
// of colour 0), in the order of the child index dx + 2 dy + 4 dz.
__device__ inline C3 red_child(const C3& q, int c) {
  const int dx = c == 1 || c == 2, dy = c == 1 || c == 3, dz = c >= 2;
  return C3{2 * q.x + dx, 2 * q.y + dy, 2 * q.z + dz};
}

// Level-0 residual restricted to level 1.  The last pre-smoothing half sweep
// solved every black row exactly for the current red values, so only red
// rows carry a residual (the black ones are zero up to rounding and are not
// evaluated): 4 lanes per level-1 cell, one per red child voxel; the
// per-slot sums are formed across the lanes.
template <typename KT, int OP>
__global__ void __launch_bounds__(kBlock) k_mg0_restrict(CellDev* cells, const int2* __restrict__ blk, int need) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active) return;
  const MGLevel& L1 = cd.lv[1];
  const int t = bb.y * kBlock + threadIdx.x;
  const int C = t >> 2, ch = t & 3;
  const bool live = C < L1.ncell;   // whole 4-lane groups share C: shuffles stay within live groups
  KT rs[3] = {0, 0, 0};
  if (live) {
    const C3 fc = red_child(lvl_coords(C, L1), ch);
    if (fc.x < cd.nx && fc.y < cd.ny && fc.z < cd.nz) {
      const KT* x0 = (const KT*)cd.x_rb;
      const int p = rb_index(cd, fc.x, fc.y, fc.z);
      const uint32_t mi = cd.meta_rb[p];
      const KT xi = x0[p], bi = ((const KT*)cd.b0)[p];
      KT D, S;
      voxel_row<KT, OP>(cd, 0, p, fc, mi, x0, false, false, D, S);
      const int L = lab_of(mi);
      const KT r = bi + S - D * xi;
      rs[0] = L == 0 ? r : (KT)0;
      rs[1] = L == 1 ? r : (KT)0;
      rs[2] = L == 2 ? r : (KT)0;
    }
  }
  for (int s = 0; s < 3; ++s) rs[s] = lane4_sum(rs[s]);
  if (!gate_state(cd, need)) return;   // uniform over the block (one cell)
  if (live && ch == 0) {
    KT* b1 = (KT*)L1.b;
    for (int s = 0; s < 3; ++s) b1[(size_t)s * L1.ncell + C] = rs[s];
  }
}

// Coarse-level (l >= 1) red-black block Gauss-Seidel update of cell C: the
// cell's slots are solved together, D_s x_s - sum_t X_st x_t = N_s with
// N_s = b_s + the neighbours' couplings.  Slots 1 and 2 (anode, cathode) are
// never coupled, so eliminating x_1 and x_2 leaves
//   x_0 = (N_0 + X_01 N_1 / D_1 + X_02 N_2 / D_2) / (D_0 - X_01^2 / D_1 - X_02^2 / D_2)
// and then x_1, x_2 from their rows (an absent slot has D = 0 and x = 0).
// Every cell of the colour then meets its equations exactly: after a half
// sweep its residual is zero up to rounding.
template <typename KT, int OP>
__device__ inline void smooth_cell(const CellDev& cd, const LV<KT>& L, const LV<KT>& Lp, KT alpha, int C, const C3& q,
                                   int mode, int need) {
  CoarseRow<KT> R;
  gather_coarse<KT, OP>(L, Lp, alpha, C, q, mode, R);
  KT D[3], Nb[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    KT d = R.E[s], nb = R.b[s];
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if (t != s) d += R.X[xidx(s, t)];
#pragma unroll
    for (int dir = 0; dir < 3; ++dir)
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const KT gp = R.Gp[dir][s * 3 + t], gm = R.Gm[dir][t * 3 + s];
        d += gp + gm;
        nb += gp * R.xn[2 * dir][t] + gm * R.xn[2 * dir + 1][t];
      }
    D[s] = d;
    Nb[s] = nb;
  }
  const KT x01 = R.X[xidx(0, 1)], x02 = R.X[xidx(0, 2)];
  const bool h1 = D[1] > (KT)0, h2 = D[2] > (KT)0;
  const KT i1 = h1 ? (KT)1 / D[1] : (KT)0, i2 = h2 ? (KT)1 / D[2] : (KT)0;
  const KT d0 = D[0] - x01 * x01 * i1 - x02 * x02 * i2;
  const KT r0 = Nb[0] + x01 * Nb[1] * i1 + x02 * Nb[2] * i2;
  R.xo[0] = (D[0] > (KT)0 && d0 > (KT)0) ? r0 / d0 : (KT)0;
  R.xo[1] = h1 ? (Nb[1] + x01 * R.xo[0]) * i1 : (KT)0;
  R.xo[2] = h2 ? (Nb[2] + x02 * R.xo[0]) * i2 : (KT)0;
  if (!gate_state(cd, need)) return;
  KT* x = L.x;
#pragma unroll
  for (int s = 0; s < 3; ++s) x[(size_t)s * L.ncell + C] = R.xo[s];
}

// Residual (per slot) of coarse cell c at level l.
template <typename KT, int OP>
__device__ inline void residual_cell(const LV<KT>& L, int c, const C3& q, KT (&r)[3]) {
  CoarseRow<KT> R;
  gather_coarse<KT, OP>(L, L, (KT)0, c, q, SM_PLAIN, R);
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const KT xs = R.xo[s];
    KT rr = R.b[s] - R.E[s] * xs;
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if (t != s) rr -= R.X[xidx(s, t)] * (xs - R.xo[t]);
#pragma unroll
    for (int dir = 0; dir < 3; ++dir)
#pragma unroll
      for (int t = 0; t < 3; ++t)
        rr -= R.Gp[dir][s * 3 + t] * (xs - R.xn[2 * dir][t]) + R.Gm[dir][t * 3 + s] * (xs - R.xn[2 * dir + 1][t]);
    r[s] = rr;
  }
}

template <typename KT, int OP>
__global__ void __launch_bounds__(kBlock) k_mgl_smooth(CellDev* cells, const int2* __restrict__ blk, int l, int color,
                                                       int mode, int it, int need) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active || l >= cd.lglob || it >= (l >= 2 ? min(cd.nu, cd.nu_c) : cd.nu)) return;
  const MGLevel& L = cd.lv[l];
  C3 q;
  if (!color_cell(bb.y * kBlock + threadIdx.x, color, L, q)) return;
  smooth_cell<KT, OP>(cd, view<KT>(L, OP), view<KT>(cd.lv[l + 1], OP), (KT)cd.alpha, lvl_cell(L, q.x, q.y, q.z), q,
                  mode, need);
}

// Level-l residual restricted to level l+1: 4 lanes per parent, one per red
// child (the black children's residuals are zero after the last half sweep).
template <typename KT, int OP>
__global__ void __launch_bounds__(kBlock) k_mgl_restrict(CellDev* cells, const int2* __restrict__ blk, int l, int need) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active || l >= cd.lglob) return;
  const MGLevel& L = cd.lv[l];
  const MGLevel& Lp = cd.lv[l + 1];
  const int t = bb.y * kBlock + threadIdx.x;
  const int P = t >> 2, ch = t & 3;
  const bool live = P < Lp.ncell;   // whole 4-lane groups share P
  KT rs[3] = {0, 0, 0};
  if (live) {
    const C3 c = red_child(lvl_coords(P, Lp), ch);
    if (c.x < L.nx && c.y < L.ny && c.z < L.nz) residual_cell<KT, OP>(view<KT>(L, OP), lvl_cell(L, c.x, c.y, c.z), c, rs);
  }
  for (int s = 0; s < 3; ++s) rs[s] = lane4_sum(rs[s]);
  if (!gate_state(cd, need)) return;   // uniform over the block (one cell)
  if (live && ch == 0) {
    KT* bp = (KT*)Lp.b;
    for (int s = 0; s < 3; ++s) bp[(size_t)s * Lp.ncell + P] = rs[s];
  }
}

// One red-black half sweep of level l inside the fused cycle (all threads
// of the workgroup; followed by a barrier).
template <typename KT, int OP>
__device__ inline void fused_half_sweep(const CellDev& cd, const LV<KT>& L, const LV<KT>& Lp, KT alpha, int l, int color,
                                        int mode) {
  const int nh = ((L.nx + 1) >> 1) * L.ny * L.nz;
  for (int t = threadIdx.x; t < nh; t += blockDim.x) {
    C3 q;
    if (color_cell(t, color, L.nx, L.ny, L.nz, cd.lv[l].inv_hx, cd.lv[l].inv_ny, q))
      smooth_cell<KT, OP>(cd, L, Lp, alpha, lvl_index(q.x, q.y, q.z, L.nx, L.ny), q, mode, -2);
  }
  __syncthreads();
}

// Levels lglob..coarsest of one cell in one workgroup (levels small enough
// that barriers are cheaper than kernel launches): pre-smoothing and
// restriction down to the coarsest level, dense coarsest solve, coarse
// correction and post-smoothing back up to lglob.  Levels lfuse.. are
// staged in LDS first (operators and vectors; the dynamic shared-memory size
// is fused_lds_bytes); levels lglob..lfuse-1 (too large for LDS, small enough
// for one workgroup) stay in device memory and run with the launched levels'
// sweep counts and restriction sums, so they compute what the launched
// kernels would.  The coarsest inverse stays in device memory (symmetric:
// read column-wise, coalesced).  Level lglob's solution ends in device
// memory: the launched level above reads it for its coarse correction.
template <typename KT, int OP>
__global__ void __launch_bounds__(kFuseBlock) k_mg_coarse_cycle(CellDev* cells, int ncells, int need) {
  constexpr int op = OP;
  extern __shared__ __align__(16) unsigned char smem[];
  const int ci = blockIdx.x;
  if (ci >= ncells) return;
  const CellDev& cd = cells[ci];
  if (!gate(cd, need)) return;
  const int lg = cd.lglob, lf = cd.lfuse, lc = cd.nlev - 1;
  const int nu = cd.nu_f;
  const KT alpha = (KT)cd.alpha;
  // device-memory levels: sweeps and restriction as in the launched kernels
  for (int l = lg; l < lf; ++l) {
    const LV<KT> L = view<KT>(cd.lv[l], op), Lp = view<KT>(cd.lv[l + 1], op);
    const int nul = l >= 2 ? min(cd.nu, cd.nu_c) : cd.nu;
    for (int it = 0; it < nul; ++it) {
      fused_half_sweep<KT, OP>(cd, L, Lp, alpha, l, 0, it == 0 ? SM_ZERO : SM_PLAIN);
      fused_half_sweep<KT, OP>(cd, L, Lp, alpha, l, 1, it == 0 ? SM_OWNZERO : SM_PLAIN);
    }
    // red children only, summed as the 4-lane restriction kernel sums them
    for (int P = threadIdx.x; P < Lp.ncell; P += blockDim.x) {
      const C3 q = lvl_coords(P, cd.lv[l + 1]);
      KT r[4][3];
      for (int ch = 0; ch < 4; ++ch) {
        const C3 c = red_child(q, ch);
        if (c.x < L.nx && c.y < L.ny && c.z < L.nz)
          residual_cell<KT, OP>(L, lvl_index(c.x, c.y, c.z, L.nx, L.ny), c, r[ch]);
        else
          r[ch][0] = r[ch][1] = r[ch][2] = (KT)0;
      }
      for (int s = 0; s < 3; ++s) Lp.b[(size_t)s * Lp.ncell + P] = (r[0][s] + r[1][s]) + (r[2][s] + r[3][s]);
    }
    __syncthreads();
  }
  KT* const base = (KT*)smem;
  // LDS element offsets of level l's x, b and operator: levels lf..lc in order
  auto offset = [&](int l) {
    size_t o = 0;
    for (int k = lf; k < l; ++k) o += (size_t)cd.lv[k].ncell * (6 + (k < lc ? kOpStride : 0));
    return o;
  };
  // level l with its arrays in LDS (built where used, so that the compiler
  // sees LDS pointers and emits LDS instructions)
  auto lds_level = [&](int l) {
    const MGLevel& G = cd.lv[l];
    const size_t o = offset(l), n = G.ncell;
    return LV<KT>{G.nx, G.ny, G.nz, G.ncell, base + o, base + o + 3 * n, base + o + 6 * n, op};
  };
  // stage: operator op of every fused level but the coarsest, right-hand side of level lf
  for (int l = lf; l < lc; ++l) {
    const size_t n = (size_t)kOpStride * cd.lv[l].ncell;
    const KT* src = (const KT*)cd.lv[l].op[op];
    KT* dst = base + offset(l) + 6 * (size_t)cd.lv[l].ncell;
    for (size_t e = threadIdx.x; e < n; e += blockDim.x) dst[e] = src[e];
  }
  {
    const size_t n = 3 * (size_t)cd.lv[lf].ncell;
    const KT* src = (const KT*)cd.lv[lf].b;
    KT* dst = base + offset(lf) + n;
    for (size_t e = threadIdx.x; e < n; e += blockDim.x) dst[e] = src[e];
  }
  __syncthreads();
  for (int l = lf; l < lc; ++l) {
    const LV<KT> L = lds_level(l);
    const LV<KT> Lp = lds_level(l + 1);
    const int nh = ((L.nx + 1) >> 1) * L.ny * L.nz;
    for (int it = 0; it < nu; ++it)
      for (int color = 0; color < 2; ++color) {
        const int mode = it == 0 ? (color == 0 ? SM_ZERO : SM_OWNZERO) : SM_PLAIN;
        for (int t = threadIdx.x; t < nh; t += blockDim.x) {
          C3 q;
          if (color_cell(t, color, L.nx, L.ny, L.nz, cd.lv[l].inv_hx, cd.lv[l].inv_ny, q))
            smooth_cell<KT, OP>(cd, L, Lp, alpha, lvl_index(q.x, q.y, q.z, L.nx, L.ny), q, mode, -2);
        }
        __syncthreads();
      }
    for (int P = threadIdx.x; P < Lp.ncell; P += blockDim.x) {
      const C3 q = lvl_coords(P, cd.lv[l + 1]);
      KT acc[3] = {0, 0, 0};
      for (int ch = 0; ch < 8; ++ch) {
        const int cx = 2 * q.x + (ch & 1), cy = 2 * q.y + ((ch >> 1) & 1), cz = 2 * q.z + (ch >> 2);
        if (cx >= L.nx || cy >= L.ny || cz >= L.nz || ((cx + cy + cz) & 1)) continue;   // black: solved exactly
        KT r[3];
        residual_cell<KT, OP>(L, lvl_index(cx, cy, cz, L.nx, L.ny), C3{cx, cy, cz}, r);
        for (int s = 0; s < 3; ++s) acc[s] += r[s];
      }
      for (int s = 0; s < 3; ++s) Lp.b[(size_t)s * Lp.ncell + P] = acc[s];
    }
    __syncthreads();
  }
  {  // coarsest: x = M^-1 b (M symmetric: row r read as column r, coalesced)
    const LV<KT> L = lds_level(lc);
    const int n = 3 * L.ncell;
    const KT* b = L.b;
    const double* M = cd.cinv[op];
    KT* x = L.x;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
      double acc = 0.0;
      for (int j = 0; j < n; ++j) acc += M[(size_t)j * n + r] * (double)b[(size_t)(j % 3) * L.ncell + j / 3];
      x[(size_t)(r % 3) * L.ncell + r / 3] = (KT)acc;
    }
    __syncthreads();
  }
  for (int l = lc - 1; l >= lf; --l) {
    const LV<KT> L = lds_level(l);
    const LV<KT> Lp = lds_level(l + 1);
    const int nh = ((L.nx + 1) >> 1) * L.ny * L.nz;
    for (int it = 0; it < nu; ++it)
      for (int color = 1; color >= 0; --color) {
        const int mode = it == 0 ? (color == 1 ? SM_CORR : SM_OWNCORR) : SM_PLAIN;
        for (int t = threadIdx.x; t < nh; t += blockDim.x) {
          C3 q;
          if (color_cell(t, color, L.nx, L.ny, L.nz, cd.lv[l].inv_hx, cd.lv[l].inv_ny, q))
            smooth_cell<KT, OP>(cd, L, Lp, alpha, lvl_index(q.x, q.y, q.z, L.nx, L.ny), q, mode, -2);
        }
        __syncthreads();
      }
  }
  {
    const size_t n = 3 * (size_t)cd.lv[lf].ncell;
    const KT* src = base + offset(lf);
    KT* dst = (KT*)cd.lv[lf].x;
    for (size_t e = threadIdx.x; e < n; e += blockDim.x) dst[e] = src[e];
  }
  if (lg < lf) __syncthreads();
  for (int l = lf - 1; l >= lg; --l) {
    const LV<KT> L = view<KT>(cd.lv[l], op), Lp = view<KT>(cd.lv[l + 1], op);
    const int nul = l >= 2 ? min(cd.nu, cd.nu_c) : cd.nu;
    for (int it = 0; it < nul; ++it) {
      fused_half_sweep<KT, OP>(cd, L, Lp, alpha, l, 1, it == 0 ? SM_CORR : SM_PLAIN);
      fused_half_sweep<KT, OP>(cd, L, Lp, alpha, l, 0, it == 0 ? SM_OWNCORR : SM_PLAIN);
    }
  }
}

// ----------------------------------------------------- block-triangular glue
// b0 = v_c - tau * v_phi on pore voxels (row operation removing migration);
// b0 is stored in colour-split order.
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_pc_pre(CellDev* cells, const int2* __restrict__ blk, int src, int need) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active) return;
  const int i = bb.y * kBlock + threadIdx.x;
  if (i >= cd.N) return;
  const KT* v = vsel<KT>(cd, src);
  const uint32_t mi = cd.meta[i];
  const KT vc = v[i], vp = v[(size_t)cd.N + i];
  const KT r = lab_of(mi) == PORE ? vc - (KT)cd.tau * vp : vc;
  if (!gate_state(cd, need)) return;
  const C3 c = c3_of(i, cd.nx, cd.ny, cd.inv_nx, cd.inv_ny);
  ((KT*)cd.b0)[rb_index(cd, c.x, c.y, c.z)] = r;
}

// b0 = v_phi - (J [z_c; 0])_phi: the potential rows' dependence on the
// concentration correction (electrolyte dln c/dc term and Butler-Volmer /
// plating concentration derivatives) moved to the right-hand side.
template <typename KT>
__global__ void __launch_bounds__(kBlock) k_pc_mid(CellDev* cells, const int2* __restrict__ blk, int src, int need) {
  const int2 bb = block_of(blk);
  const CellDev& cd = cells[bb.x];
  if (!cd.active) return;
  const int i = bb.y * kBlock + threadIdx.x;
  if (i >= cd.N) return;
  // buffer loads (see jv_row): absent neighbours read at kNoIdx (zero), the
  // anode and cathode face records through one descriptor
  constexpr uint32_t kt = sizeof(KT);
  const uint32_t N = (uint32_t)cd.N;
  const BufRes rm = buf_of(cd.meta, N * 4u);
  const BufRes rz = buf_of(cd.z, N * kt);   // concentration part of z
  const BufRes rw = buf_of(cd.wpore, N * kt);
  const BufRes rv = buf_of(vsel<KT>(cd, src), 2u * N * kt);
  const uint32_t ca_off = (uint32_t)((const char*)cd.coef_ca - (const char*)cd.coef_an);
  const BufRes rco = buf_of(cd.coef_an, ca_off + 3u * (uint32_t)(cd.F_ca > 0 ? cd.F_ca : 1) * kt);
  const C3 c = c3_of(i, cd.nx, cd.ny, cd.inv_nx, cd.inv_ny);
  int k[6];
  bool ex[6];
  neighbours6(i, c, cd.nx, cd.ny, cd.nz, k, ex);
  uint32_t kk[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) kk[j] = ex[j] ? (uint32_t)k[j] : kNoIdx;
  const int dmap[6] = {1, 0, 3, 2, 5, 4};   // neighbour slot -> face direction
  const uint32_t ui = (uint32_t)i;
  const uint32_t mi = buf_ld<uint32_t>(rm, ui * 4u);
  const KT vc = buf_ld<KT>(rz, ui * kt), wiv = buf_ld<KT>(rw, ui * kt), vpi = buf_ld<KT>(rv, ui * kt, N * kt);
  uint32_t mk[6];
  KT vk[6], wk[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    mk[j] = buf_ld<uint32_t>(rm, kk[j] * 4u);
    vk[j] = buf_ld<KT>(rz, kk[j] * kt);
    wk[j] = buf_ld<KT>(rw, kk[j] * kt);
  }
  const int L = lab_of(mi);
  const KT wi = L == PORE ? wiv : (KT)0;
  const KT Gt = (KT)(cd.Gk * cd.tth);
  KT yp = (KT)0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const int Lk = lab_of(mk[j]);
    const int d = dmap[j];
    const bool pp = L == PORE && Lk == PORE;
    const bool iface = (L == PORE) != (Lk == PORE);
    const bool pore_side = L == PORE;
    const uint32_t f = iface ? face_rank(pore_side ? mk[j] : mi, pore_side ? (d ^ 1) : d) : 0u;
    const bool an = (pore_side ? Lk : L) == ANODE;
    const uint32_t co = an ? __umul24(f, 5u * kt) : ca_off + __umul24(f, 3u * kt);   // f < 2^24
    const KT c0 = buf_ld<KT>(rco, co), c1 = buf_ld<KT>(rco, co + kt), c3 = buf_ld<KT>(rco, co + (an ? 3 : 1) * kt);
    const KT vs = pore_side ? vk[j] : vc, vpo = pore_side ? vc : vk[j];
    // interface flux derivative w.r.t. the concentrations (potential part zero)
    const KT q = c0 * vs + c1 * vpo + (an ? c3 * vpo : (KT)0);
    const KT t = pp ? Gt * (wk[j] * vk[j] - wi * vc)      // outward dj from i
                    : (iface ? (pore_side ? -q : q) : (KT)0);
    yp += ex[j] ? t : (KT)0;
  }
  if (!gate_state(cd, need)) return;
  ((KT*)cd.b0)[rb_index(cd, c.x, c.y, c.z)] = vpi - yp;
}

// ---------------------------------------------------------------- launchers
// A level's block table is empty when no cell that is still iterating has
// that level (the batch mixes grid sizes): such launches are skipped, since a
// launch of zero workgroups is a configuration error.
template <typename KT>
void launch_mg_setup(const BatchLaunch& b, hipStream_t s) {
  k_cond_rb<KT><<<b.nblk, kBlock, 0, s>>>(b.cells, b.blk);
  for (int op = 0; op < 2; ++op) {
    if (b.lvl_nblk[1] > 0) k_mg_assemble0<KT><<<b.lvl_nblk[1], kBlock, 0, s>>>(b.cells, b.lvl_blk[1], op);
    for (int l = 1; l + 1 < b.maxlev; ++l)
      if (b.lvl_nblk[l + 1] > 0)
        k_mg_assemble<KT><<<b.lvl_nblk[l + 1], kBlock, 0, s>>>(b.cells, b.lvl_blk[l + 1], l, op);
    k_mg_coarse_build<KT><<<b.ncell, kBlock, 0, s>>>(b.cells, b.ncell, op);
  }
}

template <typename KT, int OP>
static void smooth0_op(const BatchLaunch& b, int color, int mode, int it, int need, int post, hipStream_t s) {
  const int bs = b.lvlh_blk[0] ? kBlock : b.bs_smooth0;
  const int nh = b.lvlh_nblk[0] * kBlock;   // single cell: one colour's cells, rounded up to kBlock
  if (bs == 64)
    k_mg0_smooth<KT, 64, OP><<<nh / 64, 64, 0, s>>>(b.cells, nullptr, color, mode, it, need, post);
  else if (bs == 128)
    k_mg0_smooth<KT, 128, OP><<<nh / 128, 128, 0, s>>>(b.cells, nullptr, color, mode, it, need, post);
  else if (bs == 512)   // the grid rounds up: threads past the colour's last cell return at once
    k_mg0_smooth<KT, 512, OP><<<(nh + 511) / 512, 512, 0, s>>>(b.cells, nullptr, color, mode, it, need, post);
  else if (bs == 1024)
    k_mg0_smooth<KT, 1024, OP><<<(nh + 1023) / 1024, 1024, 0, s>>>(b.cells, nullptr, color, mode, it, need, post);
  else
    k_mg0_smooth<KT, kBlock, OP><<<b.lvlh_nblk[0], kBlock, 0, s>>>(b.cells, b.lvlh_blk[0], color, mode, it, need,
                                                                   post);
}

template <typename KT>
static void smooth0(const BatchLaunch& b, int op, int color, int mode, int it, int need, int post, hipStream_t s) {
  if (b.lvlh_nblk[0] <= 0) return;
  if (op == 0)
    smooth0_op<KT, 0>(b, color, mode, it, need, post, s);
  else
    smooth0_op<KT, 1>(b, color, mode, it, need, post, s);
}

template <typename KT>
void launch_smooth0_probe(const BatchLaunch& b, hipStream_t s) {
  smooth0<KT>(b, 1, 0, SM_PLAIN, 0, -2, 0, s);
}

template <typename KT>
static void smoothl(const BatchLaunch& b, int l, int op, int color, int mode, int it, int need, hipStream_t s) {
  if (b.lvlh_nblk[l] <= 0) return;
  if (op == 0)
    k_mgl_smooth<KT, 0><<<b.lvlh_nblk[l], kBlock, 0, s>>>(b.cells, b.lvlh_blk[l], l, color, mode, it, need);
  else
    k_mgl_smooth<KT, 1><<<b.lvlh_nblk[l], kBlock, 0, s>>>(b.cells, b.lvlh_blk[l], l, color, mode, it, need);
}

// One V-cycle on operator op: red-black sweeps (red then black) down to the
// fused levels, the fused coarse cycle, then sweeps (black then red) back up.
// The first post-sweep applies the coarse correction lazily.  Each cell runs
// its own number of sweeps (CellDev::nu, nu_f); the launches cover the most
// any cell of the batch asks for and the others skip the surplus.
template <typename KT>
static void vcycle(const BatchLaunch& b, int op, int need, hipStream_t s) {
  const int top = b.maxglob;   // levels >= a cell's lglob run inside k_mg_coarse_cycle
  for (int l = 0; l < top; ++l) {
    const int nu = l >= 2 ? std::min(b.max_nu, b.max_nu_c) : b.max_nu;
    if (l == 0) prof_begin(PK_SMOOTH0, s);   // the 2 nu level-0 half sweeps run back to back
    for (int it = 0; it < nu; ++it) {
      if (l == 0) {
        smooth0<KT>(b, op, 0, it == 0 ? SM_ZERO : SM_PLAIN, it, need, 0, s);
        smooth0<KT>(b, op, 1, SM_PLAIN, it, need, 0, s);
      } else {
        smoothl<KT>(b, l, op, 0, it == 0 ? SM_ZERO : SM_PLAIN, it, need, s);
        smoothl<KT>(b, l, op, 1, it == 0 ? SM_OWNZERO : SM_PLAIN, it, need, s);
      }
    }
    if (l == 0 && prof_on(PK_SMOOTH0)) prof_end_n(PK_SMOOTH0, s, 2.0 * nu * b.bytes_smooth0, 2 * nu);
    if (b.lvlr_nblk[l + 1] <= 0) continue;
    if (l == 0)
      (op == 0 ? k_mg0_restrict<KT, 0> : k_mg0_restrict<KT, 1>)<<<b.lvlr_nblk[1], kBlock, 0, s>>>(
          b.cells, b.lvlr_blk[1], need);
    else
      (op == 0 ? k_mgl_restrict<KT, 0> : k_mgl_restrict<KT, 1>)<<<b.lvlr_nblk[l + 1], kBlock, 0, s>>>(
          b.cells, b.lvlr_blk[l + 1], l, need);
  }
  (op == 0 ? k_mg_coarse_cycle<KT, 0> : k_mg_coarse_cycle<KT, 1>)<<<b.ncell, kFuseBlock, b.fused_lds * sizeof(KT), s>>>(
      b.cells, b.ncell, need);
  for (int l = top - 1; l >= 0; --l) {
    const int nu = l >= 2 ? std::min(b.max_nu, b.max_nu_c) : b.max_nu;
    if (l == 0) prof_begin(PK_SMOOTH0, s);
    for (int it = 0; it < nu; ++it) {
      if (l == 0) {
        smooth0<KT>(b, op, 1, it == 0 ? SM_CORR : SM_PLAIN, it, need, 1, s);
        smooth0<KT>(b, op, 0, SM_PLAIN, it, need, 1, s);
      } else {
        smoothl<KT>(b, l, op, 1, it == 0 ? SM_CORR : SM_PLAIN, it, need, s);
        smoothl<KT>(b, l, op, 0, it == 0 ? SM_OWNCORR : SM_PLAIN, it, need, s);
      }
    }
    if (l == 0 && prof_on(PK_SMOOTH0)) prof_end_n(PK_SMOOTH0, s, 2.0 * nu * b.bytes_smooth0, 2 * nu);
  }
}

template <typename KT>
void launch_precond(const BatchLaunch& b, int src, int need, hipStream_t s) {
  prof_begin(PK_PRECOND, s);
  k_pc_pre<KT><<<b.nblk, kBlock, 0, s>>>(b.cells, b.blk, src, need);
  vcycle<KT>(b, 0, need, s);
  k_pc_mid<KT><<<b.nblk, kBlock, 0, s>>>(b.cells, b.blk, src, need);
  vcycle<KT>(b, 1, need, s);
  if (prof_on(PK_PRECOND)) prof_end(PK_PRECOND, s, 0.0);
}

template void launch_mg_setup<float>(const BatchLaunch&, hipStream_t);
template void launch_mg_setup<double>(const BatchLaunch&, hipStream_t);
template void launch_precond<float>(const BatchLaunch&, int, int, hipStream_t);
template void launch_smooth0_probe<float>(const BatchLaunch&, hipStream_t);
template void launch_smooth0_probe<double>(const BatchLaunch&, hipStream_t);
template void launch_precond<double>(const BatchLaunch&, int, int, hipStream_t);

}  // namespace mbx
