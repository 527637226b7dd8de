// mbx_dev.h — device-side data layout and pointwise laws of the cell model.
//
// Layout in HBM (per cell, structure of arrays, voxel flat index
// i + nx*(j + ny*k)):
//   meta[N]   uint32: bits 0-1 label (0 pore, 1 anode, 2 cathode), bits 2-7
//             interface mask (bit d set when the neighbour in direction d is
//             of the other kind: pore<->solid), bits 8-31 the voxel's first
//             interface-face index in its phase's face list (solid voxels).
//   c, phi    double[N] state; n double[F_an] plated amount per anode face.
//   face coefficient arrays (per phase, canonical face order), per-voxel
//   pore coefficient and 2x2 inverse diagonal blocks in the Krylov type KT.
//   Krylov vectors: 2N entries, [0,N) concentration rows/unknowns, [N,2N)
//   potential rows/unknowns, in scaled (dimensionless) units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbx {

constexpr double kFaraday = 96485.33212;   // C/mol
constexpr double kGasR = 8.314462618;      // J/(mol K)
constexpr int kBlock = 256;                // threads per voxel block (4 wavefronts)
constexpr int kMaxRestart = 40;            // GMRES restart length bound
constexpr int kPartStride = kMaxRestart + 2;
static_assert(kMaxRestart % 8 == 0, "basis loads are issued in chunks of 8");

enum { PORE = 0, ANODE = 1, CATHODE = 2 };

// Multigrid hierarchy (per cell).  Level 0 is the voxel grid (operators
// applied matrix-free); level l >= 1 is a grid of ceil-halved cells, each
// with three slots (pore, anode, cathode aggregates of the finer level).
constexpr int kMaxLevels = 12;
constexpr int kCoarseMaxCells = 64;
constexpr int kFuseMaxCells = 256;    // levels this small run inside one workgroup per cell, staged in LDS
constexpr int kGlobFuseMaxCells = 2048;   // ... and levels this small too, from device memory
constexpr int kFuseBlock = 1024;          // threads of that workgroup (a 1280-cell level: one cell per thread and colour)
constexpr size_t kFusedLdsBytes = 60 * 1024;   // LDS the fused levels may stage
constexpr double kToBoundary = 0.1;   // a Newton update leaves at least this fraction of the distance to a bound
constexpr int kOpStride = 33;   // per coarse cell: E[3], X[3], G[3 dirs][3][3] (SoA)
struct MGLevel {
  int nx, ny, nz, ncell;
  double inv_hx, inv_nx, inv_ny;   // smallest doubles >= 1/ceil(nx/2), 1/nx, 1/ny (divmod)
  void* x;       // KT [3*ncell] (slot-major)
  void* b;       // KT [3*ncell]
  void* op[2];   // KT [kOpStride*ncell] for the concentration (0) and potential (1) operators
};

// Block -> {cell, block within the cell}: from the batch's block table, or
// {0, blockIdx.x} for a single-cell launch (no table: one dependent load less
// at the start of every kernel).
__device__ inline int2 block_of(const int2* __restrict__ blk) {
  return blk ? blk[blockIdx.x] : make_int2(0, (int)blockIdx.x);
}

__host__ __device__ inline int lab_of(uint32_t m) { return int(m & 3u); }
__host__ __device__ inline uint32_t mask_of(uint32_t m) { return (m >> 2) & 63u; }
__host__ __device__ inline uint32_t base_of(uint32_t m) { return m >> 8; }
__device__ inline uint32_t face_rank(uint32_t m, int d) {
  return base_of(m) + (uint32_t)__popc(mask_of(m) & ((1u << d) - 1u));
}

// Slots of the per-cell reduction output array `red` (written by the
// finalising kernels of the two-pass reductions).
enum {
  RED_RSQ = 0,     // sum of squared scaled residual
  RED_RMAX = 1,    // max |scaled residual|
  RED_MSQ = 2,     // line-search merit: sum of squared diagonally weighted voxel-row residuals
  RED_DNMAX = 3,   // max |n_trial - n| / n_c of the eliminated plated amounts
  RED_BAD = 4,     // infeasible entries in a trial state
  RED_DUMAX = 5,   // max |scaled update|
  RED_BSQ = 6,     // sum of squares of a Krylov vector (rhs / true residual)
  RED_INV0 = 7,    // inventories: electrolyte, anode, cathode, plated (4 slots)
  RED_VSUM = 11,   // sum over cathode top voxels of phi (must follow the inventories)
  RED_TOL = 12,    // GMRES absolute tolerance of the current solve
  RED_BETA0 = 13,  // norm of the first GMRES residual of the current solve
  RED_LTE = 14,    // max over the differential unknowns of |u - u_pred| (scaled), adaptive stepping
  RED_HNORM = 15,  // ||w|| of the current GMRES iteration (H(k+1,k) before its Givens rotation)
  RED_NSLOT = 16
};
// Slots of the per-cell device-written integer array `ictl`.
enum { CTL_DONE = 0, CTL_K = 1, CTL_ITERS = 2, CTL_NSLOT = 4 };

// Per-cell descriptor.  The host keeps a mirror and uploads the array of
// descriptors of a batch whenever a field changes.
struct CellDev {
  int nx, ny, nz, N;
  int F_an, F_ca, n_top, nblk;
  int active;         // 0: every kernel skips this cell
  int elim_n;         // 1: residual kernels solve each face's plating balance for n
  int pad0;
  const uint32_t* meta;
  double *c, *phi, *n;               // Newton iterate
  double *c_try, *phi_try, *n_try;   // trial state (residual kernels read these)
  double *c_old, *phi_old, *n_old;   // u^n
  double *c_prev, *n_prev;           // u^(n-1) of an adaptive run (concentrations, plated amounts)
  double *Rc, *Rp, *Rn;              // residual rows at the trial state
  double *dc, *dp, *dn;              // Newton direction (raw units)
  double *rn_jnn, *sq;               // per anode face: R^n/J_nn, condensation term
  const int *faces_an, *faces_ca;    // compacted interface faces per phase: solid voxel * 8 + direction
  double *fres;                      // per interface face (anode faces, then cathode faces): intercalation
                                     // current [0, F), total current [F, 2F), A/m^2, solid -> pore > 0
  void *coef_an, *coef_ca;           // KT: 5 per anode face, 3 per cathode face
  void *wpore;                       // KT: c0/c on pore voxels
  void *Vb;                          // KT: (m+1) Krylov basis vectors of 2N
  void *Zb;                          // KT: m preconditioned basis vectors of 2N (flexible GMRES)
  void *w, *z, *b;                   // KT: 2N each (Krylov work vector, preconditioned vector, rhs)
  double *x;                         // 2N: GMRES iterate, FP64 in both modes
  void *dint;                        // KT [2 rbH]: interface part of the concentration preconditioner's diagonal (colour-split)
  double *part;                      // nblk * kPartStride partial sums
  double *red;                       // RED_NSLOT outputs (device-written)
  int *ictl;                         // CTL_NSLOT flags (device-written)
  double *gm;                        // GMRES small arrays (see gm_* offsets)
  // step data (host-written)
  double dt, lam, rtol;
  int m;                             // GMRES restart length
  int pad3;
  // parameters and derived constants
  double h, A, Vol, RT, VT, beta;
  double c0, x0, y0, De, kappa, tplus, thermo;
  double Ds[2], sigma[2], cmax[2], i00[2], U0[2], U1[2];
  double i00_pl, n_c, I_app, mu_ref;
  int plating;
  int half;                          // 1: half cell, the counter-electrode slot holds a Li foil (Sec. 2.2)
  double i00_ce;                     // Li-foil rate constant, A/m^2
  // multigrid
  int nlev, lfuse;                   // levels incl. the voxel level; coarsest = nlev-1;
                                     // levels >= lfuse run in one workgroup from LDS (k_mg_coarse_cycle)
  int lglob;                         // levels lglob..lfuse-1 run in that workgroup from device memory
  MGLevel lv[kMaxLevels];
  // Level-0 multigrid arrays in colour-split (red-black) order: voxel (x,y,z)
  // of colour c = (x+y+z)&1 sits at c*rbH + (y + ny*z)*rbhx + (x>>1), with
  // rbhx = ceil(nx/2) and rbH = rbhx*ny*nz (odd nx leaves padding slots), so a
  // half sweep reads and writes whole cache lines of one colour.
  int rbhx, rbH;
  double inv_nx, inv_ny;   // smallest doubles >= 1/nx and 1/ny (divmod)
  const uint32_t* meta_rb;           // meta words in colour-split order; the face-base field (bits 8-31)
                                     // holds the start of the voxel's list in its colour's part of cond_rb
  void *x_rb;                        // KT [2 rbH] level-0 iterate of the V-cycle being run
  void *b0;                          // KT [2 rbH] right-hand side of a level-0 solve (colour-split)
  void *cond_an, *cond_ca;           // KT potential-operator conductance per interface face
  void *cond_rb;                     // KT [2 (F_an + F_ca)]: the same conductances listed per voxel in
                                     // colour-split order (each face once from each side; colour c's
                                     // lists start at c (F_an + F_ca)); cathode faces stored negated
  double *cinv[2];                   // coarsest-level dense inverses (FP64), (3*ncell)^2 each
  double alpha;                      // coarse-correction scale
  int nu, nu_f;                      // smoothing sweeps (red+black pairs) per side: launched levels / fused levels
  int nu_c;                          // sweeps on launched levels >= 2 (at most nu)
  // scaled-operator constants
  double Kd;                         // kappa (1-t+) theta RT/(F h)
  double Gk, tth, Dh, tau, Ke, Gcol;
  double Dsh[2], Gs[2], Ks[2];
  // the level-0 smoother's same-phase coupling per operator (concentration,
  // potential) and label (pore, anode, cathode): Dh Dsh, Gk Gs, in both
  // Krylov types (read as scalars, then selected per voxel)
  alignas(16) double gsame_d[2][4];
  alignas(16) float gsame_f[2][4];
};

// gm layout: H[(m+1)*m] column-major, g[m+1], cs[m], sn[m], y[m], tmp[m+1]
__host__ __device__ inline int gm_H(int m) { return 0; }
__host__ __device__ inline int gm_g(int m) { return (m + 1) * m; }
__host__ __device__ inline int gm_cs(int m) { return (m + 1) * m + (m + 1); }
__host__ __device__ inline int gm_sn(int m) { return (m + 1) * m + (m + 1) + m; }
__host__ __device__ inline int gm_y(int m) { return (m + 1) * m + (m + 1) + 2 * m; }
__host__ __device__ inline int gm_tmp(int m) { return (m + 1) * m + (m + 1) + 3 * m; }
__host__ __device__ inline int gm_size(int m) { return (m + 1) * m + 2 * (m + 1) + 3 * m; }

// Neighbour of voxel (x,y,z) in direction d, or -1 outside the box.
struct VoxCoord {
  int x, y, z;
};
// Quotient and remainder of n / d for 0 <= n < 2^31, 1 <= d <= 2^21 and
// n / d < 2^24, from inv = the smallest double >= 1/d.  Then n*inv lies in
// [n/d, n/d + 2^-20/d], and the rounded product in [floor(n/d),
// floor(n/d) + 1 - 1/d + 2^-20/d + 2^-22]: below the next integer whenever
// d <= 2^21, so its truncation is floor(n/d) with no correction step.  The
// remainder's product fits the 24-bit multiplier (full rate, where the 32-bit
// one is quarter rate).
__device__ inline int divmod(int n, int d, double inv, int& r) {
  const int q = (int)((double)n * inv);
  r = n - (int)__umul24((unsigned)q, (unsigned)d);
  return q;
}
__device__ inline VoxCoord coord_of(const CellDev& cd, int i) {
  VoxCoord v;
  const int t = divmod(i, cd.nx, cd.inv_nx, v.x);
  v.z = divmod(t, cd.ny, cd.inv_ny, v.y);
  return v;
}

// The three same-phase couplings of operator op (pore, anode, cathode),
// fetched with one wide load (so that no load waits inside a label branch).
template <typename KT>
struct Gsame {
  KT pore, an, ca;
};
template <typename KT>
__device__ inline Gsame<KT> gsame_of(const CellDev& cd, int op);
template <>
__device__ inline Gsame<float> gsame_of<float>(const CellDev& cd, int op) {
  const float4 v = *(const float4*)cd.gsame_f[op];
  return {v.x, v.y, v.z};
}
template <>
__device__ inline Gsame<double> gsame_of<double>(const CellDev& cd, int op) {
  const double2 a = *(const double2*)cd.gsame_d[op], b = *(const double2*)(cd.gsame_d[op] + 2);
  return {a.x, a.y, b.x};
}

// Raw buffer loads: the array's base and size sit in a scalar descriptor and
// each lane supplies a 32-bit byte offset, so an indexed load needs no 64-bit
// address arithmetic.  The buffer unit checks every offset against the size:
// a load at or past the end returns zero without touching memory, so an
// absent neighbour is read at kNoOff instead of being selected away.  Arrays
// read this way hold fewer than kNoOff - 4096 bytes (checked at cell
// creation), so kNoOff plus any immediate offset stays out of range.
constexpr uint32_t kNoOff = 0x80000000u;
// Element index past every per-voxel array (cells hold fewer than 2^27
// voxels; times 4 or 8 bytes it stays below 2^32 and at or past the end).
constexpr uint32_t kNoIdx = 1u << 28;
using BufRes = __amdgpu_buffer_rsrc_t;
__device__ inline BufRes buf_of(const void* p, uint32_t bytes) {
  // descriptor word 3 = 0x00020000: 32-bit data format, which raw (untyped)
  // loads and the range check use on this architecture family
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
// off: per-lane byte offset; soff: a uniform byte offset (scalar register)
// added to it, e.g. the start of a row of a structure-of-arrays block.
template <typename T>
__device__ inline T buf_ld(BufRes r, uint32_t off, uint32_t soff = 0);
template <>
__device__ inline float buf_ld<float>(BufRes r, uint32_t off, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}
template <>
__device__ inline double buf_ld<double>(BufRes r, uint32_t off, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
}
template <>
__device__ inline uint32_t buf_ld<uint32_t>(BufRes r, uint32_t off, uint32_t soff) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0);
}
__device__ inline void buf_st(BufRes r, uint32_t off, float v, uint32_t soff = 0) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, soff, 0);
}
__device__ inline void buf_st(BufRes r, uint32_t off, double v, uint32_t soff = 0) {
  typedef uint32_t u32x2 __attribute__((__vector_size__(8)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, soff, 0);
}

// Colour-split index of voxel (x, y, z) (see CellDev::rbhx).
__host__ __device__ inline int rb_index(const CellDev& cd, int x, int y, int z) {
  return ((x + y + z) & 1) * cd.rbH + (y + cd.ny * z) * cd.rbhx + (x >> 1);
}

__device__ inline int neighbour(const CellDev& cd, int i, int x, int y, int z, int d) {
  switch (d) {
    case 0: return x > 0 ? i - 1 : -1;
    case 1: return x < cd.nx - 1 ? i + 1 : -1;
    case 2: return y > 0 ? i - cd.nx : -1;
    case 3: return y < cd.ny - 1 ? i + cd.nx : -1;
    case 4: return z > 0 ? i - cd.nx * cd.ny : -1;
    default: return z < cd.nz - 1 ? i + cd.nx * cd.ny : -1;
  }
}

// State-independent part of a scaled row's diagonal (mass + same-phase
// transport; the collector term is added by the caller): the merit norm
// divides each residual row by it, so that every weighted row measures the
// error of its own unknown.
__device__ inline void weight_add(const CellDev& cd, int L, int Lk, double& wc, double& wp) {
  if (L != Lk) return;
  wc += (L == PORE) ? cd.Dh : cd.Dsh[L - 1];
  wp += (L == PORE) ? cd.Gk : cd.Gs[L - 1];
}

// Plated amount that zeroes the face's plating balance (Sec. 2.3, eq. 2.8):
//   g(n) = (n - n_old)/dt + i_pl(n)/F = 0,
//   i_pl = K f_pre(n) - E,  K = i00_pl sqrt(c_e) e^a,  E = i00_pl sqrt(c_e) e^-a,
//   a = F (phi_s - phi_e)/(2RT).
// g is increasing in n >= 0, g(0) < 0 and g(n_old + dt E/F) >= 0, so the root
// is unique in that bracket; safeguarded Newton (bisection fallback).
// Both voxels of the face call this with identical arguments.
__device__ inline double plated_root(const CellDev& cd, double ce, double ps, double pe, double n_old,
                                     double guess) {
  const double a = cd.beta * (ps - pe);
  const double sq = cd.i00_pl * sqrt(ce);
  const double K = sq * exp(a), E = sq * exp(-a);
  const double dt = cd.dt, invF = 1.0 / kFaraday;
  const double nc2 = cd.n_c * cd.n_c, nc4 = nc2 * nc2;
  double lo = 0.0, hi = n_old + dt * E * invF;
  if (!(hi > 0.0)) return 0.0;
  double n = (guess > lo && guess < hi) ? guess : 0.5 * (lo + hi);
  // Newton converges quadratically once inside the basin; stop when the
  // step is below 1e-13 relative (the next step would be at rounding level)
  // or after a fixed budget (bisection keeps the bracket valid throughout).
  for (int it = 0; it < 60; ++it) {
    const double n2 = n * n, n4 = n2 * n2, den = nc4 + n4;
    const double f = n4 / den;
    const double g = (n - n_old) / dt + (K * f - E) * invF;
    if (g > 0.0) hi = n; else lo = n;
    const double dg = 1.0 / dt + K * invF * 4.0 * n2 * n * nc4 / (den * den);
    double nn = n - g / dg;
    if (!(nn > lo && nn < hi)) nn = 0.5 * (lo + hi);
    const double step = fabs(nn - n);
    n = nn;
    if (step <= 1e-13 * fmax(n, cd.n_c * 1e-6)) break;
  }
  return n;
}

// Interface kinetics on one solid/pore face (Sec. 2.2 eq. 2.5, Sec. 2.3
// eq. 2.8).  Every caller passes the same arguments in the same order, so
// the two voxels sharing a face evaluate bit-identical currents.
struct Kin {
  double ii, ip;                 // intercalation and plating current, A/m^2 (solid -> pore > 0)
  double d_cs, d_ce, g;          // d ii / d(cs, ce, phi_s); d/dphi_e = -g
  double p_ce, g_p, p_n;         // d ip / d(ce, phi_s, n); d/dphi_e = -g_p
};

__device__ inline Kin interface_kinetics(const CellDev& cd, int ph, double cs, double ce, double ps,
                                         double pe, double nf, bool plate, bool lin) {
  Kin k;
  if (cd.half && ph == CATHODE) {
    // Li-foil counter electrode (Sec. 2.2): i = 2 i00_ce sinh(F eta / 2RT),
    // eta = Phi_foil - phi_e; no concentration dependence, no plating
    const double sh = sinh(cd.beta * (ps - pe));
    k.ii = 2.0 * cd.i00_ce * sh;
    k.ip = k.p_ce = k.g_p = k.p_n = 0.0;
    k.d_cs = k.d_ce = 0.0;
    k.g = lin ? 2.0 * cd.i00_ce * cd.beta * sqrt(1.0 + sh * sh) : 0.0;
    return k;
  }
  const int s = ph - 1;
  const double cm = cd.cmax[s];
  const double xs = cs / cm;
  const double U = cd.U0[s] + cd.U1[s] * log((1.0 - xs) / xs);
  const double eta = ps - U - pe;
  const double sq = sqrt(cs * ce);
  const double pre = 2.0 * cd.i00[s] * sq;
  const double be = cd.beta * eta;
  const double sh = sinh(be);
  k.ii = pre * sh;
  k.ip = 0.0;
  k.p_ce = k.g_p = k.p_n = 0.0;
  if (lin) {
    const double dU = -cd.U1[s] / (xs * (1.0 - xs)) / cm;
    k.g = pre * cd.beta * sqrt(1.0 + sh * sh);   // cosh
    k.d_cs = k.ii / (2.0 * cs) - k.g * dU;
    k.d_ce = k.ii / (2.0 * ce);
  } else {
    k.g = k.d_cs = k.d_ce = 0.0;
  }
  if (plate) {
    const double a = cd.beta * (ps - pe);
    const double ea = exp(a), ema = exp(-a);
    const double n2 = nf * nf, n4 = n2 * n2;
    const double nc2 = cd.n_c * cd.n_c, nc4 = nc2 * nc2;
    const double fp = n4 / (nc4 + n4);
    const double sqe = sqrt(ce);
    k.ip = cd.i00_pl * sqe * (fp * ea - ema);
    if (lin) {
      const double den = nc4 + n4;
      const double dfp = 4.0 * n2 * nf * nc4 / (den * den);
      k.p_ce = k.ip / (2.0 * ce);
      k.g_p = cd.i00_pl * sqe * cd.beta * (fp * ea + ema);
      k.p_n = cd.i00_pl * sqe * ea * dfp;
    }
  }
  return k;
}

// ---------------------------------------------------------------- reductions
// Block-wide sum / max of one double over 256 threads (4 wavefronts of 64):
// wavefront shuffle tree, then the four wave results in fixed order.
__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
__device__ inline double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}
}  // namespace mbx
