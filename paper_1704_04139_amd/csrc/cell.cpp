// cell.cpp — cell lifecycle, batched Newton-GMRES orchestration and the C ABI.
//
// One implicit Euler step (eq. 2.13) is a damped Newton iteration on the FP64
// residual; each Newton correction solves the condensed, scaled Jacobian
// system with restarted flexible GMRES (right preconditioned, the
// preconditioned basis kept as the product saw it; classical Gram-Schmidt
// with one re-orthogonalisation).  Every kernel launch covers all cells of a
// batch; the host only reads a few per-cell scalars at sync points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <map>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mbx.h"
#include "mbx_dev.h"
#include "mbx_kernels.h"
#include "prof.h"

using namespace mbx;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(MBX_EHIP, "%s: %s", #expr, hipGetErrorString(e_));   \
  } while (0)

constexpr int kRestart = 40;          // GMRES restart length (MBX_GMRES_M overrides, at most kMaxRestart)
int restart_len() {
  static int m = -1;
  if (m < 0) {
    const char* v = std::getenv("MBX_GMRES_M");
    m = v ? std::max(4, std::min(kMaxRestart, std::atoi(v))) : kRestart;
  }
  return m;
}
constexpr double kStepLimit = 4.0;   // largest scaled Newton update taken in one iteration

bool g_verbose() {
  static int v = -1;
  if (v < 0) v = std::getenv("MBX_VERBOSE") ? 1 : 0;
  return v == 1;
}

// Coarse-correction scale of the multigrid V-cycle (MBX_MG_ALPHA overrides).
double g_mg_alpha() {
  const char* e = std::getenv("MBX_MG_ALPHA");
  return e ? std::atof(e) : 1.8;
}
// smoothing sweeps a new cell starts with (MBX_MG_NU overrides the default 2)
int g_sweeps_min() {
  const char* e = std::getenv("MBX_MG_NU");
  const int v = e ? std::atoi(e) : 2;
  return v < 1 ? 1 : (v > 6 ? 6 : v);
}
// sweeps on launched levels >= 2, at most the cell's nu (MBX_MG_NU_COARSE;
// default: no limit beyond nu)
int g_sweeps_coarse() {
  const char* e = std::getenv("MBX_MG_NU_COARSE");
  const int v = e ? std::atoi(e) : 6;
  return v < 1 ? 1 : (v > 6 ? 6 : v);
}
// GMRES iterations between two host checks of the convergence flags
// (MBX_GMRES_CHECK overrides the default 2).  A converged cell runs on to
// the next check, so shorter chunks waste fewer iterations; at 128x128x320
// 1-3 were 3-4% faster per step than 4, and 8 was 4% slower.
int g_gmres_check() {
  static int v = 0;
  if (v == 0) {
    const char* e = std::getenv("MBX_GMRES_CHECK");
    v = e ? std::max(1, std::min(std::atoi(e), kMaxRestart)) : 2;
  }
  return v;
}
constexpr int kGather = RED_NSLOT + CTL_NSLOT;
uint64_t g_next_id = 1;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t off[160];
  int n = 0;
  size_t total = 0;
  size_t add(size_t bytes) {
    size_t o = total;
    off[n++] = o;
    total += align256(bytes);
    return o;
  }
};

struct LevelDims {
  int n = 0;                       // number of levels incl. the voxel level
  int lfuse = 1;                   // first level small enough to run inside one workgroup from LDS
  int lglob = 1;                   // first level run inside that workgroup (from device memory below lfuse)
  int nx[kMaxLevels], ny[kMaxLevels], nz[kMaxLevels], ncell[kMaxLevels];
};

// Ceil-halving hierarchy down to at most kCoarseMaxCells coarse cells (at
// least one coarse level).
// LDS elements (KT) the fused coarse cycle stages for levels lf..n-1: x and b
// of every level, the operator of every level but the coarsest.
size_t fused_elems(const LevelDims& d, int lf) {
  size_t e = 0;
  for (int l = lf; l < d.n; ++l) e += (size_t)d.ncell[l] * (6 + (l + 1 < d.n ? kOpStride : 0));
  return e;
}

LevelDims level_dims(int nx, int ny, int nz, size_t kt) {
  LevelDims d;
  d.nx[0] = nx;
  d.ny[0] = ny;
  d.nz[0] = nz;
  d.ncell[0] = nx * ny * nz;
  d.n = 1;
  while (d.n < kMaxLevels) {
    const int l = d.n;
    d.nx[l] = (d.nx[l - 1] + 1) / 2;
    d.ny[l] = (d.ny[l - 1] + 1) / 2;
    d.nz[l] = (d.nz[l - 1] + 1) / 2;
    d.ncell[l] = d.nx[l] * d.ny[l] * d.nz[l];
    d.n++;
    if (d.ncell[l] <= kCoarseMaxCells) break;
  }
  d.lfuse = d.n - 1;
  while (d.lfuse > 1 && d.ncell[d.lfuse - 1] <= kFuseMaxCells &&
         fused_elems(d, d.lfuse - 1) * kt <= kFusedLdsBytes)
    --d.lfuse;
  d.lglob = d.lfuse;
  while (d.lglob > 1 && d.ncell[d.lglob - 1] <= kGlobFuseMaxCells) --d.lglob;
  return d;
}

// Captured HIP graphs of the GMRES iterations between two host checks: one
// executable graph per chunk start, each valid for the launch configuration
// (block counts, tables, sweep counts) it was captured with.  Captured on a
// private stream and replayed on the cells' stream.
struct ChunkGraphs {
  std::vector<hipGraphExec_t> exec;
  std::vector<uint64_t> key;
  hipStream_t cap = nullptr;
  void clear() {
    for (hipGraphExec_t& e : exec)
      if (e) (void)hipGraphExecDestroy(e);
    exec.clear();
    key.clear();
  }
  void release() {
    clear();
    if (cap) (void)hipStreamDestroy(cap);
    cap = nullptr;
  }
};

}  // namespace

namespace mbx {
int report_error(int code, const char* msg) { return fail(code, "%s", msg); }
}  // namespace mbx

struct mbx_cell {
  uint64_t id;
  mbx_params p;
  int nx, ny, nz, N, F_an, F_ca, n_top, nblk, m;
  int64_t n_an_vox = 0, n_ca_vox = 0;   // solid voxels per electrode (the s_ac denominators)
  bool mixed;
  hipStream_t s;
  char* dmem = nullptr;
  CellDev h{};                 // host mirror of the descriptor
  CellDev* d_desc = nullptr;   // device descriptor (single-cell launches)
  int2* d_blk = nullptr;       // device block table
  double* d_gather = nullptr;
  double* h_gather = nullptr;  // pinned
  CellDev* h_desc_pinned = nullptr;
  int* faces_an = nullptr;
  int* faces_ca = nullptr;
  LevelDims ld;
  int2* lvl_blk[kMaxLevels] = {};
  int lvl_nblk[kMaxLevels] = {};
  int2* lvlr_blk[kMaxLevels] = {};
  int lvlr_nblk[kMaxLevels] = {};
  int2* lvlh_blk[kMaxLevels] = {};   // one colour of a red-black sweep (index >= 0)
  int lvlh_nblk[kMaxLevels] = {};
  // snapshot capture (caller-owned device columns)
  double* cap_c = nullptr;
  double* cap_phi = nullptr;
  int64_t cap_ld = 0;
  int cap_capacity = 0, cap_count = 0, cap_dropped = 0;
  ChunkGraphs graphs;          // GMRES iterations of single-cell steps, replayed as HIP graphs
  int bs_smooth0 = kBlock;     // workgroup sizes of single-cell launches picked by the tuner
  int bs_matvec = kBlock;
};

namespace {

// Appends the cell's current iterate to its snapshot columns (capture on).
int capture_column(mbx_cell* c, hipStream_t s) {
  if (c->cap_capacity <= 0) return MBX_OK;
  if (c->cap_count >= c->cap_capacity) {
    ++c->cap_dropped;
    return MBX_OK;
  }
  const size_t off = (size_t)c->cap_count * (size_t)c->cap_ld;
  if (c->cap_c)
    HIPCHK(hipMemcpyAsync(c->cap_c + off, c->h.c, 8 * (size_t)c->N, hipMemcpyDeviceToDevice, s));
  if (c->cap_phi)
    HIPCHK(hipMemcpyAsync(c->cap_phi + off, c->h.phi, 8 * (size_t)c->N, hipMemcpyDeviceToDevice, s));
  ++c->cap_count;
  return MBX_OK;
}

// cells of one colour of a red-black sweep on level l (upper bound)
size_t half_cells(const LevelDims& ld, int l) { return (size_t)((ld.nx[l] + 1) / 2) * ld.ny[l] * ld.nz[l]; }

size_t kt_size(int precision) { return precision == MBX_MIXED ? sizeof(float) : sizeof(double); }

int nx_of(const LevelDims& ld) { return ld.nx[0]; }

Layout make_layout(int N, int F_an, int F_ca, int nblk, int m, size_t kt, const LevelDims& ld) {
  Layout L;
  L.add(4 * (size_t)N);                       // 0 meta
  for (int k = 0; k < 8; ++k) L.add(8 * (size_t)N);   // 1..8 c phi c_try phi_try c_old phi_old Rc Rp
  L.add(16 * (size_t)N);                      // 9 dc | dp (contiguous)
  for (int k = 0; k < 7; ++k) L.add(8 * (size_t)std::max(F_an, 1));  // 10..16 n n_try n_old Rn dn rn_jnn sq
  L.add(5 * kt * std::max(F_an, 1));          // 17 coef_an
  L.add(3 * kt * std::max(F_ca, 1));          // 18 coef_ca
  L.add(kt * (size_t)N);                      // 19 wpore
  const size_t Np = 2 * (size_t)((nx_of(ld) + 1) / 2) * ld.ny[0] * ld.nz[0];   // colour-split length
  L.add(kt * Np);                             // 20 dint (colour-split)
  L.add((size_t)(m + 1) * 2 * N * kt);        // 21 Vb
  for (int k = 0; k < 3; ++k) L.add(2 * (size_t)N * kt);  // 22..24 w z b
  L.add(2 * (size_t)N * 8);                   // 25 x (FP64)
  L.add((size_t)nblk * kPartStride * 8);      // 26 part
  L.add(0);                                   // 27 (unused)
  L.add(8 * RED_NSLOT);                       // 28 red
  L.add(4 * CTL_NSLOT);                       // 29 ictl
  L.add(8 * (size_t)gm_size(m));              // 30 gm
  L.add(4 * (size_t)std::max(F_an, 1));       // 31 faces_an
  L.add(4 * (size_t)std::max(F_ca, 1));       // 32 faces_ca
  L.add(sizeof(CellDev));                     // 33 desc
  L.add(sizeof(int2) * (size_t)nblk);         // 34 blk
  L.add(8 * kGather);                         // 35 gather
  L.add(kt * Np);                             // 36 b0 (colour-split)
  L.add(kt * std::max(F_an, 1));              // 37 cond_an
  L.add(kt * std::max(F_ca, 1));              // 38 cond_ca
  const int nc = ld.ncell[ld.n - 1];
  L.add(8 * (size_t)9 * nc * nc);             // 39 cinv[0]
  L.add(8 * (size_t)9 * nc * nc);             // 40 cinv[1]
  for (int l = 1; l < ld.n; ++l) {            // 41 + 7(l-1): x, b, op0, op1, blk, blkr, blkh
    const size_t n = ld.ncell[l];
    L.add(3 * n * kt);
    L.add(3 * n * kt);
    L.add(kOpStride * n * kt);
    L.add(kOpStride * n * kt);
    L.add(sizeof(int2) * ((n + kBlock - 1) / kBlock));
    L.add(sizeof(int2) * ((4 * n + kBlock - 1) / kBlock));
    L.add(sizeof(int2) * ((half_cells(ld, l) + kBlock - 1) / kBlock));
  }
  L.add(sizeof(int2) * ((half_cells(ld, 0) + kBlock - 1) / kBlock));   // 41 + 7(n-1): level-0 blkh
  L.add(16 * (size_t)std::max(F_an + F_ca, 1));                        // 42 + 7(n-1): face results
  L.add((size_t)m * 2 * N * kt);                                       // 43 + 7(n-1): flexible-GMRES basis Z
  L.add(4 * Np);                                                       // 44 + 7(n-1): meta, colour-split
  L.add(kt * Np);                                                      // 45 + 7(n-1): level-0 iterate, colour-split
  L.add(8 * (size_t)N);                                                // 46 + 7(n-1): c at the step before u^n (adaptive runs)
  L.add(8 * (size_t)std::max(F_an, 1));                                // 47 + 7(n-1): n at the step before u^n
  L.add(kt * (size_t)std::max(2 * (F_an + F_ca), 1));                  // 48 + 7(n-1): cond_rb
  return L;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

}  // namespace

namespace mbx {
// Voltage cutoff (V_cut > 0): reached when a charge (I_app >= 0) brings the
// cell voltage up to V_cut, or a discharge brings it down to V_cut.
bool cutoff_reached(const mbx_params& p, double V) {
  if (!(p.V_cut > 0.0)) return false;
  return p.I_app >= 0.0 ? V >= p.V_cut : V <= p.V_cut;
}
}  // namespace mbx

namespace {

// Smallest double >= 1/d (d >= 1), the reciprocal the kernels' divmod needs:
// RN(1/d), moved up one step when it lies below 1/d (the fused product
// r*d - 1 carries the exact sign).
double rcp_up(int d) {
  double r = 1.0 / d;
  if (std::fma(r, (double)d, -1.0) < 0.0) r = std::nextafter(r, 2.0);
  return r;
}

int check_params(const mbx_params* p) {
  if (!p) return fail(MBX_EINVAL, "null parameter struct");
  if (!finite_pos(p->T) || !finite_pos(p->h) || !finite_pos(p->c0) || !finite_pos(p->De) ||
      !finite_pos(p->kappa) || !finite_pos(p->thermo) || !finite_pos(p->n_c) || !std::isfinite(p->I_app))
    return fail(MBX_EINVAL, "T, h, c0, De, kappa, thermo, n_c must be finite and > 0; I_app finite");
  if (!(p->x0 > 0.0 && p->x0 < 1.0) || !(p->y0 > 0.0 && p->y0 < 1.0))
    return fail(MBX_EINVAL, "initial stoichiometries must lie in (0, 1)");
  if (!(p->tplus >= 0.0 && p->tplus < 1.0)) return fail(MBX_EINVAL, "tplus must lie in [0, 1)");
  for (int s = 0; s < 2; ++s) {
    if (!finite_pos(p->Ds[s]) || !finite_pos(p->sigma[s]) || !finite_pos(p->cmax[s]) || !finite_pos(p->i00[s]) ||
        !std::isfinite(p->U0[s]) || !std::isfinite(p->U1[s]))
      return fail(MBX_EINVAL, "solid parameters must be finite and > 0 (U0, U1 finite)");
  }
  if (!(std::isfinite(p->i00_pl) && p->i00_pl >= 0.0)) return fail(MBX_EINVAL, "i00_pl must be finite and >= 0");
  if (p->precision != MBX_FP64 && p->precision != MBX_MIXED) return fail(MBX_EINVAL, "unknown precision mode");
  if (p->plating != 0 && p->plating != 1) return fail(MBX_EINVAL, "plating must be 0 or 1");
  if (!(std::isfinite(p->V_cut) && p->V_cut >= 0.0)) return fail(MBX_EINVAL, "V_cut must be finite and >= 0");
  if (p->graphs != 0 && p->graphs != 1) return fail(MBX_EINVAL, "graphs must be 0 or 1");
  if (!(std::isfinite(p->i00_ce) && p->i00_ce >= 0.0)) return fail(MBX_EINVAL, "i00_ce must be finite and >= 0");
  return MBX_OK;
}

void fill_constants(CellDev& h, const mbx_params& p, int nx, int ny) {
  h.h = p.h;
  h.A = p.h * p.h;
  h.Vol = p.h * p.h * p.h;
  h.RT = kGasR * p.T;
  h.VT = h.RT / kFaraday;
  h.beta = kFaraday / (2.0 * h.RT);
  h.c0 = p.c0;
  h.x0 = p.x0;
  h.y0 = p.y0;
  h.De = p.De;
  h.kappa = p.kappa;
  h.tplus = p.tplus;
  h.thermo = p.thermo;
  for (int s = 0; s < 2; ++s) {
    // no Li diffusion in a half cell's foil (Sec. 2.2: eq. 2.1 holds in the graphite only)
    h.Ds[s] = (s == 1 && h.half) ? 0.0 : p.Ds[s];
    h.sigma[s] = p.sigma[s];
    h.cmax[s] = p.cmax[s];
    h.i00[s] = p.i00[s];
    h.U0[s] = p.U0[s];
    h.U1[s] = p.U1[s];
  }
  h.i00_pl = p.i00_pl;
  h.i00_ce = p.i00_ce;
  h.n_c = p.n_c;
  h.I_app = p.I_app;
  h.plating = p.plating;
  h.mu_ref = std::max(std::fabs(p.I_app) / (nx * (double)ny * h.A), 1.0);
  h.Kd = p.kappa * (1.0 - p.tplus) * p.thermo * h.RT / (kFaraday * p.h);
}

// Constants of the scaled operator that depend on the step size.
void fill_step_constants(CellDev& h, double dt) {
  const double hh = h.h, mu = h.mu_ref;
  h.dt = dt;
  h.Gk = h.kappa * h.VT / (hh * mu);
  h.tth = (1.0 - h.tplus) * h.thermo;
  h.Dh = h.De * dt / (hh * hh);
  h.tau = h.tplus * dt * mu / (kFaraday * hh * h.c0);
  h.Ke = dt * mu / (hh * kFaraday * h.c0);
  h.Gcol = 2.0 * h.sigma[0] * h.VT / (hh * mu);
  for (int s = 0; s < 2; ++s) {
    h.Dsh[s] = h.Ds[s] * dt / (hh * hh);
    h.Gs[s] = h.sigma[s] * h.VT / (hh * mu);
    // the foil's concentration row carries no interface flux
    h.Ks[s] = (s == 1 && h.half) ? 0.0 : dt * mu / (hh * kFaraday * h.cmax[s]);
  }
  // same-phase couplings of the level-0 smoother per operator and label, in both Krylov types
  const double gs[2][3] = {{h.Dh, h.Dsh[0], h.Dsh[1]}, {h.Gk, h.Gs[0], h.Gs[1]}};
  for (int op = 0; op < 2; ++op)
    for (int l = 0; l < 3; ++l) {
      h.gsame_d[op][l] = gs[op][l];
      h.gsame_f[op][l] = (float)gs[op][l];
    }
}

// A batch of cells sharing every launch.
struct Batch {
  std::vector<mbx_cell*> cells;
  hipStream_t s = nullptr;
  CellDev* d_desc = nullptr;
  CellDev* h_desc = nullptr;   // pinned
  int2* d_blk = nullptr;
  double* d_gather = nullptr;
  double* h_gather = nullptr;  // pinned
  int nblk = 0;
  bool owned = false;
  bool mixed = false;
  bool use_graphs = false;      // replay the GMRES iterations as captured HIP graphs
  ChunkGraphs* graphs = nullptr;
  int m = kRestart;
  int maxlev = 0;
  int maxfuse = 1;
  int maxglob = 1;
  int2* lvl_blk[kMaxLevels] = {};
  int lvl_nblk[kMaxLevels] = {};
  int2* lvlr_blk[kMaxLevels] = {};
  int lvlr_nblk[kMaxLevels] = {};
  int2* lvlh_blk[kMaxLevels] = {};
  int lvlh_nblk[kMaxLevels] = {};
  BatchLaunch bl() const {
    BatchLaunch b{};
    for (const mbx_cell* c : cells) {
      const double N = c->N, Fa = c->F_an, Fc = c->F_ca, kt = c->mixed ? 4.0 : 8.0;
      // state, old state, labels and rows of every voxel; the face lists; the
      // plated amounts (old, guess, new) and rows; with the linearisation the
      // face records, conductances and the pore 1/c weights
      b.bytes_residual[0] += 44.0 * N + 4.0 * (Fa + Fc) + 32.0 * Fa;
      b.bytes_residual[1] += 44.0 * N + 4.0 * (Fa + Fc) + 32.0 * Fa + kt * N + (6.0 * kt + 16.0) * Fa + 4.0 * kt * Fc;
      b.bytes_matvec += (4.0 + 5.0 * kt) * N + 5.0 * kt * Fa + 3.0 * kt * Fc;
      // one half sweep: meta and b of the colour's voxels, x of the other
      // colour, the new x; averaged over the two operators: the colour's
      // interface conductances (potential operator, one per face) and its
      // per-voxel interface diagonal (concentration operator)
      b.bytes_smooth0 += (2.0 + 1.5 * kt) * N + 0.5 * kt * (Fa + Fc) + 0.25 * kt * N;
    }
    b.cells = d_desc;
    // a single cell needs no block tables: kernels map block b to {0, b}
    const bool one = cells.size() == 1;
    b.blk = one ? nullptr : d_blk;
    b.nblk = nblk;
    b.ncell = (int)cells.size();
    b.faces_single = one ? cells[0]->F_an + cells[0]->F_ca : 0;
    b.n_single = one ? cells[0]->N : 0;
    b.bs_smooth0 = one ? cells[0]->bs_smooth0 : kBlock;
    b.bs_matvec = one ? cells[0]->bs_matvec : kBlock;
    b.maxlev = maxlev;
    b.maxfuse = maxfuse;
    b.maxglob = maxglob;
    b.fused_lds = 0;
    b.max_nu = 1;
    b.max_nu_c = 1;
    for (const mbx_cell* c : cells) {
      b.fused_lds = std::max(b.fused_lds, fused_elems(c->ld, c->ld.lfuse));
      b.max_nu = std::max(b.max_nu, c->h.nu);
      b.max_nu_c = std::max(b.max_nu_c, std::min(c->h.nu, c->h.nu_c));
    }
    for (int l = 0; l < kMaxLevels; ++l) {
      b.lvl_blk[l] = one ? nullptr : lvl_blk[l];
      b.lvl_nblk[l] = lvl_nblk[l];
      b.lvlr_blk[l] = one ? nullptr : lvlr_blk[l];
      b.lvlr_nblk[l] = lvlr_nblk[l];
      b.lvlh_blk[l] = one ? nullptr : lvlh_blk[l];
      b.lvlh_nblk[l] = lvlh_nblk[l];
    }
    return b;
  }
  int upload() {
    for (size_t c = 0; c < cells.size(); ++c) h_desc[c] = cells[c]->h;
    HIPCHK(hipMemcpyAsync(d_desc, h_desc, sizeof(CellDev) * cells.size(), hipMemcpyHostToDevice, s));
    std::vector<char> on(cells.size());
    for (size_t c = 0; c < cells.size(); ++c) on[c] = cells[c]->h.active != 0;
    if (int e = set_active(on)) return e;
    // the pinned staging buffer is rewritten by the next upload
    HIPCHK(hipStreamSynchronize(s));
    return MBX_OK;
  }
  // Host copies of the full block tables of a multi-cell batch.  Launches
  // cover only the cells marked on: the device tables are rewritten with the
  // blocks of those cells whenever the set changes, so cells that have
  // finished cost no dispatched workgroups.  (An empty set keeps the tables.)
  std::vector<int2> full_blk, full_lvl[3][kMaxLevels], cur_tab[1 + 3 * kMaxLevels];
  std::vector<char> cur_on;
  int set_active(const std::vector<char>& on) {
    if (cells.size() < 2 || on == cur_on) return MBX_OK;
    bool any = false;
    for (char o : on) any = any || o;
    if (!any) return MBX_OK;
    cur_on = on;
    auto filt = [&](const std::vector<int2>& full, std::vector<int2>& out, int2* dev, int& count) -> int {
      out.clear();
      for (const int2& e : full)
        if (on[e.x]) out.push_back(e);
      count = (int)out.size();
      if (count) HIPCHK(hipMemcpyAsync(dev, out.data(), sizeof(int2) * out.size(), hipMemcpyHostToDevice, s));
      return MBX_OK;
    };
    int e = filt(full_blk, cur_tab[0], d_blk, nblk);
    for (int l = 0; l < maxlev && e == MBX_OK; ++l) {
      if (lvl_blk[l]) e = filt(full_lvl[0][l], cur_tab[1 + l], lvl_blk[l], lvl_nblk[l]);
      if (lvlr_blk[l] && e == MBX_OK) e = filt(full_lvl[1][l], cur_tab[1 + kMaxLevels + l], lvlr_blk[l], lvlr_nblk[l]);
      if (lvlh_blk[l] && e == MBX_OK)
        e = filt(full_lvl[2][l], cur_tab[1 + 2 * kMaxLevels + l], lvlh_blk[l], lvlh_nblk[l]);
    }
    if (e != MBX_OK) return e;
    // the host vectors are the copy sources
    HIPCHK(hipStreamSynchronize(s));
    return MBX_OK;
  }
  int gather() {
    launch_gather_ctl(bl(), d_gather, s);
    // a rejected launch leaves its error for the next query on this thread
    // (a library such as rocPRIM would report it as its own): surface it here
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h_gather, d_gather, sizeof(double) * kGather * cells.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return MBX_OK;
  }
  double red(int c, int slot) const { return h_gather[(size_t)c * kGather + slot]; }
  int ctl(int c, int slot) const { return (int)h_gather[(size_t)c * kGather + RED_NSLOT + slot]; }
  void release() {
    if (!owned) return;
    (void)hipFree(d_desc);
    (void)hipFree(d_blk);
    (void)hipFree(d_gather);
    for (int l = 0; l < kMaxLevels; ++l) {
      if (lvl_blk[l]) (void)hipFree(lvl_blk[l]);
      if (lvlr_blk[l]) (void)hipFree(lvlr_blk[l]);
      if (lvlh_blk[l]) (void)hipFree(lvlh_blk[l]);
    }
    (void)hipHostFree(h_desc);
    (void)hipHostFree(h_gather);
    owned = false;
  }
};

Batch single(mbx_cell* c) {
  Batch b;
  b.cells = {c};
  b.s = c->s;
  b.d_desc = c->d_desc;
  b.h_desc = c->h_desc_pinned;
  b.d_blk = c->d_blk;
  b.d_gather = c->d_gather;
  b.h_gather = c->h_gather;
  b.nblk = c->nblk;
  b.mixed = c->mixed;
  b.m = c->m;
  b.graphs = &c->graphs;
  b.use_graphs = c->p.graphs != 0;
  b.maxlev = c->ld.n;
  b.maxfuse = c->ld.lfuse;
  b.maxglob = c->ld.lglob;
  for (int l = 0; l < c->ld.n; ++l) {
    b.lvl_blk[l] = c->lvl_blk[l];
    b.lvl_nblk[l] = c->lvl_nblk[l];
    b.lvlr_blk[l] = c->lvlr_blk[l];
    b.lvlr_nblk[l] = c->lvlr_nblk[l];
    b.lvlh_blk[l] = c->lvlh_blk[l];
    b.lvlh_nblk[l] = c->lvlh_nblk[l];
  }
  return b;
}

// Cached multi-cell batch (re-used while the same cells are stepped together).
struct BatchCache {
  std::vector<uint64_t> ids;
  Batch b;
  ChunkGraphs graphs;
} g_batch_cache;
// guards g_batch_cache: batched steps from different threads (a server's
// worker and a caller) run one at a time, and destroying a cell that the
// cached batch holds waits for them
std::mutex g_batch_mu;

// The batch lives in the cache (its device block tables carry state: the
// active-cell compaction), so callers work on the cached object itself.
int make_batch(mbx_cell* const* cells, int n, Batch*& out) {
  std::vector<uint64_t> ids(n);
  for (int i = 0; i < n; ++i) ids[i] = cells[i]->id;
  if (g_batch_cache.b.owned && g_batch_cache.ids == ids) {
    out = &g_batch_cache.b;
    return MBX_OK;
  }
  g_batch_cache.b.release();
  g_batch_cache.graphs.clear();
  Batch b;
  b.cells.assign(cells, cells + n);
  b.graphs = &g_batch_cache.graphs;
  b.use_graphs = true;
  for (int c = 0; c < n; ++c) b.use_graphs = b.use_graphs && cells[c]->p.graphs != 0;
  b.s = cells[0]->s;
  b.mixed = cells[0]->mixed;
  b.m = cells[0]->m;
  std::vector<int2> tab;
  for (int c = 0; c < n; ++c)
    for (int k = 0; k < cells[c]->nblk; ++k) tab.push_back(make_int2(c, k));
  b.nblk = (int)tab.size();
  for (int c = 0; c < n; ++c) {
    b.maxlev = std::max(b.maxlev, cells[c]->ld.n);
    b.maxfuse = std::max(b.maxfuse, cells[c]->ld.lfuse);
    b.maxglob = std::max(b.maxglob, cells[c]->ld.lglob);
  }
  for (int l = 0; l < b.maxlev; ++l) {
    for (int pass = 0; pass < 3; ++pass) {
      if (l == 0 && pass < 2) continue;
      std::vector<int2> lt;
      for (int c = 0; c < n; ++c)
        if (l < cells[c]->ld.n) {
          const int nb =
              pass == 0 ? cells[c]->lvl_nblk[l] : pass == 1 ? cells[c]->lvlr_nblk[l] : cells[c]->lvlh_nblk[l];
          for (int k = 0; k < nb; ++k) lt.push_back(make_int2(c, k));
        }
      int2*& dst = pass == 0 ? b.lvl_blk[l] : pass == 1 ? b.lvlr_blk[l] : b.lvlh_blk[l];
      (pass == 0 ? b.lvl_nblk[l] : pass == 1 ? b.lvlr_nblk[l] : b.lvlh_nblk[l]) = (int)lt.size();
      b.full_lvl[pass][l] = lt;
      HIPCHK(hipMalloc(&dst, sizeof(int2) * std::max<size_t>(lt.size(), 1)));
      HIPCHK(hipMemcpyAsync(dst, lt.data(), sizeof(int2) * lt.size(), hipMemcpyHostToDevice, b.s));
    }
  }
  HIPCHK(hipMalloc(&b.d_desc, sizeof(CellDev) * n));
  HIPCHK(hipMalloc(&b.d_blk, sizeof(int2) * tab.size()));
  HIPCHK(hipMalloc(&b.d_gather, sizeof(double) * kGather * n));
  HIPCHK(hipHostMalloc(&b.h_desc, sizeof(CellDev) * n, hipHostMallocDefault));
  HIPCHK(hipHostMalloc(&b.h_gather, sizeof(double) * kGather * n, hipHostMallocDefault));
  HIPCHK(hipMemcpyAsync(b.d_blk, tab.data(), sizeof(int2) * tab.size(), hipMemcpyHostToDevice, b.s));
  HIPCHK(hipStreamSynchronize(b.s));
  b.full_blk = tab;
  b.cur_on.assign(n, 1);
  b.owned = true;
  g_batch_cache.ids = ids;
  g_batch_cache.b = b;
  out = &g_batch_cache.b;
  return MBX_OK;
}

// ------------------------------------------------------------------ GMRES
// Launch configuration a captured chunk depends on (everything the kernel
// arguments and grid sizes are made of).
uint64_t launch_key(const Batch& B, const BatchLaunch& b, int k0, int k1) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
  mix((uint64_t)(uintptr_t)b.cells);
  mix((uint64_t)(uintptr_t)b.blk);
  mix((uint64_t)b.nblk);
  mix((uint64_t)b.ncell);
  mix((uint64_t)b.maxlev);
  mix((uint64_t)b.maxfuse);
  mix((uint64_t)b.maxglob);
  mix((uint64_t)b.fused_lds);
  mix((uint64_t)b.max_nu);
  mix((uint64_t)b.max_nu_c);
  mix((uint64_t)b.faces_single);
  for (int l = 0; l < kMaxLevels; ++l) {
    mix((uint64_t)(uintptr_t)b.lvl_blk[l] ^ ((uint64_t)b.lvl_nblk[l] << 48));
    mix((uint64_t)(uintptr_t)b.lvlr_blk[l] ^ ((uint64_t)b.lvlr_nblk[l] << 48));
    mix((uint64_t)(uintptr_t)b.lvlh_blk[l] ^ ((uint64_t)b.lvlh_nblk[l] << 48));
  }
  mix((uint64_t)(uintptr_t)B.d_gather);
  mix((uint64_t)(uintptr_t)B.h_gather);
  mix((uint64_t)B.cells.size());
  mix((uint64_t)B.m);
  mix((uint64_t)k0 | ((uint64_t)k1 << 32));
  return h;
}

// GMRES iterations k0 .. k1-1 of every running cell of the batch, then the
// flags and reduction slots gathered to the host.
template <typename KT>
void launch_chunk(const BatchLaunch& bl, int k0, int k1, double* d_gather, int ncells, double* h_gather,
                  hipStream_t s, bool copy_out) {
  for (int k = k0; k < k1; ++k) {
    launch_precond<KT>(bl, k, 0, s);
    launch_matvec<KT>(bl, VEC_Z, VEC_W, 0, k, s);
    // classical Gram-Schmidt with one re-orthogonalisation (CGS2)
    launch_multidot<KT>(bl, k, 0, s);   // H(:,k) = V^T w
    launch_orth_dots<KT>(bl, k, s);     // w -= V H(:,k); tmp = V^T w
    launch_orth<KT>(bl, k, 1, s);       // w -= V tmp; H(:,k) += tmp; H(k+1,k) = |w|; Givens step of column k
    launch_scale_next<KT>(bl, k, s);    // V_{k+1} = w / |w| (cells still iterating)
  }
  if (copy_out) {
    launch_gather_ctl(bl, d_gather, s);
    (void)hipMemcpyAsync(h_gather, d_gather, sizeof(double) * kGather * ncells, hipMemcpyDeviceToHost, s);
  }
}

// The chunk as a HIP graph: captured on the first use of a configuration,
// replayed afterwards (one launch and one synchronisation per chunk).
template <typename KT>
int run_chunk_graph(Batch& B, int k0, int k1) {
  ChunkGraphs& G = *B.graphs;
  const BatchLaunch bl = B.bl();
  const uint64_t key = launch_key(B, bl, k0, k1);
  const size_t slot = (size_t)k0;
  if (G.exec.size() <= slot) {
    G.exec.resize(slot + 1, nullptr);
    G.key.resize(slot + 1, 0);
  }
  if (!G.exec[slot] || G.key[slot] != key) {
    if (G.exec[slot]) {
      (void)hipGraphExecDestroy(G.exec[slot]);
      G.exec[slot] = nullptr;
    }
    if (!G.cap) HIPCHK(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
    launch_chunk<KT>(bl, k0, k1, B.d_gather, (int)B.cells.size(), B.h_gather, G.cap, true);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(G.cap, &g);
    if (ec != hipSuccess || !g) return fail(MBX_EHIP, "GMRES graph capture: %s", hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(&G.exec[slot], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      G.exec[slot] = nullptr;
      return fail(MBX_EHIP, "GMRES graph instantiation: %s", hipGetErrorString(ei));
    }
    G.key[slot] = key;
  }
  HIPCHK(hipGraphLaunch(G.exec[slot], B.s));
  HIPCHK(hipStreamSynchronize(B.s));
  return MBX_OK;
}

template <typename KT>
int gmres(Batch& B, int max_iters, int* iters_out) {
  const int m = B.m;
  const int check = g_gmres_check();
  // kernel timing records events between launches: direct launches then
  const bool graphs = B.use_graphs && B.graphs && !prof_active();
  int total = 0;
  launch_gm_start<KT>(B.bl(), 1, B.s);
  const int refine = sizeof(KT) < sizeof(double);
  launch_gm_flags(B.bl(), 1, refine, B.s);
  while (total < max_iters) {
    int k = 0;
    for (int k0 = 0; k0 < m;) {
      const int k1 = std::min(k0 + check, m);
      if (graphs) {
        if (int e = run_chunk_graph<KT>(B, k0, k1)) return e;
      } else {
        launch_chunk<KT>(B.bl(), k0, k1, B.d_gather, (int)B.cells.size(), B.h_gather, B.s, false);
        if (int e = B.gather()) return e;
      }
      k = k1;
      bool running = false;
      std::vector<char> on(B.cells.size());
      for (size_t c = 0; c < B.cells.size(); ++c) {
        on[c] = B.cells[c]->h.active && B.ctl(c, CTL_DONE) == 0;
        running = running || on[c];
      }
      if (!running) break;
      // launch only the cells still iterating (a captured graph keeps its
      // tables: cells that finished leave its kernels at their flag test)
      if (!graphs)
        if (int e = B.set_active(on)) return e;
      k0 = k1;
    }
    total += k;
    {
      std::vector<char> on(B.cells.size());
      for (size_t c = 0; c < B.cells.size(); ++c) on[c] = B.cells[c]->h.active != 0;
      if (int e = B.set_active(on)) return e;   // cycle end: every active cell
    }
    launch_backsolve(B.bl(), B.s);
    launch_update_x<KT>(B.bl(), B.s);          // flexible GMRES: x += Z y
    launch_true_residual<KT>(B.bl(), B.s);   // w = b - J x for the cells that restart
    launch_gm_start<KT>(B.bl(), 0, B.s);
    launch_gm_flags(B.bl(), 0, refine, B.s);
    if (int e = B.gather()) return e;
    bool all = true;
    for (size_t c = 0; c < B.cells.size(); ++c) {
      if (B.cells[c]->h.active && B.ctl(c, CTL_DONE) != 3) all = false;
      if (g_verbose() && B.cells[c]->h.active)
        fprintf(stderr, "[mbx] cell %zu gmres cycle end: iters %d state %d |r| %.3e tol %.3e beta0 %.3e\n", c,
                total, B.ctl(c, CTL_DONE), std::sqrt(B.red(c, RED_BSQ)), B.red(c, RED_TOL), B.red(c, RED_BETA0));
    }
    if (all) break;
  }
  if (iters_out) *iters_out = total;
  return MBX_OK;
}

// ------------------------------------------------------------------ Newton
constexpr int kSweepsMax = 6;         // most smoothing sweeps per side the autotuning gives a cell
constexpr int kSlowSolve = 60;        // Krylov iterations of one correction that call for more smoothing
constexpr int kStallMinIter = 8;      // Newton iterations before stagnation is tested
constexpr size_t kStallWindow = 4;
constexpr int kMaxHalvings = 1;       // a failed step is retried once, as two half steps
constexpr double kEtaMax = 0.1;        // loosest GMRES relative tolerance of a Newton correction
constexpr double kEwGamma = 0.9;
template <typename KT>
int newton(Batch& B, double dt, int* status, mbx_step_info* infos) {
  const int nc = (int)B.cells.size();
  auto t0 = std::chrono::steady_clock::now();
  std::vector<int> st(nc, 1);   // 1 running, 0 converged, < 0 failed
  // both modes meet the forcing term with the true (FP64-accumulated)
  // residual: the mixed mode refines its FP32 corrections inside GMRES
  const double eta_max = kEtaMax;
  std::vector<double> rn(nc), rmax(nc), res0(nc), eta(nc, eta_max), du(nc, 0.0), lam(nc, 1.0), mr(nc), dnm(nc, 0.0),
      qconv(nc, 1.0);
  // FP32 Krylov cannot resolve relative residuals much below 1e-6
  const double eta_floor = B.cells[0]->p.krylov_rtol;
  std::vector<int> nit(nc, 0), kit(nc, 0);
  std::vector<std::vector<double>> rhist(nc);   // accepted residual 2-norms
  // snapshot columns at the step start: a failed step drops its own again
  std::vector<int> cap0(nc), capd0(nc);
  for (int c = 0; c < nc; ++c) {
    cap0[c] = B.cells[c]->cap_count;
    capd0[c] = B.cells[c]->cap_dropped;
  }
  for (int c = 0; c < nc; ++c) {
    mbx_cell* cl = B.cells[c];
    fill_step_constants(cl->h, dt);
    cl->h.elim_n = 1;
    cl->h.active = 1;
    cl->h.lam = 1.0;
    cl->h.m = B.m;
  }
  if (int e = B.upload()) return e;
  launch_copy_state(B.bl(), 2, B.s);   // u^n <- state
  launch_copy_state(B.bl(), 1, B.s);   // trial <- state
  launch_residual<KT>(B.bl(), true, B.s);
  if (int e = B.gather()) return e;
  for (int c = 0; c < nc; ++c) {
    rn[c] = std::sqrt(B.red(c, RED_RSQ));
    mr[c] = std::sqrt(B.red(c, RED_MSQ));
    rmax[c] = B.red(c, RED_RMAX);
    res0[c] = rmax[c];
    if (!std::isfinite(rn[c])) st[c] = MBX_ENAN;
  }
  int newton_max = B.cells[0]->p.newton_max;
  for (int it = 1; it <= newton_max; ++it) {
    bool any = false;
    for (int c = 0; c < nc; ++c) {
      mbx_cell* cl = B.cells[c];
      cl->h.active = st[c] == 1;
      cl->h.rtol = eta[c];
      any = any || st[c] == 1;
    }
    if (!any) break;
    if (int e = B.upload()) return e;
    launch_mg_setup<KT>(B.bl(), B.s);
    launch_rhs<KT>(B.bl(), B.s);
    int kits = 0;
    if (int e = gmres<KT>(B, B.cells[0]->p.krylov_max, &kits)) return e;
    if (int e = B.gather()) return e;
    for (int c = 0; c < nc; ++c) {
      if (st[c] != 1) continue;
      const int its = B.ctl(c, CTL_ITERS);
      kit[c] += its;
      // sweep autotuning: a cell whose corrections need many Krylov
      // iterations gets more smoothing from its next solve on (kept for
      // later steps; more sweeps cost less than the iterations they save)
      CellDev& h = B.cells[c]->h;
      if (its > kSlowSolve && h.nu < kSweepsMax) {
        h.nu = std::min(kSweepsMax, h.nu + 2);
        h.nu_f = h.nu;
        if (g_verbose()) fprintf(stderr, "[mbx] cell %d: %d Krylov iterations, smoothing sweeps -> %d\n", c, its, h.nu);
      }
    }
    launch_direction<KT>(B.bl(), B.s);
    if (int e = B.gather()) return e;
    // step-length limiter: no scaled update larger than kStepLimit (potentials
    // in RT/F, concentrations relative to c0 / c_max), then halving until the
    // state is admissible and (FP64) the scaled residual norm does not grow
    std::vector<int> searching(nc, 0);
    for (int c = 0; c < nc; ++c) {
      searching[c] = st[c] == 1;
      if (!searching[c]) continue;
      const double dfull = B.red(c, RED_DUMAX);
      lam[c] = (std::isfinite(dfull) && dfull > kStepLimit) ? kStepLimit / dfull : 1.0;
      if (!std::isfinite(dfull)) {
        if (g_verbose()) fprintf(stderr, "[mbx] cell %d newton %d: non-finite Newton direction\n", c, it);
        st[c] = MBX_ENAN;
        searching[c] = 0;
      }
    }
    for (int hlv = 0; hlv <= 20; ++hlv) {
      bool anys = false;
      for (int c = 0; c < nc; ++c) {
        B.cells[c]->h.active = searching[c];
        B.cells[c]->h.lam = lam[c];
        anys = anys || searching[c];
      }
      if (!anys) break;
      if (int e = B.upload()) return e;
      launch_trial(B.bl(), B.s);
      if (int e = B.gather()) return e;
      std::vector<double> dmax(nc, 0.0);
      for (int c = 0; c < nc; ++c) {
        if (!searching[c]) continue;
        dmax[c] = B.red(c, RED_DUMAX);
        if (B.red(c, RED_BAD) > 0.0) {
          B.cells[c]->h.active = 0;
          lam[c] *= 0.5;
        }
      }
      if (int e = B.upload()) return e;
      launch_residual<KT>(B.bl(), true, B.s);
      if (int e = B.gather()) return e;
      for (int c = 0; c < nc; ++c) {
        if (!searching[c] || !B.cells[c]->h.active) continue;
        // the scaled FP64 residual 2-norm must not grow (both modes: the mixed
        // mode's corrections meet their tolerance with the true residual)
        const double r1 = std::sqrt(B.red(c, RED_RSQ));
        const double m1 = std::sqrt(B.red(c, RED_MSQ));
        // once the iterate meets the residual tolerance the remaining
        // differences are rounding noise: take the full step
        const bool ok = std::isfinite(r1) && (r1 <= rn[c] || rmax[c] <= B.cells[c]->p.res_tol || hlv == 20);
        if (ok) {
          searching[c] = 0;
          du[c] = dmax[c] / lam[c];
          dnm[c] = B.red(c, RED_DNMAX);
          const double mprev = mr[c];
          const double rprev = rn[c];
          rn[c] = r1;
          mr[c] = m1;
          rmax[c] = B.red(c, RED_RMAX);
          const double ratio = rprev > 0.0 ? r1 / rprev : 0.0;
          qconv[c] = ratio;
          (void)mprev;
          // forcing term (Eisenstat-Walker, choice 2, gamma 0.9, alpha 2):
          // loose while Newton is far from the root, tight once it converges
          double e = kEwGamma * ratio * ratio;
          const double prev = kEwGamma * eta[c] * eta[c];
          if (prev > 0.1) e = std::max(e, prev);
          eta[c] = std::max(eta_floor, std::min(eta_max, e));
        } else {
          lam[c] *= 0.5;
        }
      }
    }
    for (int c = 0; c < nc; ++c) {
      B.cells[c]->h.active = 0;
      if (st[c] != 1) continue;
      if (searching[c]) {
        st[c] = MBX_ENEWTON;
        continue;
      }
      B.cells[c]->h.active = 1;
      nit[c] = it;
    }
    if (int e = B.upload()) return e;
    launch_copy_state(B.bl(), 0, B.s);   // accept: state <- trial
    for (int c = 0; c < nc; ++c)         // Newton stage snapshots
      if (B.cells[c]->h.active)
        if (int e = capture_column(B.cells[c], B.s)) return e;
    for (int c = 0; c < nc; ++c) {
      if (st[c] != 1) continue;
      const mbx_params& p = B.cells[c]->p;
      if (g_verbose())
        fprintf(stderr, "[mbx] cell %d newton %d: lam %.3g |r|2 %.3e |r|inf %.3e merit %.3e du %.3e dn %.3e eta %.1e gmres %d (beta0 %.3e)\n",
                c, it, lam[c], rn[c], rmax[c], mr[c], du[c], dnm[c], eta[c], B.ctl(c, CTL_ITERS), B.red(c, RED_BETA0));
      // error left after this update: the update itself, or (contraction
      // q = residual ratio of this iteration) the estimate |du| q / (1 - q)
      const double dmx = std::max(du[c], dnm[c]);
      const double q = qconv[c];
      const double err = (q < 0.5) ? dmx * q / (1.0 - q) : dmx;
      if (lam[c] == 1.0 && rmax[c] <= p.res_tol && (dmx <= p.newton_tol || err <= p.newton_tol)) {
        st[c] = 0;
        continue;
      }
      // stagnation: no 10% decrease of the residual 2-norm over the last
      // kStallWindow iterations; give up early (the caller may split the step)
      rhist[c].push_back(rn[c]);
      const size_t h = rhist[c].size();
      if (it >= kStallMinIter && h > kStallWindow && rn[c] > 0.9 * rhist[c][h - 1 - kStallWindow]) {
        if (g_verbose()) fprintf(stderr, "[mbx] cell %d newton %d: stagnated\n", c, it);
        st[c] = MBX_ENEWTON;
      }
    }
  }
  // roll back failures, outputs for the converged cells
  for (int c = 0; c < nc; ++c) {
    if (st[c] == 1) st[c] = MBX_ENEWTON;
    B.cells[c]->h.active = st[c] < 0;
    if (st[c] < 0) {
      B.cells[c]->cap_count = cap0[c];
      B.cells[c]->cap_dropped = capd0[c];
    }
  }
  if (int e = B.upload()) return e;
  launch_copy_state(B.bl(), 3, B.s);
  for (int c = 0; c < nc; ++c) B.cells[c]->h.active = 1;
  if (int e = B.upload()) return e;
  launch_outputs(B.bl(), B.s);
  if (int e = B.gather()) return e;
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int c = 0; c < nc; ++c) {
    status[c] = st[c];
    if (infos) {
      mbx_step_info& in = infos[c];
      in.newton_iters = nit[c];
      in.krylov_iters = kit[c];
      in.res0 = res0[c];
      in.res_final = rmax[c];
      in.du_final = std::max(du[c], dnm[c]);
      in.V = B.red(c, RED_VSUM) / B.cells[c]->n_top;
      in.wall_s = wall;
    }
  }
  return MBX_OK;
}

int run_step(Batch& B, double dt, int* status, mbx_step_info* infos) {
  return B.mixed ? newton<float>(B, dt, status, infos) : newton<double>(B, dt, status, infos);
}

int make_batch(mbx_cell* const* cells, int n, Batch*& out);

// One step of dt for the given cells (one launch sequence for all of them).
// Cells whose Newton iteration fails are rolled back to u^n and retried as
// two steps of dt/2, recursively up to kMaxHalvings times: the same implicit
// Euler scheme on a finer time grid.  A cell that still fails is restored to
// u^n (transactional).  infos accumulate iterations over the sub-steps.
int step_recover(std::vector<mbx_cell*> cells, double dt, int* status, mbx_step_info* infos, int depth) {
  const int n = (int)cells.size();
  Batch one;
  Batch* B = nullptr;
  if (n == 1) {
    one = single(cells[0]);
    B = &one;
  } else if (int e = make_batch(cells.data(), n, B)) {
    return e;
  }
  std::vector<mbx_step_info> inf(n);
  if (int e = run_step(*B, dt, status, inf.data())) return e;
  for (int i = 0; i < n; ++i) {
    inf[i].substeps = 1;
    if (depth == 0) {
      infos[i] = inf[i];
    } else {
      infos[i].newton_iters += inf[i].newton_iters;
      infos[i].krylov_iters += inf[i].krylov_iters;
    }
  }
  std::vector<int> fail_idx;
  for (int i = 0; i < n; ++i)
    if (status[i] == MBX_ENEWTON || status[i] == MBX_ENAN) fail_idx.push_back(i);
  if (fail_idx.empty() || depth >= kMaxHalvings) return MBX_OK;
  // retry the failed cells as two half steps, from a host copy of u^n (and
  // of the snapshot count: a retry that fails drops its columns again)
  std::vector<mbx_cell*> sub;
  std::vector<std::vector<double>> save(fail_idx.size() * 3);
  std::vector<int> cap_save(fail_idx.size()), capd_save(fail_idx.size());
  for (size_t k = 0; k < fail_idx.size(); ++k) {
    mbx_cell* c = cells[fail_idx[k]];
    sub.push_back(c);
    cap_save[k] = c->cap_count;
    capd_save[k] = c->cap_dropped;
    save[3 * k].resize(c->N);
    save[3 * k + 1].resize(c->N);
    save[3 * k + 2].resize(std::max(c->F_an, 1));
    if (int e = mbx_cell_get_state(c, save[3 * k].data(), save[3 * k + 1].data(), save[3 * k + 2].data(), 0)) return e;
  }
  if (g_verbose()) fprintf(stderr, "[mbx] %zu cell(s) failed at dt %g: retrying as two steps of %g\n", sub.size(), dt, dt / 2);
  const int m = (int)sub.size();
  std::vector<int> sst(m, 0), ok(m, 1);
  std::vector<mbx_step_info> sinf(m);
  for (int half = 0; half < 2; ++half) {
    std::vector<mbx_cell*> run;
    std::vector<int> map;
    for (int k = 0; k < m; ++k)
      if (ok[k]) {
        run.push_back(sub[k]);
        map.push_back(k);
      }
    if (run.empty()) break;
    std::vector<int> rst(run.size(), 0);
    std::vector<mbx_step_info> rinf(run.size());
    if (int e = step_recover(run, dt / 2, rst.data(), rinf.data(), depth + 1)) return e;
    for (size_t j = 0; j < run.size(); ++j) {
      const int k = map[j];
      sinf[k].newton_iters += rinf[j].newton_iters;
      sinf[k].krylov_iters += rinf[j].krylov_iters;
      sinf[k].substeps += rinf[j].substeps;
      sinf[k].res0 = half == 0 ? rinf[j].res0 : sinf[k].res0;
      sinf[k].res_final = rinf[j].res_final;
      sinf[k].du_final = rinf[j].du_final;
      sinf[k].V = rinf[j].V;
      if (rst[j] != MBX_OK) {
        ok[k] = 0;
        sst[k] = rst[j];
      }
    }
  }
  for (int k = 0; k < m; ++k) {
    const int i = fail_idx[k];
    mbx_step_info& o = infos[i];
    o.newton_iters += sinf[k].newton_iters;
    o.krylov_iters += sinf[k].krylov_iters;
    if (ok[k]) {
      status[i] = MBX_OK;
      o.substeps = sinf[k].substeps;
      o.res_final = sinf[k].res_final;
      o.du_final = sinf[k].du_final;
      o.V = sinf[k].V;
    } else {
      status[i] = sst[k];
      mbx_cell* c = sub[k];
      if (int e = mbx_cell_set_state(c, save[3 * k].data(), save[3 * k + 1].data(), save[3 * k + 2].data(), 0))
        return e;
      c->cap_count = cap_save[k];
      c->cap_dropped = capd_save[k];
    }
  }
  return MBX_OK;
}

// ------------------------------------------------------------ launch tuner
// Workgroup size of the single-cell launches of the level-0 smoother and of
// J*v, picked per grid size and precision by timing 256, 128 and 64 threads
// on the new cell's own arrays (one warm-up and three timed launches each;
// another size must be 3% faster to be taken).  The kernels compute the
// same values with any size, so results do not depend on the choice.  Kept
// per process; with MBX_TUNE_FILE the choices are read from and appended to
// that file.  MBX_TUNE=0 keeps 256; MBX_TUNE=64, 128, 256, 512 or 1024 fixes that size.
std::mutex g_tune_mu;
std::map<std::array<int, 4>, std::array<int, 2>> g_tune;
bool g_tune_loaded = false;

bool tune_valid(int bs) { return bs == 64 || bs == 128 || bs == kBlock || bs == 512 || bs == 1024; }

template <typename KT>
int time_shapes(mbx_cell* c, bool smooth, int& best) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double best_ms = 1e30;
  best = kBlock;
  int rc = MBX_OK;
  for (int bs : {kBlock, 512, 1024, 128, 64}) {
    Batch b = single(c);
    BatchLaunch bl = b.bl();
    (smooth ? bl.bs_smooth0 : bl.bs_matvec) = bs;
    for (int r = 0; r < 4; ++r) {
      if (r == 1 && hipEventRecord(e0, c->s) != hipSuccess) rc = MBX_EHIP;
      if (smooth)
        launch_smooth0_probe<KT>(bl, c->s);
      else
        launch_matvec<KT>(bl, VEC_Z, VEC_W, 0, -1, c->s);
    }
    float ms = 0.f;
    if (hipEventRecord(e1, c->s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess || hipGetLastError() != hipSuccess)
      rc = MBX_EHIP;
    if (rc != MBX_OK) break;
    if (best_ms >= 1e30 || ms < 0.97 * best_ms) {
      best = bs;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc == MBX_OK ? MBX_OK : fail(MBX_EHIP, "launch-shape tuning failed");
}

int tune_launch_shape(mbx_cell* c) {
  if (const char* fix = std::getenv("MBX_TUNE")) {
    const int v = std::atoi(fix);
    if (v == 0 || tune_valid(v)) {
      c->bs_smooth0 = c->bs_matvec = v == 0 ? kBlock : v;
      return MBX_OK;
    }
  }
  const std::array<int, 4> key = {c->nx, c->ny, c->nz, c->p.precision};
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const char* file = std::getenv("MBX_TUNE_FILE");
  if (!g_tune_loaded) {
    g_tune_loaded = true;
    if (FILE* fp = file ? std::fopen(file, "r") : nullptr) {
      int nx, ny, nz, pr, a, b;
      while (std::fscanf(fp, "%d %d %d %d %d %d", &nx, &ny, &nz, &pr, &a, &b) == 6)
        if (tune_valid(a) && tune_valid(b)) g_tune[{nx, ny, nz, pr}] = {a, b};
      std::fclose(fp);
    }
  }
  auto it = g_tune.find(key);
  if (it == g_tune.end()) {
    int a = kBlock, b = kBlock;
    if (int e = c->mixed ? time_shapes<float>(c, true, a) : time_shapes<double>(c, true, a)) return e;
    if (int e = c->mixed ? time_shapes<float>(c, false, b) : time_shapes<double>(c, false, b)) return e;
    it = g_tune.emplace(key, std::array<int, 2>{a, b}).first;
    if (FILE* fp = file ? std::fopen(file, "a") : nullptr) {
      std::fprintf(fp, "%d %d %d %d %d %d\n", c->nx, c->ny, c->nz, c->p.precision, a, b);
      std::fclose(fp);
    }
  }
  c->bs_smooth0 = it->second[0];
  c->bs_matvec = it->second[1];
  return MBX_OK;
}

int sync_outputs(mbx_cell* c) {
  Batch b = single(c);
  c->h.active = 1;
  if (int e = b.upload()) return e;
  launch_outputs(b.bl(), c->s);
  return b.gather();
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* mbx_last_error(void) { return g_err.c_str(); }

int mbx_params_default(mbx_params* p) {
  if (!p) return fail(MBX_EINVAL, "null parameter struct");
  std::memset(p, 0, sizeof *p);
  p->newton_tol = 0.0;   // the precision mode's default
  p->res_tol = 1e-6;
  p->krylov_rtol = 1e-6;
  p->newton_max = 30;
  p->krylov_max = 600;
  p->thermo = 1.0;
  p->graphs = 1;
  return MBX_OK;
}

int64_t mbx_cell_footprint(int nx, int ny, int nz, int precision, int n_an_faces, int n_ca_faces) {
  const int64_t N = (int64_t)nx * ny * nz;
  if (N <= 0 || N > (1 << 28)) return -1;
  if (nx > (1 << 21) || ny > (1 << 21) || (int64_t)ny * nz > (1 << 23)) return -1;
  const int nblk = (int)((N + kBlock - 1) / kBlock);
  Layout L = make_layout((int)N, n_an_faces, n_ca_faces, nblk, restart_len(), kt_size(precision),
                         level_dims(nx, ny, nz, kt_size(precision)));
  return (int64_t)L.total;
}

int mbx_cell_create(const uint8_t* labels, int nx, int ny, int nz, const mbx_params* pin, void* stream,
                    mbx_cell** out) {
  if (!labels || !out) return fail(MBX_EINVAL, "null labels or output pointer");
  *out = nullptr;
  if (nx < 1 || ny < 1 || nz < 2) return fail(MBX_EINVAL, "grid must be at least 1 x 1 x 2");
  const int64_t N64 = (int64_t)nx * ny * nz;
  if (N64 > (1 << 28)) return fail(MBX_EINVAL, "grid too large (more than 2^28 voxels)");
  // the kernels' index division (divmod) is exact for divisors up to 2^21 and quotients below 2^24
  if (nx > (1 << 21) || ny > (1 << 21) || (int64_t)ny * nz > (1 << 23))
    return fail(MBX_EINVAL, "grid too elongated (nx and ny at most 2^21, ny*nz at most 2^23)");
  if (int e = check_params(pin)) return e;
  mbx_params p = *pin;
  // scaled-update tolerance: 100x below each mode's state-error target (FP64 1e-8, mixed 1e-6)
  if (p.newton_tol <= 0) p.newton_tol = p.precision == MBX_MIXED ? 1e-8 : 1e-9;
  if (p.res_tol <= 0) p.res_tol = 1e-6;
  if (p.krylov_rtol <= 0) p.krylov_rtol = 1e-6;
  if (p.newton_max <= 0) p.newton_max = 30;
  if (p.krylov_max <= 0) p.krylov_max = 600;
  const int N = (int)N64;
  hipStream_t s = (hipStream_t)stream;

  // ---- phase 1: labels -> masks, face counts, prefix sums (device)
  const int Np = 2 * ((nx + 1) / 2) * ny * nz;   // colour-split slots (padding included)
  size_t scan_bytes = 0, scan_bytes_rb = 0;
  if (exclusive_scan(nullptr, scan_bytes, nullptr, nullptr, N, s) != hipSuccess ||
      exclusive_scan(nullptr, scan_bytes_rb, nullptr, nullptr, Np, s) != hipSuccess)
    return fail(MBX_EHIP, "scan size query failed");
  scan_bytes = std::max(scan_bytes, scan_bytes_rb);
  Layout T;
  const size_t o_lab = T.add(N), o_meta = T.add(4 * (size_t)N), o_ca = T.add(4 * (size_t)N),
               o_cc = T.add(4 * (size_t)N), o_oa = T.add(4 * (size_t)N), o_oc = T.add(4 * (size_t)N),
               o_fl = T.add(64), o_scan = T.add(scan_bytes), o_rbc = T.add(4 * (size_t)Np),
               o_rbo = T.add(4 * (size_t)Np);
  char* tmp = nullptr;
  if (hipMalloc(&tmp, T.total) != hipSuccess) return fail(MBX_ENOMEM, "device allocation of %zu bytes failed", T.total);
  auto cleanup_tmp = [&]() { (void)hipFree(tmp); };
  int* flags = (int*)(tmp + o_fl);
  int hflags[4] = {0, 0, 0, 0};
  int tail[4] = {0, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(tmp + o_lab, labels, N, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(flags, 0, 16, s);
  if (e == hipSuccess) {
    launch_build_meta((const uint8_t*)(tmp + o_lab), nx, ny, nz, (uint32_t*)(tmp + o_meta), (int*)(tmp + o_ca),
                      (int*)(tmp + o_cc), flags, s);
    size_t sb = scan_bytes;
    e = exclusive_scan(tmp + o_scan, sb, (const int*)(tmp + o_ca), (int*)(tmp + o_oa), N, s);
    if (e == hipSuccess) {
      sb = scan_bytes;
      e = exclusive_scan(tmp + o_scan, sb, (const int*)(tmp + o_cc), (int*)(tmp + o_oc), N, s);
    }
  }
  if (e == hipSuccess) e = hipMemcpyAsync(hflags, flags, 16, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&tail[0], tmp + o_ca + 4 * (size_t)(N - 1), 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&tail[1], tmp + o_oa + 4 * (size_t)(N - 1), 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&tail[2], tmp + o_cc + 4 * (size_t)(N - 1), 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&tail[3], tmp + o_oc + 4 * (size_t)(N - 1), 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    cleanup_tmp();
    return fail(MBX_EHIP, "cell setup: %s", hipGetErrorString(e));
  }
  if (hflags[0] & 1) {
    cleanup_tmp();
    return fail(MBX_EINVAL, "labels must be 0 (pore), 1 (anode), 2 (cathode) or 3 (Li foil)");
  }
  if ((hflags[0] & 4) && (hflags[0] & 8)) {
    cleanup_tmp();
    return fail(MBX_ELABEL, "a cell holds cathode (2) or Li foil (3) voxels, not both");
  }
  if (hflags[0] & 2) {
    cleanup_tmp();
    return fail(MBX_ELABEL, "an anode voxel shares a face with a cathode or foil voxel");
  }
  if (hflags[1] == 0 || hflags[2] == 0) {
    cleanup_tmp();
    return fail(MBX_ELABEL, "the z=0 plane needs anode solid and the z=nz-1 plane cathode (or foil) solid");
  }
  const int half = (hflags[0] & 4) ? 1 : 0;
  if (half && !(p.i00_ce > 0.0)) {
    cleanup_tmp();
    return fail(MBX_EINVAL, "a half cell (Li foil voxels) needs i00_ce > 0");
  }
  const int F_an = tail[0] + tail[1], F_ca = tail[2] + tail[3];
  if (F_an + F_ca >= (1 << 24)) {
    cleanup_tmp();
    return fail(MBX_EINVAL, "too many interface faces for the 24-bit face index");
  }
  // arrays read through 32-bit buffer offsets (largest: the FP64 GMRES iterate,
  // 16 bytes per voxel; the colour-split arrays hold at most 8 per slot)
  if (16 * (size_t)N >= (size_t)kNoOff - 4096 || 8 * (size_t)Np >= (size_t)kNoOff - 4096) {
    cleanup_tmp();
    return fail(MBX_EINVAL, "grid too large for 32-bit buffer offsets (at most about 2^27 voxels)");
  }

  // ---- phase 2: the cell's memory
  mbx_cell* c = new mbx_cell();
  c->id = g_next_id++;
  c->p = p;
  c->nx = nx;
  c->ny = ny;
  c->nz = nz;
  c->N = N;
  c->F_an = F_an;
  c->F_ca = F_ca;
  c->n_top = hflags[2];
  for (int i = 0; i < N; ++i) {
    c->n_an_vox += labels[i] == ANODE;
    c->n_ca_vox += labels[i] == CATHODE;
  }
  c->nblk = (N + kBlock - 1) / kBlock;
  c->m = restart_len();
  c->mixed = p.precision == MBX_MIXED;
  c->s = s;
  const size_t kt = kt_size(p.precision);
  c->ld = level_dims(nx, ny, nz, kt_size(p.precision));
  if (c->ld.ncell[c->ld.n - 1] > kCoarseMaxCells) {
    cleanup_tmp();
    delete c;
    return fail(MBX_EINVAL, "grid too elongated for the multigrid hierarchy");
  }
  Layout L = make_layout(N, F_an, F_ca, c->nblk, c->m, kt, c->ld);
  if (hipMalloc(&c->dmem, L.total) != hipSuccess) {
    cleanup_tmp();
    delete c;
    return fail(MBX_ENOMEM, "device allocation of %zu bytes failed", L.total);
  }
  if (std::getenv("MBX_POISON")) {
    // debugging aid: NaN bytes everywhere, so a read before the first write shows up
    if (hipMemsetAsync(c->dmem, 0xff, L.total, s) != hipSuccess) {
      cleanup_tmp();
      (void)hipFree(c->dmem);
      delete c;
      return fail(MBX_EHIP, "poison fill failed");
    }
  }
  char* b = c->dmem;
  CellDev& h = c->h;
  h.nx = nx;
  h.ny = ny;
  h.nz = nz;
  h.N = N;
  h.F_an = F_an;
  h.F_ca = F_ca;
  h.n_top = c->n_top;
  h.nblk = c->nblk;
  h.active = 1;
  h.meta = (const uint32_t*)(b + L.off[0]);
  double** d8[8] = {&h.c, &h.phi, &h.c_try, &h.phi_try, &h.c_old, &h.phi_old, &h.Rc, &h.Rp};
  for (int k = 0; k < 8; ++k) *d8[k] = (double*)(b + L.off[1 + k]);
  h.dc = (double*)(b + L.off[9]);
  h.dp = h.dc + N;
  double** f8[7] = {&h.n, &h.n_try, &h.n_old, &h.Rn, &h.dn, &h.rn_jnn, &h.sq};
  for (int k = 0; k < 7; ++k) *f8[k] = (double*)(b + L.off[10 + k]);
  h.coef_an = b + L.off[17];
  h.coef_ca = b + L.off[18];
  h.wpore = b + L.off[19];
  h.dint = b + L.off[20];
  h.Vb = b + L.off[21];
  h.w = b + L.off[22];
  h.z = b + L.off[23];
  h.b = b + L.off[24];
  h.x = (double*)(b + L.off[25]);
  h.part = (double*)(b + L.off[26]);
  h.red = (double*)(b + L.off[28]);
  h.ictl = (int*)(b + L.off[29]);
  h.gm = (double*)(b + L.off[30]);
  c->faces_an = (int*)(b + L.off[31]);
  c->faces_ca = (int*)(b + L.off[32]);
  c->d_desc = (CellDev*)(b + L.off[33]);
  c->d_blk = (int2*)(b + L.off[34]);
  c->d_gather = (double*)(b + L.off[35]);
  h.b0 = b + L.off[36];
  h.cond_an = b + L.off[37];
  h.cond_ca = b + L.off[38];
  h.cinv[0] = (double*)(b + L.off[39]);
  h.cinv[1] = (double*)(b + L.off[40]);
  h.nlev = c->ld.n;
  h.lfuse = c->ld.lfuse;
  h.lglob = c->ld.lglob;
  h.alpha = g_mg_alpha();
  h.nu = g_sweeps_min();
  h.nu_f = h.nu;
  h.nu_c = g_sweeps_coarse();
  h.lv[0].nx = nx;
  h.lv[0].ny = ny;
  h.lv[0].nz = nz;
  h.lv[0].ncell = N;
  for (int l = 0; l < c->ld.n; ++l) {
    MGLevel& lv = h.lv[l];
    const int lnx = l == 0 ? nx : c->ld.nx[l], lny = l == 0 ? ny : c->ld.ny[l];
    lv.inv_hx = rcp_up((lnx + 1) / 2);
    lv.inv_nx = rcp_up(lnx);
    lv.inv_ny = rcp_up(lny);
  }
  for (int l = 1; l < c->ld.n; ++l) {
    const int o = 41 + 7 * (l - 1);
    MGLevel& lv = h.lv[l];
    lv.nx = c->ld.nx[l];
    lv.ny = c->ld.ny[l];
    lv.nz = c->ld.nz[l];
    lv.ncell = c->ld.ncell[l];
    lv.x = b + L.off[o];
    lv.b = b + L.off[o + 1];
    lv.op[0] = b + L.off[o + 2];
    lv.op[1] = b + L.off[o + 3];
    c->lvl_blk[l] = (int2*)(b + L.off[o + 4]);
    c->lvl_nblk[l] = (lv.ncell + kBlock - 1) / kBlock;
    c->lvlr_blk[l] = (int2*)(b + L.off[o + 5]);
    c->lvlr_nblk[l] = (4 * lv.ncell + kBlock - 1) / kBlock;
    c->lvlh_blk[l] = (int2*)(b + L.off[o + 6]);
    c->lvlh_nblk[l] = (int)((half_cells(c->ld, l) + kBlock - 1) / kBlock);
  }
  c->lvlh_blk[0] = (int2*)(b + L.off[41 + 7 * (c->ld.n - 1)]);
  h.fres = (double*)(b + L.off[42 + 7 * (c->ld.n - 1)]);
  h.Zb = b + L.off[43 + 7 * (c->ld.n - 1)];
  h.rbhx = (nx + 1) / 2;
  h.rbH = h.rbhx * ny * nz;
  h.inv_nx = rcp_up(nx);
  h.inv_ny = rcp_up(ny);
  h.meta_rb = (const uint32_t*)(b + L.off[44 + 7 * (c->ld.n - 1)]);
  h.x_rb = b + L.off[45 + 7 * (c->ld.n - 1)];
  h.c_prev = (double*)(b + L.off[46 + 7 * (c->ld.n - 1)]);
  h.n_prev = (double*)(b + L.off[47 + 7 * (c->ld.n - 1)]);
  h.cond_rb = b + L.off[48 + 7 * (c->ld.n - 1)];
  h.faces_an = c->faces_an;
  h.faces_ca = c->faces_ca;
  c->lvlh_nblk[0] = (int)((half_cells(c->ld, 0) + kBlock - 1) / kBlock);
  h.m = c->m;
  h.lam = 1.0;
  h.rtol = 1e-6;
  h.half = half;
  fill_constants(h, p, nx, ny);
  fill_step_constants(h, 1.0);
  std::vector<int2> tab(c->nblk);
  for (int k = 0; k < c->nblk; ++k) tab[k] = make_int2(0, k);
  int rc = MBX_OK;
  e = hipHostMalloc(&c->h_gather, sizeof(double) * kGather, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc(&c->h_desc_pinned, sizeof(CellDev), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemcpyAsync((void*)h.meta, tmp + o_meta, 4 * (size_t)N, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) {
    launch_finish_meta(N, (uint32_t*)h.meta, (const int*)(tmp + o_oa), (const int*)(tmp + o_oc), c->faces_an,
                       c->faces_ca, s);
    launch_meta_rb(h, (int*)(tmp + o_rbc), s);
    size_t sb = scan_bytes;
    e = exclusive_scan(tmp + o_scan, sb, (const int*)(tmp + o_rbc), (int*)(tmp + o_rbo), Np, s);
    if (e == hipSuccess) launch_meta_rb_base(h, (const int*)(tmp + o_rbo), s);
  }
  // every face joins a voxel of each colour: each colour's lists hold F_an + F_ca entries
  int rbt[3] = {0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(&rbt[0], tmp + o_rbo + 4 * (size_t)h.rbH, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&rbt[1], tmp + o_rbo + 4 * (size_t)(Np - 1), 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&rbt[2], tmp + o_rbc + 4 * (size_t)(Np - 1), 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  const bool lists_ok = rbt[0] == F_an + F_ca && rbt[1] + rbt[2] == 2 * (F_an + F_ca);
  if (e == hipSuccess) e = hipMemsetAsync(h.ictl, 0, 4 * CTL_NSLOT, s);
  if (e == hipSuccess) e = hipMemsetAsync(h.red, 0, 8 * RED_NSLOT, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->d_blk, tab.data(), sizeof(int2) * tab.size(), hipMemcpyHostToDevice, s);
  std::vector<std::vector<int2>> ltabs(3 * c->ld.n);
  for (int l = 0; l < c->ld.n && e == hipSuccess; ++l) {
    for (int pass = 0; pass < 3 && e == hipSuccess; ++pass) {
      if (l == 0 && pass < 2) continue;
      const int nb = pass == 0 ? c->lvl_nblk[l] : pass == 1 ? c->lvlr_nblk[l] : c->lvlh_nblk[l];
      std::vector<int2>& t = ltabs[3 * l + pass];
      t.resize(nb);
      for (int k = 0; k < nb; ++k) t[k] = make_int2(0, k);
      e = hipMemcpyAsync(pass == 0 ? c->lvl_blk[l] : pass == 1 ? c->lvlr_blk[l] : c->lvlh_blk[l], t.data(),
                         sizeof(int2) * t.size(), hipMemcpyHostToDevice, s);
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  cleanup_tmp();
  if (e != hipSuccess) {
    rc = fail(MBX_EHIP, "cell setup: %s", hipGetErrorString(e));
  } else if (!lists_ok) {
    rc = fail(MBX_EHIP, "colour-split face lists hold %d + %d entries for %d faces", rbt[0],
              rbt[1] + rbt[2] - rbt[0], F_an + F_ca);
  } else {
    Batch bt = single(c);
    rc = bt.upload();
    if (rc == MBX_OK) {
      launch_init_state(bt.bl(), s);
      rc = sync_outputs(c);
    }
    if (rc == MBX_OK) rc = tune_launch_shape(c);
  }
  if (rc != MBX_OK) {
    mbx_cell_destroy(c);
    return rc;
  }
  *out = c;
  return MBX_OK;
}

void mbx_cell_destroy(mbx_cell* c) {
  if (!c) return;
  if (c->s) (void)hipStreamSynchronize(c->s);
  else (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> lk(g_batch_mu);
  for (size_t k = 0; k < g_batch_cache.ids.size(); ++k)
    if (g_batch_cache.ids[k] == c->id) {
      g_batch_cache.b.release();
      g_batch_cache.graphs.clear();
      g_batch_cache.ids.clear();
      break;
    }
  c->graphs.release();
  (void)hipFree(c->dmem);
  (void)hipHostFree(c->h_gather);
  (void)hipHostFree(c->h_desc_pinned);
  delete c;
}

int mbx_cell_step(mbx_cell* c, double dt, mbx_step_info* info) {
  if (!c) return fail(MBX_EINVAL, "null cell");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(MBX_EINVAL, "dt must be finite and > 0");
  int st = 0;
  mbx_step_info tmp{};
  const auto t0 = std::chrono::steady_clock::now();
  if (int e = step_recover({c}, dt, &st, info ? info : &tmp, 0)) return e;
  if (info) info->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st == MBX_ENEWTON) return fail(MBX_ENEWTON, "Newton did not converge; state left at u^n");
  if (st == MBX_ENAN) return fail(MBX_ENAN, "non-finite residual; state left at u^n");
  return st;
}

int mbx_batch_step(mbx_cell* const* cells, int n, double dt, int* status_out, mbx_step_info* infos) {
  if (!cells || n < 1 || !status_out) return fail(MBX_EINVAL, "null cells/status or n < 1");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(MBX_EINVAL, "dt must be finite and > 0");
  for (int i = 0; i < n; ++i) {
    if (!cells[i]) return fail(MBX_EINVAL, "null cell %d", i);
    if (cells[i]->mixed != cells[0]->mixed) return fail(MBX_EINVAL, "cells of one batch must share a precision mode");
    if (cells[i]->s != cells[0]->s) return fail(MBX_EINVAL, "cells of one batch must share a stream");
    for (int j = 0; j < i; ++j)
      if (cells[j] == cells[i]) return fail(MBX_EINVAL, "cell %d appears twice", i);
  }
  std::lock_guard<std::mutex> lk(g_batch_mu);
  std::vector<mbx_step_info> tmp(infos ? 0 : n);
  return step_recover(std::vector<mbx_cell*>(cells, cells + n), dt, status_out, infos ? infos : tmp.data(), 0);
}

int mbx_cell_capture(mbx_cell* c, double* c_snap, double* phi_snap, int64_t ld, int capacity) {
  if (!c) return fail(MBX_EINVAL, "null cell");
  if (capacity < 0) return fail(MBX_EINVAL, "capacity must be >= 0");
  if (capacity == 0 || (!c_snap && !phi_snap)) {
    c->cap_c = c->cap_phi = nullptr;
    c->cap_capacity = c->cap_count = c->cap_dropped = 0;
    return MBX_OK;
  }
  if (ld < c->N) return fail(MBX_EINVAL, "ld must be >= the number of voxels");
  c->cap_c = c_snap;
  c->cap_phi = phi_snap;
  c->cap_ld = ld;
  c->cap_capacity = capacity;
  c->cap_count = c->cap_dropped = 0;
  return capture_column(c, c->s);
}

int mbx_cell_captured(const mbx_cell* c, int* count, int* dropped) {
  if (!c) return fail(MBX_EINVAL, "null cell");
  if (count) *count = c->cap_count;
  if (dropped) *dropped = c->cap_dropped;
  return MBX_OK;
}

int mbx_cell_set_current(mbx_cell* c, double I_app) {
  if (!c) return fail(MBX_EINVAL, "null cell");
  if (!std::isfinite(I_app)) return fail(MBX_EINVAL, "I_app must be finite");
  c->p.I_app = I_app;
  fill_constants(c->h, c->p, c->nx, c->ny);
  return MBX_OK;
}

int mbx_cell_counts(const mbx_cell* c, int64_t* n_vox, int64_t* n_an, int64_t* n_ca, int64_t* n_top) {
  if (!c) return fail(MBX_EINVAL, "null cell");
  if (n_vox) *n_vox = c->N;
  if (n_an) *n_an = c->F_an;
  if (n_ca) *n_ca = c->F_ca;
  if (n_top) *n_top = c->n_top;
  return MBX_OK;
}

int mbx_cell_get_state(const mbx_cell* c, double* cf, double* phi, double* n_pl, int device_ptrs) {
  if (!c) return fail(MBX_EINVAL, "null cell");
  const hipMemcpyKind k = device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (cf) HIPCHK(hipMemcpyAsync(cf, c->h.c, 8 * (size_t)c->N, k, c->s));
  if (phi) HIPCHK(hipMemcpyAsync(phi, c->h.phi, 8 * (size_t)c->N, k, c->s));
  if (n_pl && c->F_an) HIPCHK(hipMemcpyAsync(n_pl, c->h.n, 8 * (size_t)c->F_an, k, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  return MBX_OK;
}

int mbx_cell_set_state(mbx_cell* c, const double* cf, const double* phi, const double* n_pl, int device_ptrs) {
  if (!c || !cf || !phi || (!n_pl && c->F_an)) return fail(MBX_EINVAL, "null argument");
  const hipMemcpyKind k = device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIPCHK(hipMemcpyAsync(c->h.c, cf, 8 * (size_t)c->N, k, c->s));
  HIPCHK(hipMemcpyAsync(c->h.phi, phi, 8 * (size_t)c->N, k, c->s));
  if (c->F_an) HIPCHK(hipMemcpyAsync(c->h.n, n_pl, 8 * (size_t)c->F_an, k, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  return MBX_OK;
}

int mbx_cell_voltage(const mbx_cell* cc, double* V) {
  if (!cc || !V) return fail(MBX_EINVAL, "null argument");
  mbx_cell* c = const_cast<mbx_cell*>(cc);
  if (int e = sync_outputs(c)) return e;
  *V = c->h_gather[RED_VSUM] / c->n_top;
  return MBX_OK;
}

int mbx_cell_inventory(const mbx_cell* cc, double out[4]) {
  if (!cc || !out) return fail(MBX_EINVAL, "null argument");
  mbx_cell* c = const_cast<mbx_cell*>(cc);
  if (int e = sync_outputs(c)) return e;
  for (int k = 0; k < 4; ++k) out[k] = c->h_gather[RED_INV0 + k];
  return MBX_OK;
}

int mbx_cell_launch_shape(const mbx_cell* c, int* smooth0_threads, int* matvec_threads) {
  if (!c) return fail(MBX_EINVAL, "null cell");
  if (smooth0_threads) *smooth0_threads = c->bs_smooth0;
  if (matvec_threads) *matvec_threads = c->bs_matvec;
  return MBX_OK;
}

int mbx_cell_mean_solid(const mbx_cell* cc, double out[2]) {
  if (!cc || !out) return fail(MBX_EINVAL, "null argument");
  mbx_cell* c = const_cast<mbx_cell*>(cc);
  if (int e = sync_outputs(c)) return e;
  out[0] = c->h_gather[RED_INV0 + 1] / (c->h.Vol * (double)c->n_an_vox);
  out[1] = c->h_gather[RED_INV0 + 2] / (c->h.Vol * (double)c->n_ca_vox);
  return MBX_OK;
}

int mbx_cell_run(mbx_cell* c, double dt, int max_steps, double* V_out, int* steps_out, int* cutoff_out,
                 int* retried) {
  if (!c || !steps_out) return fail(MBX_EINVAL, "null cell or steps_out");
  if (max_steps < 0) return fail(MBX_EINVAL, "max_steps must be >= 0");
  *steps_out = 0;
  if (cutoff_out) *cutoff_out = 0;
  if (retried) *retried = 0;
  for (int k = 0; k < max_steps; ++k) {
    mbx_step_info info{};
    if (int e = mbx_cell_step(c, dt, &info)) return e;
    *steps_out = k + 1;
    if (V_out) V_out[k] = info.V;
    if (retried && info.substeps > 1) ++*retried;
    if (cutoff_reached(c->p, info.V)) {
      if (cutoff_out) *cutoff_out = 1;
      break;
    }
  }
  return MBX_OK;
}

// Adaptive implicit Euler (reading R-5 of the time-step control of Sec.
// 2.4): step sizes change by factors of 2; a step whose Newton iteration
// fails or whose error estimate exceeds tol is rolled back and redone with
// half the step; an accepted step whose estimate is at most tol/4 doubles the
// next one.  The estimate is half the distance of the step from the linear
// extrapolation of the two previous accepted states, the explicit Euler step
// on an implicit Euler trajectory (the first step has none).
int mbx_cell_run_adaptive(mbx_cell* c, double t_end, double dt0, double dt_min, double dt_max, double tol,
                          int max_steps, double* t_out, double* V_out, int* steps_out, int* rejected_out,
                          int* cutoff_out) {
  if (!c || !steps_out) return fail(MBX_EINVAL, "null cell or steps_out");
  if (!(std::isfinite(t_end) && t_end >= 0.0)) return fail(MBX_EINVAL, "t_end must be finite and >= 0");
  if (!(std::isfinite(dt0) && dt0 > 0.0 && std::isfinite(dt_min) && dt_min > 0.0 && std::isfinite(dt_max) &&
        dt_max >= dt_min))
    return fail(MBX_EINVAL, "need dt0 > 0 and 0 < dt_min <= dt_max");
  if (!(std::isfinite(tol) && tol > 0.0)) return fail(MBX_EINVAL, "tol must be finite and > 0");
  if (max_steps < 0) return fail(MBX_EINVAL, "max_steps must be >= 0");
  *steps_out = 0;
  if (rejected_out) *rejected_out = 0;
  if (cutoff_out) *cutoff_out = 0;
  double t = 0.0, dt = dt0, dt_prev = 0.0;
  int steps = 0;
  Batch one = single(c);
  while (t < t_end && steps < max_steps) {
    const double h = std::min(dt, t_end - t);
    const int cap = c->cap_count, capd = c->cap_dropped;
    int st = 0;
    mbx_step_info info{};   // iteration counts only: a step without retry leaves V unset
    // one try without the internal half-step retry: rejection is this loop's
    if (int e = step_recover({c}, h, &st, &info, kMaxHalvings)) return e;
    double est = -1.0;   // < 0: no estimate (first step)
    if (st == MBX_OK && steps > 0) {
      if (int e = one.upload()) return e;
      launch_lte(one.bl(), h / dt_prev, c->s);
      if (int e = one.gather()) return e;
      est = 0.5 * one.red(0, RED_LTE);   // implicit minus explicit Euler: twice the local error
      if (!std::isfinite(est)) est = INFINITY;
    }
    if (st != MBX_OK || est > tol) {
      if (st == MBX_OK) {
        // converged but too inaccurate: back to u^n, snapshot column dropped
        c->h.active = 1;
        if (int e = one.upload()) return e;
        launch_copy_state(one.bl(), 3, c->s);
        launch_outputs(one.bl(), c->s);
        if (int e = one.gather()) return e;
        c->cap_count = cap;
        c->cap_dropped = capd;
      }
      if (rejected_out) ++*rejected_out;
      dt = h / 2.0;
      if (dt < dt_min) return fail(MBX_ENEWTON, "adaptive step below dt_min at t = %g; state left at t", t);
      continue;
    }
    // accepted: u^n becomes the history of the next estimate
    c->h.active = 1;
    if (int e = one.upload()) return e;
    launch_copy_state(one.bl(), 5, c->s);
    t = t + h < t_end ? t + h : t_end;
    double V = 0.0;
    if (int e = mbx_cell_voltage(c, &V)) return e;
    if (t_out) t_out[steps] = t;
    if (V_out) V_out[steps] = V;
    ++steps;
    *steps_out = steps;
    dt_prev = h;
    dt = (est >= 0.0 && est <= tol / 4.0) ? std::min(2.0 * h, dt_max) : h;
    if (cutoff_reached(c->p, V)) {
      if (cutoff_out) *cutoff_out = 1;
      break;
    }
  }
  HIPCHK(hipStreamSynchronize(c->s));
  return MBX_OK;
}

static int load_eval_state(mbx_cell* c, const double* cu, const double* pu, const double* nu, const double* cold,
                           const double* nold, double dt) {
  if (!cu || !pu || !cold || (c->F_an && (!nu || !nold))) return fail(MBX_EINVAL, "null argument");
  if (!(std::isfinite(dt) && dt > 0.0)) return fail(MBX_EINVAL, "dt must be finite and > 0");
  const size_t N8 = 8 * (size_t)c->N, F8 = 8 * (size_t)c->F_an;
  HIPCHK(hipMemcpyAsync(c->h.c_try, cu, N8, hipMemcpyHostToDevice, c->s));
  HIPCHK(hipMemcpyAsync(c->h.phi_try, pu, N8, hipMemcpyHostToDevice, c->s));
  HIPCHK(hipMemcpyAsync(c->h.c_old, cold, N8, hipMemcpyHostToDevice, c->s));
  if (c->F_an) {
    HIPCHK(hipMemcpyAsync(c->h.n_try, nu, F8, hipMemcpyHostToDevice, c->s));
    HIPCHK(hipMemcpyAsync(c->h.n_old, nold, F8, hipMemcpyHostToDevice, c->s));
  }
  fill_step_constants(c->h, dt);
  c->h.active = 1;
  c->h.elim_n = 0;   // ... at the caller's plated amounts
  Batch b = single(c);
  return b.upload();
}

int mbx_cell_residual(mbx_cell* c, const double* cu, const double* pu, const double* nu, const double* cold,
                      const double* nold, double dt, double* Rc, double* Rphi, double* Rn) {
  if (!c || !Rc || !Rphi || (c->F_an && !Rn)) return fail(MBX_EINVAL, "null argument");
  if (int e = load_eval_state(c, cu, pu, nu, cold, nold, dt)) return e;
  Batch b = single(c);
  if (c->mixed) launch_residual<float>(b.bl(), false, c->s);
  else launch_residual<double>(b.bl(), false, c->s);
  HIPCHK(hipMemcpyAsync(Rc, c->h.Rc, 8 * (size_t)c->N, hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipMemcpyAsync(Rphi, c->h.Rp, 8 * (size_t)c->N, hipMemcpyDeviceToHost, c->s));
  if (c->F_an) HIPCHK(hipMemcpyAsync(Rn, c->h.Rn, 8 * (size_t)c->F_an, hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  return MBX_OK;
}

int mbx_cell_jvp(mbx_cell* c, const double* cu, const double* pu, const double* nu, const double* cold,
                 const double* nold, double dt, const double* v, double* y) {
  if (!c || !v || !y) return fail(MBX_EINVAL, "null argument");
  if (int e = load_eval_state(c, cu, pu, nu, cold, nold, dt)) return e;
  Batch b = single(c);
  const size_t N16 = 16 * (size_t)c->N;
  HIPCHK(hipMemsetAsync(c->h.ictl, 0, 4 * CTL_NSLOT, c->s));
  if (c->mixed) launch_residual<float>(b.bl(), true, c->s);
  else launch_residual<double>(b.bl(), true, c->s);
  HIPCHK(hipMemcpyAsync(c->h.dc, v, N16, hipMemcpyHostToDevice, c->s));
  if (c->mixed) {
    launch_convert<float>(b.bl(), VEC_Z, 0, c->s);
    launch_matvec<float>(b.bl(), VEC_Z, VEC_W, 0, -1, c->s);
    launch_convert<float>(b.bl(), VEC_W, 1, c->s);
  } else {
    launch_convert<double>(b.bl(), VEC_Z, 0, c->s);
    launch_matvec<double>(b.bl(), VEC_Z, VEC_W, 0, -1, c->s);
    launch_convert<double>(b.bl(), VEC_W, 1, c->s);
  }
  HIPCHK(hipMemcpyAsync(y, c->h.dc, N16, hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  return MBX_OK;
}

int mbx_cell_precond(mbx_cell* c, const double* cu, const double* pu, const double* nu, const double* cold,
                     const double* nold, double dt, const double* v, double* z) {
  if (!c || !v || !z) return fail(MBX_EINVAL, "null argument");
  if (int e = load_eval_state(c, cu, pu, nu, cold, nold, dt)) return e;
  Batch b = single(c);
  const size_t N16 = 16 * (size_t)c->N;
  if (c->mixed) launch_residual<float>(b.bl(), true, c->s);
  else launch_residual<double>(b.bl(), true, c->s);
  if (c->mixed) launch_mg_setup<float>(b.bl(), c->s);
  else launch_mg_setup<double>(b.bl(), c->s);
  HIPCHK(hipMemcpyAsync(c->h.dc, v, N16, hipMemcpyHostToDevice, c->s));
  if (c->mixed) {
    launch_convert<float>(b.bl(), VEC_W, 0, c->s);
    launch_precond<float>(b.bl(), VEC_W, -2, c->s);
    launch_convert<float>(b.bl(), VEC_Z, 1, c->s);
  } else {
    launch_convert<double>(b.bl(), VEC_W, 0, c->s);
    launch_precond<double>(b.bl(), VEC_W, -2, c->s);
    launch_convert<double>(b.bl(), VEC_Z, 1, c->s);
  }
  HIPCHK(hipMemcpyAsync(z, c->h.dc, N16, hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  return MBX_OK;
}

int mbx_cell_solve(mbx_cell* c, const double* cu, const double* pu, const double* nu, const double* cold,
                   const double* nold, double dt, const double* rhs, double rtol, double* x, int* iters) {
  if (!c || !rhs || !x) return fail(MBX_EINVAL, "null argument");
  if (!(rtol > 0.0 && rtol < 1.0)) return fail(MBX_EINVAL, "rtol must lie in (0, 1)");
  if (int e = load_eval_state(c, cu, pu, nu, cold, nold, dt)) return e;
  Batch b = single(c);
  const size_t N16 = 16 * (size_t)c->N;
  c->h.rtol = rtol;
  if (int e = b.upload()) return e;
  int its = 0;
  HIPCHK(hipMemcpyAsync(c->h.dc, rhs, N16, hipMemcpyHostToDevice, c->s));
  if (c->mixed) {
    launch_residual<float>(b.bl(), true, c->s);
    launch_mg_setup<float>(b.bl(), c->s);
    launch_convert<float>(b.bl(), VEC_B, 0, c->s);
    launch_convert<float>(b.bl(), VEC_W, 0, c->s);
    launch_zero_x<float>(b.bl(), c->s);
    launch_norm_w<float>(b.bl(), c->s);
    if (int e = gmres<float>(b, c->p.krylov_max, &its)) return e;
    launch_convert<float>(b.bl(), VEC_X, 1, c->s);
  } else {
    launch_residual<double>(b.bl(), true, c->s);
    launch_mg_setup<double>(b.bl(), c->s);
    launch_convert<double>(b.bl(), VEC_B, 0, c->s);
    launch_convert<double>(b.bl(), VEC_W, 0, c->s);
    launch_zero_x<double>(b.bl(), c->s);
    launch_norm_w<double>(b.bl(), c->s);
    if (int e = gmres<double>(b, c->p.krylov_max, &its)) return e;
    launch_convert<double>(b.bl(), VEC_X, 1, c->s);
  }
  HIPCHK(hipMemcpyAsync(x, c->h.dc, N16, hipMemcpyDeviceToHost, c->s));
  HIPCHK(hipStreamSynchronize(c->s));
  if (int e = b.gather()) return e;
  if (iters) *iters = b.ctl(0, CTL_ITERS);
  return MBX_OK;
}

}  // extern "C"
