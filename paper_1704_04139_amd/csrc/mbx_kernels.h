// mbx_kernels.h — host-side launchers of the kernels in kernels.hip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mbx_dev.h"

namespace mbx {

// Krylov vector selectors (>= 0: basis vector j).
enum { VEC_Z = -1, VEC_W = -2, VEC_B = -3, VEC_X = -4 };

// One launch over a batch: device descriptor array and block table
// (blk[b] = {cell index, block index within the cell}).
struct BatchLaunch {
  CellDev* cells;
  const int2* blk;
  int nblk;
  int ncell;
  int faces_single;                      // interface faces of the cell of a single-cell launch (blk == nullptr)
  int n_single;                          // voxels of that cell
  int bs_smooth0, bs_matvec;             // threads per workgroup of the level-0 smoother and of J*v in a
                                         // single-cell launch (64, 128 or 256; table launches use kBlock)
  int maxlev;                            // max multigrid levels over the batch
  int maxfuse;                           // max first LDS-staged fused level over the batch
  int maxglob;                           // max first fused level (device-memory levels included) over the batch
  size_t fused_lds;                      // LDS elements (KT) of the fused coarse cycle, max over the batch
  int max_nu;                            // most smoothing sweeps any cell of the batch asks for
  int max_nu_c;                          // ... on launched levels >= 2
  const int2* lvl_blk[kMaxLevels];       // block tables over each level's cells (index >= 1)
  int lvl_nblk[kMaxLevels];
  const int2* lvlr_blk[kMaxLevels];      // block tables with 4 lanes per level cell, one per red child (index >= 1)
  int lvlr_nblk[kMaxLevels];
  const int2* lvlh_blk[kMaxLevels];      // block tables over one colour of a red-black sweep (index >= 0)
  int lvlh_nblk[kMaxLevels];
  // algorithmic bytes per launch (summed over the batch), for timing records
  double bytes_residual[2];              // [0] residual only, [1] with linearisation
  double bytes_matvec;
  double bytes_smooth0;                  // one level-0 red-black half sweep
};

void launch_build_meta(const uint8_t* lab, int nx, int ny, int nz, uint32_t* meta, int* cnt_an, int* cnt_ca,
                       int* flags, hipStream_t s);
void launch_finish_meta(int N, uint32_t* meta, const int* off_an, const int* off_ca, int* faces_an, int* faces_ca,
                        hipStream_t s);
void launch_init_state(const BatchLaunch& b, hipStream_t s);
// colour-split copy of the finished meta words (cd: host copy of the descriptor, device pointers);
// cnt (2 rbH ints) receives each slot's interface-face count
void launch_meta_rb(const CellDev& cd, int* cnt, hipStream_t s);
// face-base fields of the colour-split meta words from off = exclusive scan of cnt
void launch_meta_rb_base(const CellDev& cd, const int* off, hipStream_t s);
// rocPRIM exclusive prefix sum of n ints (temp == nullptr: query temp_bytes)
hipError_t exclusive_scan(void* temp, size_t& temp_bytes, const int* in, int* out, int n, hipStream_t s);

template <typename KT> void launch_residual(const BatchLaunch& b, bool lin, hipStream_t s);
template <typename KT> void launch_rhs(const BatchLaunch& b, hipStream_t s);
// y_dst = J v_src; keep >= 0 stores v_src as preconditioned basis vector `keep` (flexible GMRES)
template <typename KT> void launch_matvec(const BatchLaunch& b, int src, int dst, int need, int keep, hipStream_t s);
template <typename KT> void launch_convert(const BatchLaunch& b, int sel, int dir, hipStream_t s);
template <typename KT> void launch_zero_x(const BatchLaunch& b, hipStream_t s);
template <typename KT> void launch_norm_w(const BatchLaunch& b, hipStream_t s);
template <typename KT> void launch_multidot(const BatchLaunch& b, int k, int tgt, hipStream_t s);
template <typename KT> void launch_orth(const BatchLaunch& b, int k, int src, hipStream_t s);
// first Gram-Schmidt pass (coefficients H(:,k)) fused with the dot products of
// the second pass (into tmp)
template <typename KT> void launch_orth_dots(const BatchLaunch& b, int k, hipStream_t s);
template <typename KT> void launch_scale_next(const BatchLaunch& b, int k, hipStream_t s);
void launch_backsolve(const BatchLaunch& b, hipStream_t s);
// x += Z y for the cells whose cycle just closed
template <typename KT> void launch_update_x(const BatchLaunch& b, hipStream_t s);
template <typename KT> void launch_true_residual(const BatchLaunch& b, hipStream_t s);
template <typename KT> void launch_gm_start(const BatchLaunch& b, int first, hipStream_t s);
// refine: a cell whose cycle converged restarts if its true residual misses the tolerance
void launch_gm_flags(const BatchLaunch& b, int first, int refine, hipStream_t s);
void launch_gather_ctl(const BatchLaunch& b, double* out, hipStream_t s);
template <typename KT> void launch_direction(const BatchLaunch& b, hipStream_t s);
void launch_trial(const BatchLaunch& b, hipStream_t s);
void launch_copy_state(const BatchLaunch& b, int mode, hipStream_t s);
void launch_outputs(const BatchLaunch& b, hipStream_t s);
// adaptive stepping: scaled max |u - u_pred| of the differential unknowns into red[RED_LTE]
void launch_lte(const BatchLaunch& b, double w, hipStream_t s);

// multigrid preconditioner (mg.hip)
// one level-0 red-black half sweep (operator op, colour 0, no GMRES gate) on
// the cell's current arrays: the workgroup-size tuner's probe
template <typename KT> void launch_smooth0_probe(const BatchLaunch& b, hipStream_t s);
template <typename KT> void launch_mg_setup(const BatchLaunch& b, hipStream_t s);
// z = M^-1 v_src; need: GMRES state gate (>= 0 equal, -1 cycle end, -2 always)
template <typename KT> void launch_precond(const BatchLaunch& b, int src, int need, hipStream_t s);

// POD by the method of snapshots (pod.hip).  Snapshots S: n x m column-major.
int gram_tile();               // edge of the Gram tiles (pairs index tiles of this size)
int gram_all_cols();           // sets at most this wide: one workgroup per row slice computes every pair
int gram_rows_step();          // rows per split are a multiple of this
int modes_cols_per_thread();   // kpad is a multiple of this
// partial Gram tiles part[(y npairs + p) tile^2] of W S[:, ti] ^T S[:, tj] over row slice y
void launch_gram(const double* S, int64_t n, int m, int64_t lds, const double* w, int64_t rows_per_split, int nsplit,
                 const int2* pairs, int npairs, double* part, hipStream_t s);
// K (m x m, symmetric) = sum of the slices, in slice order
void launch_gram_reduce(const double* part, int nsplit, const int2* pairs, int npairs, int m, double* K, hipStream_t s);
// U[:, q] = S C[:, q] for q < k (C row-major m x kpad)
void launch_modes(const double* S, int64_t n, int m, int64_t lds, const double* C, int kpad, int k, double* U,
                  int64_t ldu, hipStream_t s);

// Sets the calling thread's mbx_last_error message and returns code.
int report_error(int code, const char* msg);

}  // namespace mbx
