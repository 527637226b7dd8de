/* mbx.h — C ABI of the MI355X full-order implicit cell-step library.
 *
 * The library advances the voxel-resolved full-cell lithium-ion model of
 * arXiv 1704.04139 (MULTIBAT), Sec. 2.2-2.4, one implicit Euler step at a
 * time on one AMD Instinct MI355X (gfx950):
 *   - unknowns (Sec. 2.4, eq. 2.13): one concentration c and one potential
 *     phi per voxel (electrolyte c_e, phi_e in pore voxels; solid c_s, Phi_s in
 *     anode/cathode voxels) and one plated-lithium amount n_f (mol/m^2) per
 *     anode/pore face;
 *   - fluxes: solid diffusion and conduction (eqs. 2.1-2.2), electrolyte
 *     diffusion, migration and the dmu/dc term (eqs. 2.3-2.4), Butler-Volmer
 *     intercalation on every solid/pore face (eq. 2.5 with the interface
 *     conditions of eq. 2.4), plating/stripping with the f_pre regularisation
 *     on every anode/pore face (eqs. 2.8-2.12, Sec. 2.3);
 *   - collectors: the z = 0 plane holds the anode at phi = 0 (across half a
 *     voxel); the z = L plane feeds the applied current uniformly into the
 *     cathode solid faces it touches.  Lateral sides carry no flux.
 *   - solve: Newton's method on the FP64 residual with a preconditioned
 *     Krylov method (GMRES) for the corrections; FP64 throughout, or FP32
 *     Krylov/preconditioner with FP64 residual and refinement (MBX_MIXED).
 *
 * Conventions
 *   - SI units everywhere (m, s, mol, A, V, K).
 *   - Labels: uint8, 0 = pore/electrolyte, 1 = anode active material,
 *     2 = cathode active material, 3 = Li-metal foil: the counter electrode
 *     of a half cell (Sec. 2.2), which takes the cathode's place (a cell
 *     holds 2 or 3, not both).  Voxel (i, j, k) has flat index
 *     i + nx*(j + ny*k); k = 0 touches the anode collector, k = nz-1 the
 *     cathode (foil) collector.
 *   - Interface faces are numbered per phase in canonical order: by solid
 *     voxel flat index, then by direction 0:-x 1:+x 2:-y 3:+y 4:-z 5:+z as
 *     seen from the solid voxel.  Plated amounts n_pl[] follow the anode
 *     face order.
 *   - Every function returns 0 on success or a negative MBX_E* code; no
 *     exception crosses the ABI.  mbx_last_error() returns a thread-local
 *     message for the last failure on the calling thread.
 *   - A cell is not thread-safe: calls on one cell must not overlap.
 *   - Pointers marked "device" are HIP device (or managed) addresses; all
 *     others are host addresses.  The library never takes ownership of
 *     caller memory; it copies what it needs.
 */
#ifndef MBX_H
#define MBX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MBX_OK = 0,
  MBX_EINVAL = -1,   /* bad argument (null pointer, size, parameter out of range) */
  MBX_ELABEL = -2,   /* labels invalid: anode touches cathode (or foil), cathode and foil labels mixed, or a
                        collector plane holds no solid of its electrode */
  MBX_ENEWTON = -3,  /* Newton did not converge within newton_max iterations */
  MBX_ENAN = -4,     /* non-finite value in the state or residual */
  MBX_ENOMEM = -5,   /* device allocation failed */
  MBX_EBUDGET = -6,  /* request does not fit the server's memory budget */
  MBX_EHIP = -7,     /* HIP runtime error */
  MBX_ESTATE = -8    /* call not valid in the object's current state */
};

enum { MBX_FP64 = 0, MBX_MIXED = 1 };

/* Physical and numerical parameters (SI units).  Physical meaning follows
 * Sec. 2.2-2.3: intercalation i = 2 i00 sqrt(c_s c_e) sinh(F eta/(2RT)),
 * eta = Phi_s - U(c_s/c_max) - phi_e, U(x) = U0 + U1 ln((1-x)/x);
 * plating i_pl = i00_pl sqrt(c_e) (f_pre(n) e^{F eta_pl/2RT} - e^{-F eta_pl/2RT}),
 * eta_pl = Phi_s - phi_e, f_pre(n) = n^4/(n_c^4 + n^4). */
typedef struct {
  double T;              /* temperature, K (isothermal, Sec. 2.2) */
  double I_app;          /* applied current, A; > 0 charges (anode lithiates) */
  double h;              /* voxel edge, m */
  double c0;             /* initial electrolyte concentration, mol/m^3 */
  double x0, y0;         /* initial anode / cathode stoichiometry c_s/c_max */
  double De, kappa, tplus, thermo;   /* electrolyte diffusivity m^2/s, conductivity S/m,
                                        transference number, thermodynamic factor */
  double Ds[2];          /* solid diffusivity, [0] anode, [1] cathode, m^2/s */
  double sigma[2];       /* solid conductivity, S/m */
  double cmax[2];        /* maximum solid concentration, mol/m^3 */
  double i00[2];         /* intercalation rate constant, A m/mol */
  double U0[2], U1[2];   /* open-circuit potential coefficients, V */
  double i00_pl;         /* plating rate constant, A m^-1/2 mol^-1/2 */
  double n_c;            /* f_pre constant, mol/m^2 */
  int plating;           /* 0: no plating reaction, 1: plating/stripping on */
  int precision;         /* MBX_FP64 or MBX_MIXED */
  double newton_tol;     /* scaled update tolerance (if <= 0: 1e-9 for MBX_FP64, 1e-8 for MBX_MIXED) */
  double res_tol;        /* scaled residual tolerance (default 1e-6 if <= 0) */
  double krylov_rtol;    /* floor of the GMRES relative tolerance (forcing term) (default 1e-6 if <= 0) */
  int newton_max;        /* Newton iteration cap (default 30 if <= 0) */
  int krylov_max;        /* GMRES iteration cap per Newton iteration (default 600 if <= 0); at the cap the
                            correction is taken as it stands (inexact Newton) */
  double V_cut;          /* cell-voltage cutoff, V (0: none).  A run (mbx_cell_run, a served request) stops
                            after the first step whose voltage reaches it: V >= V_cut while charging
                            (I_app > 0), V <= V_cut while discharging; no interpolation within the step */
  int graphs;            /* 1 (mbx_params_default): the GMRES iterations between two host checks run as a
                            captured HIP graph, replayed with one launch; 0: direct kernel launches.  Same
                            kernels and results either way.  A batch uses graphs if all its cells do. */
  double i00_ce;         /* half cell (labels 3, Sec. 2.2): rate constant of the Li-foil counter electrode,
                            A/m^2, i = 2 i00_ce sinh(F (Phi_foil - phi_e) / 2RT); required > 0 when the
                            labels hold foil voxels, unused otherwise.  The foil takes the cathode's
                            conductivity sigma[1]; its concentration unknown carries no equation (it keeps
                            y0 cmax[1]); the cathode's Ds[1], i00[1], U0[1], U1[1] are unused */
} mbx_params;

typedef struct {
  int newton_iters;      /* Newton iterations taken */
  int krylov_iters;      /* total GMRES iterations in the step */
  double res0;           /* scaled residual max-norm at the start of the step */
  double res_final;      /* scaled residual max-norm at acceptance */
  double du_final;       /* scaled max-norm of the last Newton update */
  double V;              /* cell voltage after the step, V */
  double wall_s;         /* wall time of the step, s */
  int substeps;          /* implicit Euler steps the step took: 1, or 2 after a retried failure */
} mbx_step_info;

typedef struct mbx_cell mbx_cell;

/* Fill *p with the library's defaults for the numerical knobs (newton_tol = 0:
 * the precision mode's default) and zeros for the physical fields.  Returns MBX_EINVAL on a null pointer. */
int mbx_params_default(mbx_params *p);

/* Create a cell from voxel labels (Sec. 2.4: the voxel image defines the
 * finite-volume mesh; Sec. 2.6: image plus parameters define a simulation).
 *   labels : host, nx*ny*nz bytes, layout above; copied, caller keeps ownership
 *   p      : host; copied
 *   stream : hipStream_t to run on (NULL = the default stream)
 *   out    : receives the handle; the cell owns its device memory
 * The state is set to the zero-current equilibrium: c = c0 in pores,
 * x0*c_max / y0*c_max in the solids, phi_anode = 0, phi_e = -U_an(x0),
 * phi_cathode = U_ca(y0) - U_an(x0) (a half cell's foil: -U_an(x0)),
 * n_f = n_c (f/(1-f))^(1/4) with f = exp(-F U_an(x0)/RT), which makes every
 * interface current vanish.
 * Size limits: nz >= 2, nx*ny*nz below 2^27 voxels (the kernels address
 * the FP64 GMRES iterate, 16 bytes per voxel, with 32-bit byte offsets), fewer
 * than 2^24 interface faces (anode plus cathode), nx and ny at most 2^21 and
 * ny*nz at most 2^23 (the kernels' index division).
 * Errors: MBX_EINVAL (bad sizes/parameters), MBX_ELABEL, MBX_ENOMEM, MBX_EHIP. */
int mbx_cell_create(const uint8_t *labels, int nx, int ny, int nz,
                    const mbx_params *p, void *stream, mbx_cell **out);

/* Release all device memory of the cell (null is ignored). */
void mbx_cell_destroy(mbx_cell *c);

/* Advance one implicit Euler step of size dt (s), eq. 2.13: solve
 * F(u^{n+1}; u^n) = 0 by Newton + preconditioned GMRES.  If Newton fails
 * (no convergence within newton_max iterations, or no 10% decrease of the
 * residual over 4 iterations after the 8th), the step is retried once as two
 * steps of dt/2 (the same scheme on a finer time grid; info->substeps).
 * Transactional: on any error (MBX_ENEWTON, MBX_ENAN, MBX_EHIP) the state
 * stays at u^n.  info may be null.  Blocks until the step is complete. */
int mbx_cell_step(mbx_cell *c, double dt, mbx_step_info *info);

/* Change the applied current (A) for the following steps (parameter mu of
 * Sec. 2.5 enters affinely through the boundary term). */
int mbx_cell_set_current(mbx_cell *c, double I_app);

/* Sizes: voxels, anode interface faces (= plated-amount entries), cathode
 * interface faces, cathode collector faces.  Any pointer may be null. */
int mbx_cell_counts(const mbx_cell *c, int64_t *n_vox, int64_t *n_an_faces,
                    int64_t *n_ca_faces, int64_t *n_top);

/* Copy the state out.  cfield, phi: N doubles each; n_pl: n_an_faces doubles
 * (anode face order above).  device_ptrs = 1: the three pointers are device
 * addresses (copied device-to-device on the cell's stream), 0: host.  Any of
 * the three pointers may be null to skip that field. */
int mbx_cell_get_state(const mbx_cell *c, double *cfield, double *phi, double *n_pl,
                       int device_ptrs);

/* Overwrite the state (both u^n and the Newton iterate); same layouts as
 * mbx_cell_get_state.  All three pointers are required. */
int mbx_cell_set_state(mbx_cell *c, const double *cfield, const double *phi,
                       const double *n_pl, int device_ptrs);

/* Snapshot capture for the POD of Sec. 2.5, whose snapshot sets hold the
 * solution of every time step and the intermediate Newton stages.  From this
 * call on, the cell appends its state as one column of c_snap and one of
 * phi_snap (device addresses, column-major, leading dimension ld >= N, room
 * for capacity columns; either may be null to skip that field): first the
 * current state, then the iterate after every accepted Newton update (the
 * last one of a step is the step's solution).  The columns of a step that
 * fails are dropped again (the state is restored to u^n).  Once capacity
 * columns are taken, further ones are counted as dropped and not written.
 * The copies run on the cell's stream, ordered with its steps.  The caller
 * owns the buffers and keeps them alive while capture is on; capacity = 0
 * (or both pointers null) turns capture off.  Errors: MBX_EINVAL. */
int mbx_cell_capture(mbx_cell *c, double *c_snap, double *phi_snap, int64_t ld, int capacity);

/* Columns written since mbx_cell_capture, and columns that found no room. */
int mbx_cell_captured(const mbx_cell *c, int *count, int *dropped);

/* Cell voltage (Sec. 2.5 output functional s_cp): mean over the cathode
 * collector faces of the solid potential extrapolated across half a voxel
 * with the applied flux; the anode collector is the 0 V reference. */
int mbx_cell_voltage(const mbx_cell *c, double *V);

/* Mean lithium concentration of each electrode's active material, mol/m^3:
 * out[0] anode, out[1] cathode (Sec. 2.5 output functional s_ac, the average
 * Li concentration in the electrode, a linear functional of the state). */
int mbx_cell_mean_solid(const mbx_cell *c, double out[2]);

/* Step loop with the voltage cutoff (Sec. 2.5 output s_cp as the stopping
 * criterion of a charge): advances up to max_steps implicit Euler steps of dt
 * (each as mbx_cell_step) and stops after the first step whose cell voltage
 * reaches p->V_cut (see mbx_params; V_cut = 0 runs all max_steps).
 *   V_out     : host, max_steps doubles or null; receives V after each step taken
 *   steps_out : steps completed (required)
 *   cutoff_out: 1 if the cutoff stopped the run, else 0 (may be null)
 *   retried   : steps that were retried as two half steps (may be null)
 * Returns MBX_OK, or the code of the first failed step (the state then stays
 * at the start of that step, *steps_out counts the steps before it). */
int mbx_cell_run(mbx_cell *c, double dt, int max_steps, double *V_out, int *steps_out, int *cutoff_out,
                 int *retried);

/* Adaptive implicit Euler from the cell's current state over [0, t_end]
 * (time-step control of Sec. 2.4; the error estimate and controller are a
 * reading of it).  Each step is one mbx_cell_step without its internal retry.
 * Its local error is estimated from the linear extrapolation of the two
 * previous accepted states, u_pred = u^n + (dt/dt_prev)(u^n - u^(n-1)), which
 * on an implicit Euler trajectory is the explicit Euler step from u^n:
 *   est = max |u^(n+1) - u_pred| / 2
 * over the concentrations (relative to c0 in the electrolyte, c_max in the
 * solid) and the plated amounts (relative to n_c); the potentials are
 * algebraic and do not enter.  The first step has no estimate.  A step whose
 * Newton iteration fails, or whose est > tol, is rolled back and redone with
 * half the step; an accepted step with est <= tol/4 doubles the next step (at
 * most dt_max); a step that would pass t_end is shortened to end there.  The
 * run stops at t_end, after max_steps accepted steps, or after the first step
 * whose voltage reaches p->V_cut.
 *   t_out, V_out : host, max_steps doubles each or null; the time and cell
 *                  voltage after each accepted step
 *   steps_out    : accepted steps (required); rejected_out: rejected steps
 *   cutoff_out   : 1 if the voltage cutoff stopped the run (may be null)
 * Returns MBX_EINVAL for t_end < 0, dt0 <= 0, dt_min <= 0, dt_max < dt_min,
 * tol <= 0 or max_steps < 0; MBX_ENEWTON when the step would have to fall
 * below dt_min (the state then stays at the last accepted step). */
int mbx_cell_run_adaptive(mbx_cell *c, double t_end, double dt0, double dt_min, double dt_max, double tol,
                          int max_steps, double *t_out, double *V_out, int *steps_out, int *rejected_out,
                          int *cutoff_out);

/* Workgroup sizes (threads) the library picked for this cell's single-cell
 * launches of the level-0 multigrid smoother and of J*v: at creation it times
 * 256, 512, 1024, 128 and 64 threads on the cell's own arrays and keeps the
 * fastest (another size must be 3% faster than 256), once per grid size and
 * precision per process (environment MBX_TUNE_FILE: read and append the
 * choices to that file; MBX_TUNE=0: always 256; MBX_TUNE=64/128/256/512/1024:
 * that size).  Results do not depend on the choice.
 * Batched launches use 256.  Either pointer may be null. */
int mbx_cell_launch_shape(const mbx_cell *c, int *smooth0_threads, int *matvec_threads);

/* Lithium inventories (mol) in electrolyte, anode solid, cathode solid and
 * the plated layer (Sec. 2.4 conservative scheme: at convergence the total
 * changes only through the applied current).  out[4]. */
int mbx_cell_inventory(const mbx_cell *c, double out[4]);

/* FP64 residual F(u; u_old) of eq. 2.13 for caller-given u = (c_u, phi_u,
 * n_u) and u_old = (c_old, n_old) (host arrays, layouts as get_state) and
 * step dt, on the cell's geometry and parameters.  Writes the raw rows
 * (mol/s for c and n rows, A for phi rows) to Rc[N], Rphi[N],
 * Rn[n_an_faces] (host).  Does not change the cell's state.  Used to check
 * the operator against a reference implementation. */
int mbx_cell_residual(mbx_cell *c, const double *c_u, const double *phi_u, const double *n_u,
                      const double *c_old, const double *n_old, double dt,
                      double *Rc, double *Rphi, double *Rn);

/* Jacobian-vector product of the Newton system the solver hands to GMRES,
 * at state u = (c_u, phi_u, n_u) with u_old = (c_old, n_old) and step dt
 * (host arrays as for mbx_cell_residual), applied to v (host, 2N doubles:
 * [0,N) concentration, [N,2N) potential entries).  The operator is
 *   J_hat = D_r (J_uu - J_un J_nn^-1 J_nu) D_u,
 * the Jacobian of eq. 2.13 with the plated unknowns eliminated face by face
 * (J_nn is diagonal) and scaled by D_u = diag(c_ref, RT/F) (c_ref = c0 in
 * pores, c_max in solids) and D_r = diag(dt/(h^3 c_ref), 1/(h^2 mu_ref)),
 * mu_ref = max(|I_app|/(nx ny h^2), 1 A/m^2).  Computed by the solver's own
 * linearisation and matrix-free kernel in the cell's precision mode.
 * Writes y (host, 2N doubles).  Does not change the cell's state. */
int mbx_cell_jvp(mbx_cell *c, const double *c_u, const double *phi_u, const double *n_u,
                 const double *c_old, const double *n_old, double dt, const double *v, double *y);

/* Applies the solver's preconditioner M^-1 ~ J_hat^-1 (same operator as in
 * mbx_cell_jvp, linearised at u with u_old and dt) to v (host, 2N doubles);
 * writes z (host, 2N doubles).  In the cell's precision mode.  Does not
 * change the cell's state.  Used to check the preconditioner. */
int mbx_cell_precond(mbx_cell *c, const double *c_u, const double *phi_u, const double *n_u,
                     const double *c_old, const double *n_old, double dt, const double *v, double *z);

/* Solves J_hat x = rhs (operator of mbx_cell_jvp at u, u_old, dt) with the
 * solver's preconditioned GMRES to relative residual rtol; rhs and x are
 * host arrays of 2N doubles; *iters (may be null) receives the GMRES
 * iteration count.  In the cell's precision mode; the cell's state is not
 * changed.  This is the linear-solve service an outer Newton or
 * model-reduction driver would call. */
int mbx_cell_solve(mbx_cell *c, const double *c_u, const double *phi_u, const double *n_u,
                   const double *c_old, const double *n_old, double dt, const double *rhs, double rtol,
                   double *x, int *iters);

/* Batched stepping: advance n cells (all of one precision mode) by one step
 * of dt each, sharing every kernel launch across the cells.  status_out[i]
 * receives each cell's own result code (as mbx_cell_step); the function
 * returns MBX_OK if the batch ran (cells may still have failed individually)
 * or an error for invalid arguments.  infos may be null. */
int mbx_batch_step(mbx_cell *const *cells, int n, double dt, int *status_out,
                   mbx_step_info *infos);

/* ---------------------------------------------------------------- serving
 * Continuous-batching step server for many independent parameter queries
 * (the many-query setting of Sec. 1 and Sec. 2.5, here answered by the full
 * order model).  A request is a voxel image, a parameter set and a number
 * of implicit Euler steps of the server's dt.  One worker thread owns all
 * device work: it admits queued requests first-come first-served while their
 * device footprint (mbx_cell_footprint) fits the budget next to the running
 * cells, creates their cells (state resident in device memory), advances all
 * running cells by one step per mbx_batch_step, and retires a request after
 * its last step (or its first failed step), releasing its memory.  New
 * requests join at the next step.  A request's results do not depend on
 * which other requests share its batches (deterministic per-cell
 * reductions).  submit / poll / result / drain / stats are thread-safe and
 * do not touch the device. */
typedef struct mbx_server mbx_server;

enum { MBX_REQ_DONE = 0, MBX_REQ_QUEUED = 1, MBX_REQ_RUNNING = 2 };

typedef struct {
  int status;            /* MBX_REQ_*, or the negative MBX_E* code the request failed with */
  int steps_done;        /* completed steps */
  double V;              /* cell voltage after the last completed step, V */
  double t_submit;       /* server clock (s, mbx_server_clock) at submission */
  double t_admit;        /* ... when its cell was created (0 while queued) */
  double t_done;         /* ... when it finished or failed (0 before) */
  int64_t newton_iters;  /* totals over its steps */
  int64_t krylov_iters;
  int64_t n_vox;         /* voxels (after admission) */
  int64_t n_an_faces;    /* anode interface faces = length of the plated-amount array (after admission) */
  int cutoff;            /* 1 if a step brought the voltage to the request's cutoff (p->V_cut); the
                            request stopped after that step */
  int retried;           /* steps that were retried as two half steps (dt/2 each) */
  double s_ac[2];        /* mean anode / cathode solid concentration after the last step, mol/m^3 */
} mbx_request_info;

typedef struct {
  int64_t steps_run;     /* cell-steps completed */
  int64_t batches;       /* batched steps launched */
  double busy_s;         /* wall time spent inside batched steps, s */
  int64_t bytes_in_use;  /* footprint of the admitted requests, bytes */
  int running, queued;
} mbx_server_info;

/* Create a server: budget_bytes of device memory for cells, precision mode
 * (MBX_FP64 / MBX_MIXED) and step dt (s) shared by all requests, keep_state
 * = 1 to keep each finished request's final state on the host for
 * mbx_server_result, stream as for mbx_cell_create (device work runs on the
 * device current at this call).  Starts the worker thread.
 * Errors: MBX_EINVAL, MBX_EHIP. */
int mbx_server_create(int64_t budget_bytes, int precision, double dt, int keep_state, void *stream,
                      mbx_server **out);

/* Queue a request (labels and parameters as mbx_cell_create; copied) for
 * n_steps steps, fewer if p->V_cut stops it first; *id receives its handle.  p->precision must equal the
 * server's.  MBX_EBUDGET if the request alone exceeds the budget. */
int mbx_server_submit(mbx_server *s, const uint8_t *labels, int nx, int ny, int nz, const mbx_params *p,
                      int n_steps, int64_t *id);

/* Snapshot of a request's progress. MBX_EINVAL for an unknown id. */
int mbx_server_poll(mbx_server *s, int64_t id, mbx_request_info *info);

/* Final state of a finished request (keep_state servers): layouts as
 * mbx_cell_get_state, host pointers, any may be null.  MBX_ESTATE if the
 * request is not MBX_REQ_DONE or the server does not keep states. */
int mbx_server_result(mbx_server *s, int64_t id, double *cfield, double *phi, double *n_pl);

/* Message of a request that ended with an error (status < 0), as
 * mbx_last_error gave it when the request failed: copied, NUL-terminated and
 * truncated, into buf of len bytes (host memory owned by the caller).  An
 * empty string for a request without an error.  MBX_EINVAL for an unknown id
 * or a null buf / len < 1. */
int mbx_server_error(mbx_server *s, int64_t id, char *buf, int len);

/* Block until no request is queued or running, at most timeout_s seconds
 * (MBX_ESTATE on time-out). */
int mbx_server_drain(mbx_server *s, double timeout_s);

/* Seconds since the server was created (the clock of mbx_request_info). */
double mbx_server_clock(const mbx_server *s);

int mbx_server_stats(mbx_server *s, mbx_server_info *out);

/* Stop the worker (after the step in flight) and release every cell. */
void mbx_server_destroy(mbx_server *s);

/* Kernel timing for measurement: after mbx_profile(k), every launch of
 * kernel class k (1 FP64 residual + linearisation, 2 matrix-free J*v,
 * 3 level-0 multigrid smoothing half-sweep, 4 whole preconditioner
 * application, 5 Gram-matrix kernel of mbx_pod; 0 stops timing) is bracketed by a pair of HIP events recorded
 * on the stream it runs on, together with the launch's algorithmic bytes
 * (every array element the operation must read or write, counted once).
 * Class 3 brackets each group of back-to-back half sweeps of one V-cycle side
 * with one event pair.  mbx_profile clears earlier records.
 * mbx_profile_read waits for the recorded events and returns the number of
 * timed launches, their summed duration (ms) and summed algorithmic bytes.
 * Timing adds event records to the stream; it is not meant to be left on in
 * production. */
int mbx_profile(int kernel);
int mbx_profile_read(int64_t *launches, double *total_ms, double *total_bytes);

/* Most snapshots one POD takes (the host eigen-decomposition is O(m^3)). */
#define MBX_POD_MAX_SNAPSHOTS 512

/* POD of a snapshot set by the method of snapshots (Sec. 2.5; Sirovich's
 * method, which the paper cites): K = S^T W S, K = V diag(lam) V^T with lam
 * descending, sigma_i = sqrt(max(lam_i, 0)), modes u_i = S v_i / sigma_i.
 * S: n x m snapshots, device, column-major, leading dimension lds >= n,
 * 1 <= m <= MBX_POD_MAX_SNAPSHOTS.  w: n positive weights of the inner product
 * (device; null: Euclidean).  A mode is kept while sigma_i > rtol sigma_1
 * (Sec. 3.2 uses rtol = 1e-7), at most k_max of them.  Each mode's sign
 * makes the largest-magnitude entry of v_i positive (the first on ties).
 * Outputs: modes (device, n x k_max column-major, leading dimension
 * ldm >= n; columns k.. are not written), sigma (host, all m singular
 * values, descending), *k_out = number of kept modes.  K is formed on the
 * GPU's FP64 matrix cores; its eigen-decomposition runs on the host
 * (Householder tridiagonalisation and implicit QR, mbx_sym_eig).  Singular values below about 1e-8 sigma_1 carry the rounding of
 * K (the method squares the condition number).  Allocates a device
 * workspace of at most about 8 (2560 x 1024 + m^2 + 32 m ceil(k/32)) bytes
 * (the partial Gram tiles of the row slices, K, the eigenvector
 * coefficients) for the call and synchronises the stream.  Errors: MBX_EINVAL, MBX_ENOMEM,
 * MBX_ENAN (non-finite Gram matrix), MBX_EHIP. */
int mbx_pod(const double *S, int64_t n, int m, int64_t lds, const double *w, double rtol, int k_max,
            double *modes, int64_t ldm, double *sigma, int *k_out, void *stream);

/* mbx_pod without any device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Arguments, results, errors and numerics are those of
 * mbx_pod (the same kernels, bit-identical results).  The workspace is a
 * static device array of 21 MiB that each device the library runs on holds
 * until the process ends; it covers every m <= MBX_POD_MAX_SNAPSHOTS (a
 * request that would need more fails with MBX_EINVAL and a message).  Its
 * device address is looked up once per device, on the first call with that
 * device current.  Every call on one device shares that device's array:
 * calls that overlap on one device (several threads or streams) race and
 * must be serialised by the caller.  Synchronises the stream.  Host work
 * arrays of O(m^2) doubles still come from the host heap. */
int mbx_pod_noalloc(const double *S, int64_t n, int m, int64_t lds, const double *w, double rtol, int k_max,
                    double *modes, int64_t ldm, double *sigma, int *k_out, void *stream);

/* The eigen-decomposition step of mbx_pod on its own (host memory): A is a
 * symmetric m x m matrix (column-major; exactly symmetric, else
 * MBX_EINVAL), lam receives the m eigenvalues in descending order and V
 * (m x m, column-major) the eigenvectors, signed as in mbx_pod.  Householder
 * reduction to tridiagonal form, then implicit symmetric QR steps with the
 * Wilkinson shift.  Errors: MBX_EINVAL, MBX_ENAN (non-finite entry or no
 * convergence). */
int mbx_sym_eig(int m, const double *A, double *lam, double *V);

/* Device bytes a cell of this size would allocate (for admission control);
 * -1 for a shape mbx_cell_create refuses by its size limits. */
int64_t mbx_cell_footprint(int nx, int ny, int nz, int precision, int n_an_faces, int n_ca_faces);

/* Message for the last failure on this thread ("" if none). */
const char *mbx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MBX_H */
