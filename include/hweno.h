/*
 * hweno.h -- C ABI of the MI355X FP64 HWENO-GR library (libhweno.so).
 *
 * The library evaluates the per-stage spatial residual of the fifth-order
 * finite-volume HWENO scheme with gradient reconstruction for the
 * compressible Navier-Stokes equations (arXiv 2608.10569) and advances it
 * with the SSP-RK3 scheme with modified first-order moments, on one GPU.
 *
 * Problem statement (Sec. 2.1 and 3.1 of the paper): a uniform grid of
 * nx (x ny) cells on [x0,x1] (x [y0,y1]); unknowns per cell are the cell
 * average and the scaled first-order moments of the conserved variables
 * u = (rho, rho*u, (rho*v,) E); ideal gas with ratio of specific heats
 * gamma; viscous terms with the dynamic viscosity mu(T) (the paper's 1/Re)
 * and the Prandtl number Pr; ghost-cell boundary conditions of Remark 4.1.
 *
 * State layout ("D1"): a contiguous FP64 array U[m][c][j][i] (2D) or
 * U[m][c][i] (1D), x index fastest, interior cells only:
 *   m = 0 cell average, 1 xi-moment (1/|I| int u (x-x_i)/dx), 2 eta-moment
 *   (2D only); c = rho, rho*u, (rho*v,) E.
 *   2D: 12 * nx * ny doubles;  1D: 6 * nx doubles.
 *
 * Conventions
 *  - Every function returns hweno_status; nothing throws or aborts across
 *    the ABI (a failed host allocation inside a call is reported as
 *    HWENO_E_NOMEM).  hweno_status_string() names a status.
 *  - Array arguments documented as "device" are GPU pointers (HIP device
 *    memory of the device current when the context was created).  The
 *    caller owns every pointer it passes; the library keeps none after a
 *    call returns, except the workspace given to hweno_set_workspace.
 *  - The library allocates no device memory.  All scratch lives in a
 *    caller-provided workspace of hweno_workspace_bytes() bytes.
 *  - Calls are ordered on the HIP stream set with hweno_set_stream (default:
 *    the null stream).  hweno_rk_step and hweno_residual with a non-NULL
 *    diag synchronise that stream once; other calls are asynchronous.
 *  - Device faults surface at the next synchronising call as
 *    HWENO_E_DEVICE.  A context is not thread-safe; distinct contexts are
 *    independent.
 */
#ifndef HWENO_H
#define HWENO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HWENO_API __attribute__((visibility("default")))

typedef struct hweno_ctx hweno_ctx;

typedef enum hweno_status {
    HWENO_OK = 0,
    HWENO_E_INVAL = 1,          /* invalid argument (size, parameter, BC pairing, NULL) */
    HWENO_E_DEVICE = 2,         /* HIP runtime or kernel error */
    HWENO_E_WORKSPACE = 3,      /* no workspace set, or too small / misaligned */
    HWENO_E_INADMISSIBLE = 4,   /* restart cap reached: a stage kept nonpositive rho or p */
    HWENO_E_NONFINITE = 5,      /* input state with non-finite values or rho<=0 / p<=0 */
    HWENO_E_STATE = 6,          /* no state set yet */
    HWENO_E_NOMEM = 7           /* host memory allocation failed (the context is unchanged
                                   when the failure precedes any change; otherwise recreate it) */
} hweno_status;

/* Ghost-cell rules of Remark 4.1. */
typedef enum hweno_bc_kind {
    HWENO_BC_PERIODIC = 0,      /* must be set on both sides of a direction */
    HWENO_BC_OUTFLOW = 1,       /* ghost cells copy the adjacent interior cell (average and moments) */
    HWENO_BC_INFLOW = 2,        /* prescribed state (average), zero moments */
    HWENO_BC_SLIP = 3,          /* reflective / slip wall / symmetry: normal velocity odd */
    HWENO_BC_NOSLIP = 4         /* adiabatic no-slip wall: both velocity components odd */
} hweno_bc_kind;

typedef struct hweno_grid {
    int dim;                    /* 1 or 2 */
    int nx, ny;                 /* interior cells; each >= 4; ny ignored for dim = 1 */
    double x0, x1, y0, y1;      /* domain; x1 > x0 (and y1 > y0 in 2D) */
} hweno_grid;

/* Eq. (2.1) / (3.1): the paper's 1/Re is mu(T) = mu_ref * (T/T_ref)^mu_exp
 * with T = p/rho; mu_exp = 0 is the paper's constant viscosity. */
typedef struct hweno_physics {
    double gamma;               /* > 1 */
    double Pr;                  /* > 0 */
    double mu_ref;              /* >= 0 (0: Euler limit) */
    double mu_exp;              /* exponent of the power law; 0 = constant */
    double T_ref;               /* > 0 */
} hweno_physics;

typedef struct hweno_bcs {
    int kind[4];                /* hweno_bc_kind for xlo, xhi, ylo, yhi (1D: first two) */
    double inflow[4][4];        /* per side, primitive (rho, u, v, p) used with HWENO_BC_INFLOW;
                                   1D uses (rho, u, p) in the first three slots */
} hweno_bcs;

/* Scheme constants (Sec. 5 preamble and Appendix A). */
typedef struct hweno_options {
    double cfl;                 /* CFL number of the time-step rule (paper: 0.6) */
    double b_visc;              /* viscous time-step constant b (paper: 0.001); <= 0 or +inf
                                   turns the viscous bound b*h^2/mu_ref off; NaN is invalid */
    double eps_pp;              /* positivity floor (paper: 1e-12) */
    double eps_weno;            /* nonlinear-weight epsilon (paper: 1e-8) */
    double t_final;             /* steps are clipped to end at t_final; <= 0: no clipping */
    int linear_weights;         /* 1: omega = gamma (test mode); 0: nonlinear weights */
    int max_halvings;           /* restarts with dt/2 allowed per step (>= 0) */
    int linear_gradients;       /* 1: omega = gamma in the gradient reconstruction only
                                   (the linear counterpart of Remark 3.1); 0: paper */
    int keep_stages;            /* 2D single grid: 1 keeps the residual intermediates of the
                                   three RK stages apart (2 x 248 doubles more workspace per
                                   ghosted cell), so that hweno_rk_step_vjp evaluates three
                                   residuals instead of five; 0 (default): one set */
    int gradients;              /* viscous gradients: 0 (default) HWENO-GR, the paper's scheme
                                   (weak-derivative moments reconstructed, Sec. 2.2 / 3.2);
                                   1 HWENO-DR, its comparison scheme (the convective
                                   reconstruction differentiated with its weights kept,
                                   eqs. (2.5) / (3.5)); the reverse-mode calls refuse DR and a
                                   batch needs one value for all its instances */
} hweno_options;

/* Diagnostics of the last call (Sec. 5 preamble; Table 5.3 PP activity). */
typedef struct hweno_diag {
    double t;                   /* time after the call */
    double dt;                  /* step size used (rk_step) */
    double alpha_star;          /* max over interior face traces of max(|u|,|v|) + c, stage 1 */
    double beta_max;            /* max Lax-Friedrichs coefficient over faces (all stages) */
    double min_rho, min_p;      /* min cell-average density / pressure of the last stage */
    unsigned long long pp_cells;/* cell-stages where the positivity limiter acted */
    int restarts;               /* dt halvings taken by this step */
    int pad;
} hweno_diag;

/* Fills the paper's constants: cfl 0.6, b 0.001, eps_pp 1e-12, eps_weno 1e-8,
 * no clipping, nonlinear weights, 64 halvings (the 1D Sedov start of
 * Example 5.5 needs 51 in its first step), keep_stages 0. */
HWENO_API hweno_status hweno_default_options(hweno_options* opt);

/* Validates the problem and creates a context (host memory only).
 * Errors: HWENO_E_INVAL for a NULL argument, dim not 1/2, nx/ny < 4,
 * empty domain, gamma <= 1, Pr <= 0, mu_ref < 0, T_ref <= 0, unknown BC
 * kind, a periodic side paired with a non-periodic one, inflow density or
 * pressure <= 0, cfl <= 0, eps_pp <= 0, eps_weno <= 0, max_halvings < 0,
 * b_visc or t_final NaN, keep_stages or gradients not 0/1. */
HWENO_API hweno_status hweno_create(const hweno_grid* grid, const hweno_physics* phys,
                                    const hweno_bcs* bcs, const hweno_options* opt,
                                    hweno_ctx** out);

HWENO_API hweno_status hweno_destroy(hweno_ctx* ctx);

/* Device bytes the caller must provide (256-byte aligned). */
HWENO_API hweno_status hweno_workspace_bytes(const hweno_ctx* ctx, size_t* bytes);

/* Hands the library a device buffer of at least hweno_workspace_bytes();
 * it stays owned by the caller and must outlive the context's use. */
HWENO_API hweno_status hweno_set_workspace(hweno_ctx* ctx, void* dev_ptr, size_t bytes);

/* Inflow that varies along a side (Remark 4.1's prescribed inflow state, per
 * boundary cell; Example 5.9's jet).  Single 2D grids only; `side` (0 xlo,
 * 1 xhi, 2 ylo, 3 yhi) must be of kind HWENO_BC_INFLOW.  prim: host array of
 * n primitive states (rho, u, v, p), row-major (n, 4), copied before return:
 * n = ny for an x side (boundary rows bottom to top), n = nx for a y side
 * (boundary columns left to right; the ghost columns beyond the corners take
 * the end states).  Every ghost cell of boundary cell k gets state k with zero
 * moments.  prim = NULL returns the side to its constant state.  Errors:
 * HWENO_E_INVAL for a batch or 1D context, a side of another kind, a wrong n,
 * or a state that is not finite with rho > 0 and p > 0.  Kept across
 * hweno_set_workspace. */
HWENO_API hweno_status hweno_set_inflow_profile(hweno_ctx* ctx, int side, const double* prim,
                                                int n);

/* Inflow data that vary in time (Example 5.11's forced inflow).  Stores for
 * `side` (kind HWENO_BC_INFLOW, single 2D grid) the profiles in force at the
 * three stage times of the next hweno_rk_step_inflow call: prim1 at t^n,
 * prim2 at t^n + dt, prim3 at t^n + dt/2 (the stage times of eq. (2.12)), each
 * in the layout and with the checks of hweno_set_inflow_profile.  All three
 * NULL clears the side's stage profiles.  Other calls keep using the side's
 * profile or constant state. */
HWENO_API hweno_status hweno_set_inflow_stages(hweno_ctx* ctx, int side, const double* prim1,
                                               const double* prim2, const double* prim3, int n);

/* One SSP-RK3 step of fixed size dt > 0 in which every side with stage
 * profiles (hweno_set_inflow_stages) fills its ghost cells of stage k from
 * profile k.  Stage times are fixed by dt, so a rejected stage is an error
 * (HWENO_E_INADMISSIBLE) instead of a restart.  Single 2D grids only
 * (HWENO_E_INVAL otherwise); diag as for hweno_rk_step. */
HWENO_API hweno_status hweno_rk_step_inflow(hweno_ctx* ctx, double dt, hweno_diag* diag);

/* Masked domain (Examples 5.8 and 5.10: a non-rectangular domain inside the
 * grid's rectangle).  mask: host array of ny x nx bytes, row-major (j * nx + i),
 * nonzero = solid; copied before return.  Every solid cell within 4 cells of
 * the fluid (in both directions) is filled before each residual as the
 * mirror image, across the nearest wall face along +x, -x, +y, -y (ties in
 * that order), of a fluid cell, with the parities of the box walls (Remark
 * 4.1) for `wall` = HWENO_BC_SLIP (reflective) or HWENO_BC_NOSLIP (adiabatic
 * no-slip); a mirror off the grid or in solid falls back to the first fluid
 * cell in that direction.  Solid cells carry no residual (zeros from
 * hweno_residual), keep their state through the RK stages, and are not
 * checked for admissibility; their values in hweno_get_state are those of
 * the last fill.  mask = NULL removes the mask.  Single 2D grids only; the
 * reverse-mode calls refuse a masked grid.  Errors: HWENO_E_INVAL (batch or
 * 1D context, another wall kind, no fluid cell). */
HWENO_API hweno_status hweno_set_solid(hweno_ctx* ctx, const unsigned char* mask, int wall);

/* Solid cells that hold a prescribed state instead of a mirror image
 * (Example 5.10: the exact post-shock state imposed along part of the bottom
 * of its channel, beside a reflective wall).  fixed: host array of ny x nx
 * bytes, row-major, nonzero = such a cell, each solid in the mask of
 * hweno_set_solid; copied before return.  state: host (rho, u, v, p).  Every
 * such cell within 4 cells of the fluid is set before each residual to the
 * conservative state with zero first moments, as the ghost cells of an
 * inflow side are (Remark 4.1); they count as solid for the mirror search of
 * the other solid cells and are never a mirror's source.  fixed = NULL makes
 * every solid cell a mirror again; hweno_set_solid clears the setting.
 * Errors: HWENO_E_INVAL (no mask, batch or 1D context, a fixed cell that is
 * not solid, state NULL, rho or p not positive, a value not finite). */
HWENO_API hweno_status hweno_set_solid_state(hweno_ctx* ctx, const unsigned char* fixed,
                                             const double* state);

/* Stream (hipStream_t) on which all later work of this context is ordered. */
HWENO_API hweno_status hweno_set_stream(hweno_ctx* ctx, void* hip_stream);

/* Copies a D1 state (device) in and sets the time.  Asynchronous. */
HWENO_API hweno_status hweno_set_state(hweno_ctx* ctx, const double* U, double t);

/* Copies the current state out (device, D1) and returns the time. */
HWENO_API hweno_status hweno_get_state(hweno_ctx* ctx, double* U, double* t);

/* Spatial residual of eq. (2.2) / (3.2) at the state U (device, D1):
 * R (device, same layout as U) receives (F^1, F^2[, F^3]); Vhat (device)
 * receives the modified moments of eq. (2.4) / (3.4): 1D Vhat[c][i]
 * (3*nx), 2D Vhat[q][j][i] with q = hat-v of c = 0..3, then hat-w of
 * c = 0..3 (8*nx*ny).  Uses the workspace; leaves the context state alone.
 * diag may be NULL (no synchronisation). */
HWENO_API hweno_status hweno_residual(hweno_ctx* ctx, const double* U, double* R, double* Vhat,
                                      hweno_diag* diag);

/* For callers that cannot allocate device memory or hand the library a
 * workspace -- code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc: hweno_residual with every intermediate in a
 * library-owned static device buffer of HWENO_NOALLOC_BYTES (256 MiB) per
 * device, which each device the library runs on holds until the process
 * ends.  Same arguments, results and diag as hweno_residual (the same
 * kernels, so the same bits); no hweno_set_workspace is needed and the
 * context's workspace and state are left alone.  The call allocates nothing
 * (no hipMalloc/hipFree, no host allocation); its first call on a device
 * looks up the buffer's device address once.
 * Size limit: 2D needs 1776 * (nx + 8) * (ny + 8) bytes plus about 3 KiB
 * (e.g. up to 380 x 380 cells), 1D 352 * (nx + 8) plus 512 bytes; larger
 * grids return HWENO_E_WORKSPACE.  Single grids without inflow profiles,
 * stage profiles or a solid mask (those live in the workspace): otherwise
 * HWENO_E_INVAL.  All calls on one device share the buffer and it keeps the
 * last call's contents (every value a call reads it has written itself
 * first): calls that overlap on one device -- concurrent streams, threads
 * or contexts -- race and must be serialised by the caller. */
#define HWENO_NOALLOC_BYTES ((size_t)256 << 20)
HWENO_API hweno_status hweno_residual_noalloc(hweno_ctx* ctx, const double* U, double* R,
                                              double* Vhat, hweno_diag* diag);

/* One SSP-RK3 step of eq. (2.12) on the context state.  dt > 0: that step;
 * dt <= 0: dt = min(cfl*h/alpha*, b*h^2/mu_ref, t_final - t) with alpha*
 * from the stage-1 face traces (Sec. 5 preamble).  A stage with a cell of
 * nonpositive density or pressure (or a non-finite value) rejects the step,
 * which is redone from t^n with dt/2, at most max_halvings times; then
 * HWENO_E_INADMISSIBLE with the state unchanged.  Synchronises once per
 * attempt. */
HWENO_API hweno_status hweno_rk_step(hweno_ctx* ctx, double dt, hweno_diag* diag);

/* One SSP-RK3 step of size dt > 0 with a prescribed source added to the
 * residual of every stage (manufactured solutions, Examples 5.1 and 5.2):
 * src1, src2, src3 (device, layout of R in hweno_residual) are the source
 * moments at the stage times t, t + dt and t + dt/2.  Since the sources fix
 * the stage times there are no restarts: a stage with a nonpositive density
 * or pressure returns HWENO_E_INADMISSIBLE with the state unchanged.
 * Synchronises once. */
HWENO_API hweno_status hweno_rk_step_source(hweno_ctx* ctx, double dt, const double* src1,
                                            const double* src2, const double* src3,
                                            hweno_diag* diag);

/* Reverse mode (vector-Jacobian product) of hweno_residual at the state U
 * (device, D1), single 1D or 2D grids:
 *   Ubar = (dR/dU)^T Rbar + (dVhat/dU)^T Vbar        (device, D1, overwritten)
 *   *mu_bar = (dR/dmu_ref) . Rbar                    (host double; NULL: skip)
 * With mu_exp != 0 the viscosity mu_ref (T/T_ref)^mu_exp is differentiated
 * with respect to the state at every flux point, and mu_bar is the
 * derivative in mu_ref of the whole law (T_ref and mu_exp held fixed).
 * Rbar has the layout of R, Vbar that of Vhat (NULL: zero).  The branches of
 * the forward point are kept (positivity-limiter thetas and their argmin
 * points, the Lax-Friedrichs maximum and its argmax, |.| in the nonlinear
 * weights with derivative sign(x), 0 at 0); ties go to the lowest index.
 * Every sum is a fixed-order gather, so results are bitwise reproducible.
 * Uses the workspace (the forward intermediates are recomputed); with a
 * non-NULL mu_bar the call synchronises.  Reverse-mode part of the
 * differentiable rollout (the paper's
 * scheme of eq. (3.2); adjoint of its Sec. 3 residual).  Masked grids
 * (hweno_set_solid): solid cells carry no residual, so Rbar and Vbar there
 * are ignored; the adjoint of the mirror fill (Remark 4.1 applied inside the
 * grid) sends the solid cells' share to their mirror sources, and Ubar is
 * zero on every solid cell.  HWENO_E_INVAL also for a context with
 * options.gradients = 1 (DR). */
HWENO_API hweno_status hweno_residual_vjp(hweno_ctx* ctx, const double* U, const double* Rbar,
                                          const double* Vbar, double* Ubar, double* mu_bar);

/* Reverse mode of one SSP-RK3 step of eq. (2.12) taken with the fixed step
 * dt > 0 from the state U0 (device, D1), single 1D or 2D grids (mu(T) as in
 * hweno_residual_vjp): with
 * U3 = step(U0) as hweno_rk_step computes it for that dt,
 *   U0bar = (dU3/dU0)^T U3bar              (device, D1, overwritten)
 *   *mu_bar = (dU3/dmu_ref) . U3bar        (host double; NULL: skip)
 * dt is held constant (the time-step rule is not differentiated).  The two
 * intermediate stages are recomputed from U0 with the forward kernels; the
 * three stage residual adjoints then run in reverse, branch and tie rules as
 * in hweno_residual_vjp, bitwise reproducible.  Each adjoint needs the
 * intermediates of its stage residual: with keep_stages = 0 they are
 * recomputed (five residual evaluations per call), with keep_stages = 1 the
 * second and third stage keep theirs (three); the results are the same bits.
 * U3bar must not overlap U0.
 * Masked grids: each stage fills the solid cells next to the fluid from
 * their mirror sources in place and leaves every solid cell at that filled
 * input, so U3 there is the mirror image of the last stage input (fluid
 * values, with the wall signs) and U3bar on solid cells flows back to those
 * sources; a caller that takes solid cells as no data passes zeros there.
 * U0bar is zero on the solid cells next to the fluid (their input values are
 * overwritten).
 * Uses the workspace; leaves the context state alone; with a non-NULL
 * mu_bar the call synchronises.  HWENO_E_INVAL for dt <= 0 (and, as for
 * hweno_residual_vjp, for DR contexts).  1D grids always recompute (five
 * residual evaluations per call). */
HWENO_API hweno_status hweno_rk_step_vjp(hweno_ctx* ctx, const double* U0, double dt,
                                         const double* U3bar, double* U0bar, double* mu_bar);

/* Recorded steps: the step adjoint from a recording instead of a
 * recomputation (single 2D grids; HBM spent to skip the three stage
 * residuals hweno_rk_step_vjp evaluates).  A recording buffer holds nslots
 * slots; each keeps the three ghosted stage inputs of one RK step and the
 * full intermediates of their residuals (966 doubles per ghosted cell, plus
 * the slot descriptors).
 * hweno_record_bytes: size of a buffer for nslots slots.
 * hweno_set_record: device buffer (owned by the caller, at least
 *   hweno_record_bytes long; HWENO_E_WORKSPACE if shorter) for nslots slots;
 *   nslots = 0 removes it.  Every slot starts unrecorded.
 * hweno_rk_step_record: one SSP-RK3 step of the fixed size dt > 0 from U0
 *   (device, D1) into U3 (device, D1; may not overlap U0), recorded in slot
 *   `slot`.  The step is not checked for admissibility: it is meant to
 *   repeat a step the forward pass has already taken.  Leaves the context
 *   state alone.  Its residuals run the full-layout kernels of the
 *   reverse mode, whose roundings differ from the forward's in a few
 *   entries: U3 agrees with hweno_rk_step's result to within a unit or so in
 *   the last place.
 * hweno_rk_step_vjp_recorded: U0bar = (dU3/dU0)^T U3bar of the step recorded
 *   in `slot`: the same bits as hweno_rk_step_vjp from that step's U0 and
 *   dt.  *mu_bar as hweno_rk_step_vjp (the call synchronises); mu_bar = NULL
 *   adds this step's mu adjoint to a device-side running sum instead, with
 *   no synchronisation (hweno_take_mu_bar reads and clears it; a call with
 *   a non-NULL mu_bar restarts it).  HWENO_E_INVAL for an unrecorded slot.
 * The recordings use the buffer until the next hweno_rk_step_record of the
 * slot or hweno_set_record; HWENO_E_INVAL as for hweno_rk_step_vjp.  Masked
 * grids as in hweno_rk_step_vjp. */
HWENO_API hweno_status hweno_record_bytes(const hweno_ctx* ctx, int nslots, size_t* bytes);
HWENO_API hweno_status hweno_set_record(hweno_ctx* ctx, void* buffer, size_t bytes, int nslots);
HWENO_API hweno_status hweno_rk_step_record(hweno_ctx* ctx, int slot, const double* U0,
                                            double dt, double* U3);
HWENO_API hweno_status hweno_rk_step_vjp_recorded(hweno_ctx* ctx, int slot,
                                                  const double* U3bar, double* U0bar,
                                                  double* mu_bar);
/* The running sum of mu adjoints of hweno_rk_step_vjp_recorded calls made
 * with mu_bar = NULL (host double), which is then cleared.  Synchronises. */
HWENO_API hweno_status hweno_take_mu_bar(hweno_ctx* ctx, double* mu_bar);

/* Per-kernel-class GPU time, measured with HIP events while timing is
 * enabled.  A class of one kernel has the kernel record the events at the
 * start and end of its execution (hipExtLaunchKernel: the dispatch is not
 * counted); classes 4 and 6 record them on the stream around their launches.
 * Classes:
 * 0 ghost fill, 1 characteristic reconstruction + limiter, 2 weak-derivative
 * moments, 3 gradient reconstruction + volume flux, 4 face fluxes, 5 stage
 * update / assembly, 6 a whole batched run (hweno_batch_run), 7 face fluxes
 * fused with the stage update / assembly (tiles.flux = 0). */
typedef struct hweno_timing {
    double ms[8];                       /* summed elapsed milliseconds */
    unsigned long long launches[8];     /* timed launches */
} hweno_timing;

/* enable = bit mask of the kernel classes above to record (bit k = class k;
 * 0 stops recording; events are created on first use).  Each recorded launch
 * adds two event records to the stream, so time a long run with the classes
 * of interest only.  At most 1024 launches are recorded between two reads of
 * the totals (rk_step reads them at the end of every step). */
HWENO_API hweno_status hweno_set_timing(hweno_ctx* ctx, int enable);

/* Synchronises the stream, returns the totals; reset != 0 zeroes them. */
HWENO_API hweno_status hweno_get_timing(hweno_ctx* ctx, hweno_timing* out, int reset);

HWENO_API const char* hweno_status_string(hweno_status s);

/* ---------------------------------------------------------------------------
 * Batches: many independent 2D grids of different sizes and physics advanced
 * together.  Every kernel launch of the pipeline covers all instances (a
 * block finds its instance from a prefix table of block counts), and a run of
 * nsteps steps is recorded once as a HIP graph and replayed with one launch.
 * Each instance keeps its own step rule (Sec. 5 preamble: dt from its stage-1
 * wave speed, its viscosity and its t_final, computed on the device), its own
 * restarts (a rejected step is retried with dt/2 in the next step slot) and
 * its own diagnostics.  The workspace, stream and timing calls above apply to
 * a batch context; the single-grid state, residual, step and adjoint calls
 * return HWENO_E_INVAL for it.
 * ------------------------------------------------------------------------- */
#define HWENO_BATCH_MAX 4096

/* n instances (1 <= n <= HWENO_BATCH_MAX); grids[i].dim must be 2; each
 * instance is validated as by hweno_create, and all must have the same
 * options.gradients.  Arrays of length n. */
HWENO_API hweno_status hweno_batch_create(int n, const hweno_grid* grids,
                                          const hweno_physics* phys, const hweno_bcs* bcs,
                                          const hweno_options* opts, hweno_ctx** out);

/* State and time of instance i (device, D1 layout of that instance). */
HWENO_API hweno_status hweno_batch_set_state(hweno_ctx* ctx, int i, const double* U, double t);
HWENO_API hweno_status hweno_batch_get_state(hweno_ctx* ctx, int i, double* U, double* t);

/* Advances every instance by nsteps accepted SSP-RK3 steps (fewer if its
 * t_final is reached).  One graph launch covers the run; instances that needed
 * restarts finish with extra single-step launches.  With two or more
 * instances the graph holds two concurrent chains, each advancing a group of
 * instances (consecutive in the schedule order, about equal cells), so one
 * group's reconstruction runs beside the other's memory-bound kernels; each
 * instance's results do not depend on the grouping.  Checks the input states
 * first (HWENO_E_NONFINITE for an instance with a bad cell; it is not
 * advanced).  An instance that exhausts max_halvings stops at its last
 * accepted state and the call returns HWENO_E_INADMISSIBLE after the others
 * have finished.  Synchronises. */
HWENO_API hweno_status hweno_batch_run(hweno_ctx* ctx, int nsteps);

/* Diagnostics of instance i from the last run: t, dt of its last accepted
 * step, alpha_star / beta_max / min_rho / min_p of its last attempt,
 * pp_cells summed over the run's accepted steps, restarts in the run; pad
 * holds the number of accepted steps. */
HWENO_API hweno_status hweno_batch_get_diag(hweno_ctx* ctx, int i, hweno_diag* out);

/* Work per block of the tunable kernels and the instance order of a launch. */
typedef struct hweno_tiles {
    int recon;      /* cells per block of the characteristic reconstruction: 16 or 32 */
    int grad;       /* cells per block of the gradient reconstruction: 32 or 64; 0:
                       the weak moments (eqs. 3.6-3.8) are formed inside the gradient
                       kernel, per 16 x 4 tile of cells and the ring around it, in
                       LDS instead of through HBM (same results; the reverse mode's
                       forward launches keep the separate kernels, whose weak
                       moments the adjoint reads) */
    int flux;       /* faces per block of the face-flux kernels: 64 or 128; 0: no
                       separate flux kernels -- the update kernel forms the fluxes
                       of each 32 x 8 tile of cells in LDS (same results) */
    int order;      /* batch schedule: 0 instances as given, 1 largest first */
    int xcd;        /* 1: each of the 8 XCDs (own L2) takes a contiguous range of a
                       launch's blocks, so neighbouring rows share an L2; 0: launch order */
} hweno_tiles;

/* 2D contexts (single grid or batch).  Results do not depend on the tiles.
 * A new context uses recon 32, grad 32, flux 0, order 0, xcd 1. */
HWENO_API hweno_status hweno_get_tiles(const hweno_ctx* ctx, hweno_tiles* out);
HWENO_API hweno_status hweno_set_tiles(hweno_ctx* ctx, const hweno_tiles* tiles);

/* Autotuner: times `reps` residual evaluations (each with a stage update) of
 * the current state(s) for each candidate tile of every tunable kernel, keeps
 * the fastest per kernel (for the face fluxes: split or fused into the
 * update, by the time of fluxes plus update; for the weak moments and the
 * gradients: split or fused, by the time of both), then the faster block order
 * and (batches) the faster instance order, and sets them; `chosen` may be
 * NULL.  Needs the state(s) set; leaves them unchanged.  Synchronises. */
HWENO_API hweno_status hweno_autotune(hweno_ctx* ctx, int reps, hweno_tiles* chosen);

#ifdef __cplusplus
}
#endif

#endif /* HWENO_H */
