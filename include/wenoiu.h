/*
 * wenoiu.h -- C ABI of libwenoiu, the MI355X (gfx950) implementation of the
 * WENO interpolation-based, upwind-biased (WENOIU) schemes with free-stream
 * preservation of Li & Sun (arXiv 1810.11103) for the 2-D Euler equations on
 * curvilinear grids.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers to fp64 memory owned by the
 *    caller; the library never frees them.  Apart from wiu_batched_plan (which
 *    allocates the plan's tables and scratch, freed by wiu_plan_destroy), no
 *    entry point allocates device memory: scratch comes from a caller-provided
 *    workspace `ws` of at least wiu_workspace_bytes() bytes (256-byte aligned).
 *  - Layout is structure-of-arrays, row-major, the xi index i fastest, no
 *    padding.  A conservative state U is [4][ny][nx] = (rho, rho u, rho v, e)
 *    with e = p/(gamma-1) + rho (u^2+v^2)/2 (Sec. 2.1).  Node coordinates
 *    x, y are [ny][nx].
 *  - Metric array M (wiu_metrics_size() bytes): nine planes of
 *    (ny + 2 WIU_GHOST) x (nx + 2 WIU_GHOST) doubles, node (i, j) at
 *    (j + WIU_GHOST) * (nx + 2 WIU_GHOST) + (i + WIU_GHOST), followed by an
 *    8-double tag recording the scheme and grid the metrics were built for:
 *      plane 0 xi_x^, 1 xi_y^, 2 eta_x^, 3 eta_y^, 4 J^{-1}  at nodes (i, j)
 *      plane 5 xi_x^, 6 xi_y^ at (i+1/2, j); 7 eta_x^, 8 eta_y^ at (i, j+1/2)
 *    (hatted metrics carry the factor J^{-1}, Sec. 2.1).
 *  - Every call is asynchronous on `stream` (a hipStream_t, 0 = null stream)
 *    and returns a host-side code: WIU_OK, or a negative WIU_E* code when the
 *    arguments fail the host checks (nothing is launched then).  Conditions
 *    found on the device (folded grid cell, non-physical state, metrics of
 *    another scheme) latch bits into a status word in `ws`, read with
 *    wiu_status().
 *  - Calls that share one workspace must not overlap in time (use one stream
 *    per workspace).
 */
#ifndef WENOIU_H
#define WENOIU_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* wiu_stream_t; /* hipStream_t */

/* Scheme variants: third/fifth order with one or two midpoints
 * (Eqs. 3.4, 3.8, 3.16, 3.20 with their central operators 3.7, 3.9, 3.19,
 * 3.21) and the seventh-order schemes of the Appendix with one, two, four and
 * six midpoints (r = 4 interpolation of Table A1 with the fourth-order
 * mapping).  Two printed Appendix coefficients are read as corrected (7-2MP:
 * f_j weight -93; 7-6MP: node term 3840 f_j), the values for which each h
 * decomposes into its printed central operator (Eq. 2.7). */
enum {
  WIU_3_1MP = 0, WIU_3_2MP = 1, WIU_5_1MP = 2, WIU_5_2MP = 3,
  WIU_7_1MP = 4, WIU_7_2MP = 5, WIU_7_4MP = 6, WIU_7_6MP = 7
};

/* Boundary rule per direction.  PERIODIC: states wrap; coordinates repeat
 * shifted by the period.  TRANSMISSIVE: states copy the boundary node;
 * coordinates extend linearly from the last two nodes.  (The paper fixes no
 * boundary rule; these are the library's.) */
enum { WIU_BC_PERIODIC = 0, WIU_BC_TRANSMISSIVE = 1 };

/* Rule for the states beyond one side of a non-periodic direction (the
 * paper states none; the library's), in wiu_grid.side[] ordered x low,
 * x high, y low, y high:
 *   WIU_SIDE_TRANSMISSIVE  copy of the boundary node (default, value 0);
 *   WIU_SIDE_WALL          reflecting slip wall: mirror image about the
 *                          boundary node with the momentum component along
 *                          the boundary node's metric direction reversed;
 *   WIU_SIDE_FIXED         the conservative state wiu_grid.fixed[side]
 *                          (e.g. supersonic inflow).
 * Coordinates extend linearly beyond every non-periodic side.  The rules
 * are ignored for periodic directions.
 *   WIU_SIDE_INTERFACE     (blocks of a batched plan only, wiu_block) the
 *                          side continues into a side of another block;
 *                          see the multi-block section below. */
enum { WIU_SIDE_TRANSMISSIVE = 0, WIU_SIDE_WALL = 1, WIU_SIDE_FIXED = 2, WIU_SIDE_INTERFACE = 3 };

#define WIU_GHOST 4

/* host-side return codes */
#define WIU_OK 0
#define WIU_EINVAL (-1)  /* null pointer, bad size or enum, bad parameter */
#define WIU_EHIP (-2)    /* a HIP runtime call or kernel launch failed */

/* device-latched status bits (wiu_status) */
#define WIU_ST_JACOBIAN 1 /* J^{-1} <= 0 or non-finite at some node (folded cell) */
#define WIU_ST_NONPHYS 2  /* rho <= 0, p <= 0 or a non-finite state entry */
#define WIU_ST_SCHEME 4   /* metrics were built for another scheme or grid */
#define WIU_ST_ARGMAX 8   /* adjoint: no node of a line reproduced its maximum wave speed */

typedef struct {
  int nx, ny;               /* nodes per direction (>= 1; >= 2 if transmissive) */
  int bc_x, bc_y;           /* WIU_BC_* */
  double period_x, period_y; /* domain lengths of periodic directions */
  int side[4];              /* WIU_SIDE_* of x low, x high, y low, y high (0: transmissive) */
  double fixed[4][4];       /* conservative state beyond a WIU_SIDE_FIXED side */
} wiu_grid;

/* Variables the midpoint values are interpolated in (Sec. 2.4): the
 * characteristic variables of the reference node (the paper's choice,
 * Sec. 3.4), or component by component the conservative or the primitive
 * (rho, u, v, p) variables.  All three are taken as deviations from the
 * reference node's values, so a uniform state is reproduced exactly. */
enum { WIU_VARS_CHARACTERISTIC = 0, WIU_VARS_CONSERVATIVE = 1, WIU_VARS_PRIMITIVE = 2 };

/* Nonlinear weights of the interpolation: Jiang-Shu (Eqs. 3.12-3.13, with the
 * mapping when ppm = 1; the paper's), or WENO-Z, which Sec. 7 names as a
 * possible alternative: alpha_k = C_k (1 + (tau / (eps + IS_k))^2) with
 * tau = |IS_0 - IS_1|, |IS_0 - IS_2|, |IS_0 + 3 IS_1 - 3 IS_2 - IS_3| for
 * r = 2, 3, 4, no mapping. */
enum { WIU_WEIGHTS_JS = 0, WIU_WEIGHTS_Z = 1 };

/* Split of the leading midpoint flux f_{j+1/2} of each h (Sec. 7 singles it
 * out and names Steger-Warming and van Leer): Lax-Friedrichs with the line
 * eigenvalue (the paper's), Steger-Warming or van Leer along the midpoint
 * metric.  The correction terms of the 2-, 4- and 6-midpoint schemes and
 * the nodal fluxes keep the Lax-Friedrichs split, so FSP is kept. */
enum { WIU_SPLIT_LF = 0, WIU_SPLIT_SW = 1, WIU_SPLIT_VL = 2 };

typedef struct {
  double gamma;    /* ratio of specific heats, 1.4 */
  double alpha_lf; /* Lax-Friedrichs factor alpha, 1.1 (Sec. 2.3: 1.1-1.2) */
  double eps;      /* WENO epsilon, 1e-40 with the mapping (Sec. 3.2(3)) */
  int ppm;         /* 1: piecewise-polynomial mapping of the weights (Eqs. 3.15, 3.23) */
  int vars;        /* WIU_VARS_* */
  double alpha_h;  /* free parameter alpha of the one-midpoint families (Eq. 3.5 for
                      WIU_3_1MP, Eq. 3.17 for WIU_5_1MP, Appendix (1) for WIU_7_1MP);
                      1 gives Eqs. 3.4, 3.16 and the printed 7-1MP scheme and is the
                      only value the other schemes accept.  The metrics depend on it
                      (the central operator Eq. 2.7 derives from the scheme), so
                      wiu_metrics takes the same parameters. */
  int weights;     /* WIU_WEIGHTS_* */
  int split;       /* WIU_SPLIT_* */
} wiu_params;

/* Bytes of the metric array M for this grid (planes + tag). */
size_t wiu_metrics_size(const wiu_grid* g);

/* Bytes of workspace every entry point below needs for this grid. */
size_t wiu_workspace_bytes(const wiu_grid* g);

/* Grid metrics in conservative form (Sec. 2.2), differentiated with the
 * scheme's own central operator delta^{c,(1)} (Sec. 2.3, Eqs. 3.7/3.9/3.19/
 * 3.21, Appendix) whose midpoint values come from a fixed linear
 * interpolation in each direction (Sec. 2.4: six-point central for the
 * third- and fifth-order schemes, eight-point for the seventh-order ones),
 * evaluated on coordinate differences.  In 2-D:
 * xi_x^ = y_eta, xi_y^ = -x_eta, eta_x^ = -y_xi, eta_y^ = x_xi,
 * J^{-1} = x_xi y_eta - x_eta y_xi.  Midpoint metrics interpolate the nodal
 * ones in their own direction.  Only p->alpha_h is read (p may be NULL for
 * alpha_h = 1): with alpha_h != 1 the operator is the one Eq. 2.7 defines
 * for the general one-midpoint form.  Fills the ghost band and the tag of M
 * (scheme, grid, alpha_h) and latches WIU_ST_JACOBIAN if J^{-1} <= 0 at an
 * interior node.  Sweeps latch WIU_ST_SCHEME when the tag does not match the
 * scheme, grid and alpha_h they run with. */
int wiu_metrics(const wiu_grid* g, int scheme, const wiu_params* p, const double* x, const double* y, double* M,
                void* ws, wiu_stream_t stream);

/* Write the tag of M for metrics produced elsewhere (e.g. imported): the
 * caller vouches that they were built with `scheme`'s central operator at
 * p->alpha_h (p may be NULL for alpha_h = 1). */
int wiu_set_metrics_tag(const wiu_grid* g, int scheme, const wiu_params* p, double* M, wiu_stream_t stream);

/* Line eigenvalues of the Lax-Friedrichs splitting (Sec. 2.3):
 * lam_xi[j] = alpha max_i (|U^| + c|xi^|) over row j, lam_eta[i] likewise over
 * column i with eta^.  Outputs are device arrays of ny and nx doubles. */
int wiu_line_eigenvalues(const wiu_grid* g, const wiu_params* p, const double* U, const double* M,
                         double* lam_xi, double* lam_eta, void* ws, wiu_stream_t stream);

/* Spatial residual dU/dt = -[(H^xi_{i+1/2} - H^xi_{i-1/2}) + (H^eta_{j+1/2} -
 * H^eta_{j-1/2})] / J^{-1} (Eq. 2.2 with Eq. 3.2), H = h^+ + h^- of the scheme
 * (Sec. 3.2-3.3), midpoint fluxes from characteristic WENO interpolation with
 * the mapped weights (Secs. 3.2(3), 3.3(3), 3.4) and Lax-Friedrichs line
 * eigenvalues (Sec. 2.3).  dUdt may not alias U. */
int wiu_rhs(const wiu_grid* g, int scheme, const wiu_params* p, const double* U, const double* M, double* dUdt,
            void* ws, wiu_stream_t stream);

/* Time step dt = cfl / max_ij [(|U^| + c|xi^|) + (|V^| + c|eta^|)] / J^{-1},
 * written to the device scalar *dt_dev (no host synchronisation). */
int wiu_cfl_dt(const wiu_grid* g, const wiu_params* p, const double* U, const double* M, double cfl,
               double* dt_dev, void* ws, wiu_stream_t stream);

/* One third-order TVD Runge-Kutta step (Shu-Osher form, Sec. 6) of size
 * *dt_dev (device scalar), in place on U. */
int wiu_rk3_step(const wiu_grid* g, int scheme, const wiu_params* p, double* U, const double* M,
                 const double* dt_dev, void* ws, wiu_stream_t stream);

/* wiu_cfl_dt followed by wiu_rk3_step, sharing one pass over U for the CFL
 * maximum and the first stage's line eigenvalues: *dt_dev receives the CFL
 * time step of U, then U advances by it.  Same results as the two calls. */
int wiu_rk3_step_cfl(const wiu_grid* g, int scheme, const wiu_params* p, double* U, const double* M, double cfl,
                     double* dt_dev, void* ws, wiu_stream_t stream);

/* nsteps (>= 1) CFL-limited RK3 steps in one call, the time marching of
 * Sec. 6: dt_dev[s] (device array of nsteps doubles, caller-owned) receives
 * step s's time step, computed on the device from the state it starts from.
 * Results are those of nsteps wiu_rk3_step_cfl calls, bit for bit; only the
 * first step has a separate maxima pass over U, later steps take the line
 * eigenvalues and the CFL maximum of their state from the last stage of the
 * step before, which accumulates them as it writes that state.  WIU_EINVAL
 * for nsteps < 1 or invalid arguments, before anything is launched. */
int wiu_rk3_steps_cfl(const wiu_grid* g, int scheme, const wiu_params* p, double* U, const double* M, double cfl,
                      int nsteps, double* dt_dev, void* ws, wiu_stream_t stream);

/* ---- Allocation-free RK3 step ------------------------------------------------
 * For callers that cannot allocate device memory or pass a workspace: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same step and same results as wiu_rk3_step (the same
 * kernels), with its scratch (two sets of line maxima and two stage buffers,
 * wiu_noalloc_bytes() bytes) in one static device array of
 * WIU_NOALLOC_SCRATCH_BYTES per device, which each device the library runs
 * on holds from the first call until the process ends; the call itself
 * allocates nothing.  Grids whose scratch exceeds the array (beyond about
 * 1.1 million nodes, e.g. 1024 x 1024 fits) are rejected with WIU_EINVAL
 * before anything is launched.  The current device must be the one `stream`
 * belongs to; the first call on a device looks up the array's address there
 * (make that first call outside graph capture).  Every call on one device
 * shares its array: calls that overlap in time on one device (other streams,
 * other threads) race and must be serialised by the caller.  Device-side
 * conditions latch the WIU_ST_* bits into the caller's device int
 * *status_dev (bits are OR-ed in, never cleared). */
#define WIU_NOALLOC_SCRATCH_BYTES ((size_t)72 << 20)

/* Scratch bytes wiu_rk3_step_noalloc needs for this grid (0 for an invalid
 * grid); a grid is accepted when this is at most WIU_NOALLOC_SCRATCH_BYTES. */
size_t wiu_noalloc_bytes(const wiu_grid* g);

int wiu_rk3_step_noalloc(const wiu_grid* g, int scheme, const wiu_params* p, double* U, const double* M,
                         const double* dt_dev, int* status_dev, wiu_stream_t stream);

/* ---- Adjoints (metrics held fixed) ------------------------------------------
 * Reverse-mode derivatives of the residual and of one RK3 step with respect
 * to the state, for gradients through time integration.  Third- and
 * fifth-order schemes with the paper's configuration only (characteristic
 * variables, alpha_h = 1, Jiang-Shu weights, Lax-Friedrichs split;
 * WIU_EINVAL otherwise).  Non-smooth points:
 * the line eigenvalue's maximum passes its adjoint to the first maximal node
 * of the line; |U^| has derivative sign(U^) with sign(0) = 0.  The result is
 * deterministic (no floating-point atomics). */

/* Ubar = (d rhs / dU)^T Gbar at state U (overwrites Ubar; no aliasing). */
int wiu_rhs_vjp(const wiu_grid* g, int scheme, const wiu_params* p, const double* U, const double* M,
                const double* Gbar, double* Ubar, void* ws, wiu_stream_t stream);

/* Size in bytes of a step record: the line maxima (Sec. 2.3) of the three
 * stage states of one RK3 step, kept by the caller between a forward step
 * and its adjoint so the adjoint need not recompute them (device memory,
 * 8-byte aligned, opaque). */
size_t wiu_step_record_bytes(const wiu_grid* g);

/* wiu_rk3_step that also stores the two intermediate stage states U1, U2
 * (caller-owned [4][ny][nx]) for a later wiu_rk3_step_vjp, and, when `rec`
 * is not NULL, the step record of U, U1, U2. */
int wiu_rk3_step_stages(const wiu_grid* g, int scheme, const wiu_params* p, double* U, const double* M,
                        const double* dt_dev, double* U1, double* U2, void* rec, void* ws, wiu_stream_t stream);

/* nsteps (>= 1) steps of wiu_rk3_step_stages in one call, for the stored
 * stages of a differentiated time integration: step s copies its U_n to
 * stages[s][0] and writes U1, U2 to stages[s][1], stages[s][2] (stages:
 * caller-owned [nsteps][3][4][ny][nx]) and its step record to recs[s]
 * (caller-owned, nsteps records of wiu_step_record_bytes, required); U
 * advances in place by nsteps steps of size *dt_dev.  States and the line
 * maxima of the records are those of nsteps wiu_rk3_step_stages calls bit
 * for bit; only the first step has a separate maxima pass, later steps take
 * the line maxima of their U_n from the last stage of the step before. */
int wiu_rk3_steps_stages(const wiu_grid* g, int scheme, const wiu_params* p, double* U, const double* M,
                         const double* dt_dev, int nsteps, double* stages, void* recs, void* ws, wiu_stream_t stream);

/* Ubar_n = (d U^{n+1} / d U^n)^T Ubar_np1 for one RK3 step of size *dt_dev
 * from U_n.  U1, U2: the stored stage states, or both NULL to recompute them;
 * rec: the step record written with them, or NULL (requires U1, U2 when set;
 * WIU_EINVAL otherwise).  Ubar_n may alias Ubar_np1. */
int wiu_rk3_step_vjp(const wiu_grid* g, int scheme, const wiu_params* p, const double* U_n, const double* U1,
                     const double* U2, const void* rec, const double* M, const double* dt_dev,
                     const double* Ubar_np1, double* Ubar_n, void* ws, wiu_stream_t stream);

/* Synchronise `stream`, return the latched status bits of `ws` in *status
 * and clear them when `clear` is non-zero. */
int wiu_status(void* ws, wiu_stream_t stream, int* status, int clear);

/* Zero the status word and scratch header of a fresh workspace. */
int wiu_workspace_init(void* ws, wiu_stream_t stream);

const char* wiu_strerror(int code);

/* ---- Batched multi-block stepping ------------------------------------------
 * Many independent grid blocks of uneven sizes (the multi-block grids of
 * the paper's motivation, Sec. 1) advanced together: per RK stage one launch
 * of each sweep covers the tiles of all blocks (one workgroup per entry of a
 * device tile table, in XCD-aware order), one wave-maximum pass per step
 * serves the first stage and the eta sweeps of stages 1 and 2 accumulate the
 * next stage's line maxima; the launches of a step can be replayed as one
 * captured HIP graph.
 *
 * Each block's state lives in U_all at off_U (doubles, [4][ny][nx]) and its
 * metrics in M_all at off_M (doubles, wiu_metrics_size() bytes), computed
 * beforehand for the same scheme: with wiu_metrics for a block without
 * interfaces, with wiu_blocks_metrics for a grid whose blocks are coupled.
 * The plan binds these pointers, owns its device tables and scratch
 * (allocated when the plan is created, freed by wiu_plan_destroy) and a
 * per-block time step.
 *
 * Sides of non-periodic directions (x low, x high, y low, y high) take the
 * rules of wiu_grid (side, fixed; zero-initialised fields give transmissive
 * sides) or WIU_SIDE_INTERFACE: the paper motivates its schemes with
 * multi-block grids (Sec. 1) but defines no coupling; the library's rule is
 * that the block's lines continue into the neighbour.  Blocks are
 * right-handed; side s of block b abuts side nbr_side[s] of block nbr[s]
 * (which points back), both with the same number of nodes, and the
 * neighbour is at least WIU_MB_REACH nodes deep across that side.  Along a
 * side a node has a position counted counterclockwise around its block;
 * the two sides meet with those orders opposed (position t is the
 * neighbour's n - 1 - t), and ghost layer m >= 1 is the neighbour's node
 * layer m - 1 (no overlap).  Then
 *   - states beyond the side are the neighbour's (of the same RK stage);
 *   - coordinates beyond it are the neighbour's plus shift[s] (non-zero
 *     across a periodic seam only; the neighbour's shift is its negative),
 *     so both blocks evaluate their metrics on one coordinate field
 *     (free-stream preservation and conservation across the interface);
 *     at a corner the interface of the x direction is crossed first;
 *   - the Lax-Friedrichs eigenvalue of a line (Sec. 2.3) is the maximum over
 *     the whole line through every block it crosses;
 *   - wiu_batched_cfl_dt gives every set of blocks joined by interfaces its
 *     smallest step (steps set from the host must agree within a set).
 * A plan that violates these rules is rejected with WIU_EINVAL. */
#define WIU_MB_REACH 15
typedef struct {
  int nx, ny, bc_x, bc_y;
  double period_x, period_y;
  long long off_U, off_M;
  int side[4];          /* WIU_SIDE_* of x low, x high, y low, y high */
  int nbr[4];           /* WIU_SIDE_INTERFACE: neighbour block index */
  int nbr_side[4];      /* WIU_SIDE_INTERFACE: the neighbour's side (0..3) */
  double shift[4][2];   /* WIU_SIDE_INTERFACE: added to the neighbour's (x, y) */
  double fixed[4][4];   /* WIU_SIDE_FIXED: conservative state */
  long long off_X;      /* wiu_blocks_metrics: x at X_all + off_X, y right after (nx ny doubles each) */
} wiu_block;

/* Metrics of every block of a multi-block grid (nine planes with ghost band
 * and tag per block, as wiu_metrics; Secs. 2.2-2.4 and the scheme's central
 * operator) on the coupled coordinates described above.  X_all: device
 * coordinates at each block's off_X; M_all: output at each block's off_M;
 * work: device scratch of wiu_blocks_metrics_work_size() bytes, caller-owned.
 * Asynchronous on `stream` except that the block table is copied to `work`
 * synchronously.  Returns WIU_EINVAL for an invalid block set, scheme or
 * parameter; folded cells latch WIU_ST_JACOBIAN in the status word at the
 * start of `work` (read it with wiu_status(work, ...)). */
size_t wiu_blocks_metrics_work_size(const wiu_block* blocks, int nblocks, int scheme);
int wiu_blocks_metrics(const wiu_block* blocks, int nblocks, int scheme, const wiu_params* p, const double* X_all,
                       double* M_all, void* work, wiu_stream_t stream);

typedef struct wiu_plan wiu_plan;

/* xi_variant / eta_variant select the tile shapes (see wiu_set_tuning). */
int wiu_batched_plan(const wiu_block* blocks, int nblocks, int scheme, const wiu_params* p, int xi_variant,
                     int eta_variant, double* U_all, const double* M_all, wiu_plan** plan);
int wiu_batched_info(const wiu_plan* plan, long long* cells, int* tiles_xi, int* tiles_eta);
/* Per-block time steps: from the host (synchronous), from the CFL rule on the
 * device (Sec. 2.3 wave speeds, as wiu_cfl_dt per block), or read back. */
int wiu_batched_set_dt(wiu_plan* plan, const double* dt_host, wiu_stream_t stream);
int wiu_batched_cfl_dt(wiu_plan* plan, double cfl, wiu_stream_t stream);
int wiu_batched_get_dt(const wiu_plan* plan, double* dt_host, wiu_stream_t stream);
/* One TVD-RK3 step of every block.  use_graph != 0 replays a captured graph
 * of the step (captured on first use, bound to the plan's pointers). */
int wiu_batched_rk3_step(wiu_plan* plan, int use_graph, wiu_stream_t stream);
int wiu_batched_status(wiu_plan* plan, wiu_stream_t stream, int* status, int clear);
/* Waits for the device, then frees the plan (also when the wait fails, which
 * returns WIU_EHIP). */
int wiu_plan_destroy(wiu_plan* plan);

/* ---- Three-dimensional grids ----------------------------------------------
 * The paper's method in its general form (Sec. 2.1, Eq. 2.2): Q = (rho,
 * rho u, rho v, rho w, e), metrics in the symmetric conservative form
 * (Eq. 2.4) with each scheme's central operator in every derivative,
 * J^{-1} by Eq. 2.5, midpoint metrics by the linear interpolation of the
 * 2-D path (Sec. 2.4), the characteristic projection of Sec. 3.4 with five
 * eigenvectors along the unit direction (shear waves along t2 and t1: t1
 * the axis of the smallest component of n, ties to the later axis, made
 * orthogonal to n; t2 = t1 x n), TVD-RK3.  J^{-1} by Eq. 2.5 or Eq. 2.6
 * (wiu3_metrics).  wiu_params selects the options as in 2-D: the
 * interpolation variables (component-wise on deviations for conservative
 * or primitive (rho, u, v, w, p) variables), alpha_h of the one-midpoint
 * schemes, the weights, and the Steger-Warming or van Leer split of the
 * leading midpoint flux (the 3-D forms of the 2-D splits).
 *
 * Layouts (device, caller-owned): coordinates x, y, z and each state
 * component [nz][ny][nx], i fastest; U [5][nz][ny][nx]; M 19 planes of
 * (nx+8)(ny+8)(nz+8) doubles (ghost band 4): xi^ (x, y, z), eta^, zeta^,
 * J^{-1} at nodes, then xi^ at (i+1/2), eta^ at (j+1/2), zeta^ at (k+1/2),
 * followed by an 8-double tag; the sweeps latch WIU_ST_SCHEME and write
 * nothing if the tag does not match.  ws: wiu3_workspace_bytes() bytes
 * (status word first, read with wiu_status); zero it once with
 * wiu_workspace_init.  Directions are periodic or bounded; beyond a bounded
 * end the side's rule of wiu_grid (transmissive, reflecting wall with the
 * momentum along the boundary node's metric direction reversed, or a fixed
 * state; invalid rules or non-physical fixed states make the grid invalid),
 * coordinates extended linearly.
 * All calls are asynchronous on `stream`. */
typedef struct {
  int nx, ny, nz;
  int bc[3];            /* WIU_BC_* of x, y, z */
  double period[3];     /* periods of periodic directions */
  int side[6];          /* WIU_SIDE_TRANSMISSIVE / _WALL / _FIXED of x low .. z high (0: transmissive) */
  double fixed[6][5];   /* conservative state beyond a WIU_SIDE_FIXED side */
} wiu_grid3;

size_t wiu3_metrics_size(const wiu_grid3* g);
size_t wiu3_workspace_bytes(const wiu_grid3* g);
/* p may be NULL (alpha_h = 1); its alpha_h enters the metric operator of
 * the one-midpoint schemes as in wiu_metrics and is recorded in the tag.
 * jform: 5 for J^{-1} by Eq. 2.5, 1/3 sum_{m,l} n^_{m,l} D_m x_l, or 6 for
 * Eq. 2.6, 1/3 sum_{m,l} D_m(n^_{m,l} x_l) (the paper allows either; the
 * nine metric components are the same).  The tag records it. */
int wiu3_metrics(const wiu_grid3* g, int scheme, int jform, const wiu_params* p, const double* x, const double* y,
                 const double* z, double* M, void* ws, wiu_stream_t stream);
/* dU/dt of Eq. 2.2 (one direction pass per coordinate direction). */
int wiu3_rhs(const wiu_grid3* g, int scheme, const wiu_params* p, const double* U, const double* M, double* dUdt,
             void* ws, wiu_stream_t stream);
/* dt = cfl / max over nodes of sum_d (|U^_d| + c|k_d|) / J^{-1}, written to the device scalar dt. */
int wiu3_cfl_dt(const wiu_grid3* g, const wiu_params* p, const double* U, const double* M, double cfl, double* dt,
                void* ws, wiu_stream_t stream);
/* One TVD-RK3 step of U in place with the device scalar time step dt (Sec. 6). */
int wiu3_rk3_step(const wiu_grid3* g, int scheme, const wiu_params* p, double* U, const double* M, const double* dt,
                  void* ws, wiu_stream_t stream);
/* wiu3_cfl_dt followed by wiu3_rk3_step, sharing one pass over U for the
 * CFL maximum and the first stage's line maxima: *dt (device scalar)
 * receives the CFL time step of U, then U advances by it.  Same results as
 * the two calls.  WIU_EINVAL unless cfl > 0. */
int wiu3_rk3_step_cfl(const wiu_grid3* g, int scheme, const wiu_params* p, double* U, const double* M, double cfl,
                      double* dt, void* ws, wiu_stream_t stream);
/* nsteps (>= 1) successive wiu3_rk3_step_cfl steps of U in place (Sec. 6,
 * each at the CFL time step of the state it starts from); dt points to
 * nsteps device doubles, dt[s] receiving the size of step s.  Same results,
 * bit for bit, as nsteps wiu3_rk3_step_cfl calls: only the first step has a
 * separate pass over U for the maxima; the last stage of each step forms
 * the next step's line maxima and CFL maximum as it writes the state.
 * WIU_EINVAL unless cfl > 0 and nsteps >= 1. */
int wiu3_rk3_steps_cfl(const wiu_grid3* g, int scheme, const wiu_params* p, double* U, const double* M, double cfl,
                       int nsteps, double* dt, void* ws, wiu_stream_t stream);

/* Tile shapes of the two sweep kernels (dir 0 = xi, 1 = eta).  Several
 * shapes are compiled; the choice is process-wide and affects speed only,
 * never results.  wiu_tuning_variants() returns how many shapes a direction
 * has, wiu_set_tuning() selects one (WIU_EINVAL when out of range). */
int wiu_tuning_variants(int dir);
int wiu_set_tuning(int dir, int variant);
int wiu_get_tuning(int dir);

/* Kernel timing for benchmarks.  While enabled, every launch of the
 * library's kernels is bracketed by HIP events recorded on its launch stream.
 * wiu_profile_read() synchronises the device, returns the number of launches
 * and their mean duration in milliseconds for kernel `id` (WIU_K_*), and
 * clears that kernel's records. */
enum {
  WIU_K_WAVE_MAX = 0, WIU_K_SWEEP_XI = 1, WIU_K_SWEEP_ETA = 2, WIU_K_METRICS = 3,
  WIU_K_SWEEP3 = 4,  /* 3-D direction pass */
  WIU_K_COUNT = 5
};
int wiu_profile_enable(int on);
int wiu_profile_read(int id, long long* count, double* mean_ms);

#ifdef __cplusplus
}
#endif

#endif /* WENOIU_H */
