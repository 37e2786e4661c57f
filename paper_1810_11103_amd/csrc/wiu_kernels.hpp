// Kernel launch interface of libwenoiu (internal to the library).
#pragma once

#include "wenoiu.h"
#include "wiu_device.hpp"

namespace wiu {

// Compiled tile shapes of the sweeps, (variant, items along a line, lines per
// workgroup); one list serves the per-grid and the batched launches.
#define WIU_XI_TILES(X) X(0, 128, 1) X(1, 256, 1) X(2, 64, 2)
#define WIU_ETA_TILES(X) X(0, 32, 4) X(1, 64, 4) X(2, 32, 8) X(3, 64, 8) X(4, 32, 16)
constexpr int WIU_N_XI_TILES = 3, WIU_N_ETA_TILES = 5;

// Arguments of one direction sweep (see sweep_kernel).
struct SweepArgs {
  Dims d;
  const double* U;                      // state the fluxes are built from
  const double* M;                      // metrics (with tag)
  const unsigned long long* lam_xi;     // raw line maxima (bit patterns)
  const unsigned long long* lam_eta;
  double gamma, alpha, eps;
  int ppm;
  int vars;                             // interpolation variables (WIU_VARS_*)
  double ah;                            // free parameter of the one-midpoint schemes
  int weights;                          // WIU_WEIGHTS_*
  int split;                            // WIU_SPLIT_* of the leading midpoint flux
  // rules beyond the sides of non-periodic directions (x lo, x hi, y lo,
  // y hi): 0 transmissive, 1 reflecting wall, 2 fixed state `fixed`,
  // 3 interface (batched blocks): ghost layer m (1 <= m < WIU_MB_REACH) of
  // line l is nbU[side][c * nbnp[side] + g0 + m gm + l gl]
  int side[4];
  double fixed[4][4];
  const double* nbU[4];
  long long nbnp[4], g0[4], gm[4], gl[4];
  // 0 (xi) write R^xi; 1 (eta) dU/dt = -(R^xi + R^eta)/J^{-1};
  // 3 (xi) write P = ca U0 + cb (U - dt R^xi/J^{-1}) into the R^xi buffer;
  // 2 (eta) RK stage U_out = P - cb dt R^eta/J^{-1}
  int mode;
  double* Rxi;                          // R^xi or P (written by xi, read by eta)
  double* out;                          // dU/dt or the new RK stage state
  const double* U0;                     // RK base state U^n
  const double* dt;                     // device scalar time step
  double ca, cb;                        // stage: ca U0 + cb (U + dt dU/dt)
  int* status;
  // eta sweep in mode 2 only: when set, the line maxima of the new stage
  // state are accumulated here (cleared beforehand) for the next stage
  unsigned long long* nlam_xi;
  unsigned long long* nlam_eta;
  // with them, when set: per eta line (column i, nx entries, cleared
  // beforehand) the CFL maximum of the new state, max over the line's nodes
  // of (s_xi + s_eta) / J^{-1} as the separate maxima pass forms it
  unsigned long long* ncfl;
};

// One block of a batched multi-block problem (device table entry).  The
// table holds element offsets; kernels add them to the base pointers they
// receive as arguments (pointers stored in memory would be generic and cost
// flat accesses).
struct BlockDev {
  Dims d;
  long long oU, oM;              // state in U_all, metrics in M_all
  long long oRxi, oU1, oU2, oDt; // R^xi / partial stage update, stage states, dt: in ws
  long long oLam, oLam2;         // two sets of line maxima (lam_xi[ny], lam_eta[nx], cfl[1]) in lam
  // sides of non-periodic directions: rule (WIU_SIDE_*), fixed states, and
  // for interfaces the neighbour block and the affine map of ghost layer m
  // on line l to the neighbour's node, g0 + m gm + l gl
  int side[4], nbr[4];
  long long g0[4], gm[4], gl[4];
  double fixed[4][4];
};

struct BatchArgs {
  const BlockDev* blocks;
  const int4* tiles;         // {block, bx, by, 0}
  int ntiles;
  int stage;                 // RK stage 0, 1, 2
  double gamma, alpha, eps;
  int ppm;
  int vars;                  // interpolation variables (WIU_VARS_*)
  double ah;                 // free parameter of the one-midpoint schemes
  int weights, split;        // WIU_WEIGHTS_*, WIU_SPLIT_*
  int* status;
  double* U_all;             // bases of the offsets in BlockDev
  const double* M_all;
  double* ws;
  unsigned long long* lam;
  int xi_mode;               // sweep mode of the xi launches (3); a kernel argument
                             // rather than a constant, which keeps the epilogue lean
};

// Arguments of the adjoint sweeps and their per-line fix-up.
struct AdjArgs {
  Dims d;
  const double* U;                      // state the residual was evaluated at
  const double* M;
  const double* Gbar;                   // adjoint of dU/dt
  double* Ubar;                         // adjoint of U (written or accumulated)
  const unsigned long long* lam_xi;     // raw line maxima of U
  const unsigned long long* lam_eta;
  double gamma, alpha, eps;
  int ppm;
  // Output: contributions are scaled by coef = coef_c * (*coef_dt, or 1);
  // the first pass (accumulate 0) writes Ubar = sum_k base_a[k] base_x[k] +
  // coef g (null base_x[k] skipped), later passes add coef g.
  int accumulate;
  double coef_c;
  const double* coef_dt;
  const double* base_x[3];
  double base_a[3];
  double* lam_part;                     // [lines][segments] eigenvalue adjoints
  int* arg_part;                        // [lines][segments] first maximal node per tile
  int* status;
  double* ghost;                        // [lines][2][6][4] off-line contributions
  // eta sweep only, when set: the xi sweep's partials and ghosts, folded
  // into the eta output (the xi direction's per-line fix-up, done in place)
  const double* x_lam_part;
  const int* x_arg_part;
  const double* x_ghost;
  int x_nseg;
};

hipError_t launch_adj_sweep(int scheme, int dir, const AdjArgs& a, hipStream_t st, bool fixup);
int adj_nseg(int dir, int n_al);
hipError_t launch_sweep(int scheme, int dir, int variant, const SweepArgs& a, hipStream_t st);
hipError_t launch_batched_sweep(int scheme, int dir, int variant, const BatchArgs& a, hipStream_t st);
hipError_t launch_batched_wave_max(const BatchArgs& a, hipStream_t st);
hipError_t launch_batched_cfl_dt(const BatchArgs& a, int nblocks, double cfl, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long* p, long long n, hipStream_t st);
void sweep_tile_shape(int dir, int variant, int& na, int& nb);
int scheme_extra(int scheme);
int sweep_variants(int dir);
hipError_t launch_wave_max(const Dims& d, const double* U, const double* M, double gam, unsigned long long* lx,
                           unsigned long long* le, unsigned long long* cfl, int* status, hipStream_t st);
hipError_t launch_metrics(const Dims& d, int scheme, double ah, const double* x, const double* y, double* M,
                          double* T, int* status, hipStream_t st);
// Central metric operator of a scheme as an antisymmetric node stencil
// sum_m d_m (g_{i+m} - g_{i-m}), m = 1..METRIC_REACH, and the width of the
// nodal-metric band the midpoint interpolation needs.
constexpr int METRIC_REACH = 7;
struct MetricStencil {
  double d[METRIC_REACH];
};
MetricStencil metric_stencil(int scheme, double a);
int metric_band(int scheme);
// Stored metrics (nodal and midpoint planes with ghost band, tag) from the
// nodal metrics T[5] on a band of width B.
hipError_t launch_metrics_band(const Dims& d, int scheme, double ah, int B, const double* T, double* M, int* status,
                               hipStream_t st);
// Maximum over each group of line maxima (lam[mem[start[g] .. start[g+1])]),
// written back to every member.
hipError_t launch_group_max(unsigned long long* lam, const int* start, const int* mem, int ngroups, hipStream_t st);
// Event-timing scope of kernel `id` (WIU_K_*) on `st` while timing is
// enabled (null otherwise); prof_close records its end.
void* prof_open(int id, hipStream_t st);
void prof_close(void* h);
hipError_t launch_cfl_dt(const unsigned long long* cfl_max, double cfl, double* dt, hipStream_t st);
// dt = cfl / max of n per-line CFL maxima
hipError_t launch_cfl_dt_lines(const unsigned long long* cfl_lines, int n, double cfl, double* dt, hipStream_t st);
hipError_t launch_lambda_out(const Dims& d, double alpha, const unsigned long long* lx, const unsigned long long* le,
                             double* ox, double* oe, hipStream_t st);
hipError_t launch_set_tag(const Dims& d, int scheme, double ah, double* M, hipStream_t st);
hipError_t launch_zero_header(int* p, int n, hipStream_t st);

}  // namespace wiu
