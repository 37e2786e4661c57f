// C ABI of libwenoiu: argument checks, workspace carving and kernel launch
// sequences.  Declarations and the documentation of every entry point are in
// include/wenoiu.h.
#include "wenoiu.h"
#include "wiu_kernels.hpp"

#include <string.h>

#include <mutex>
#include <utility>
#include <vector>

using namespace wiu;

namespace {

// ---- optional kernel timing ----------------------------------------------
struct ProfRec { int id; hipEvent_t a, b; };
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;

struct ProfScope {
  int id; hipStream_t st; hipEvent_t a = nullptr, b = nullptr; bool on;
  ProfScope(int id_, hipStream_t st_) : id(id_), st(st_) {
    on = g_prof_on && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess &&
         hipEventRecord(a, st) == hipSuccess;
    if (!on) drop();
  }
  ~ProfScope() {
    if (!on) return;
    if (hipEventRecord(b, st) != hipSuccess) {
      drop();
      return;
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.push_back({id, a, b});
  }
  // a scope that cannot be timed keeps no events
  void drop() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    a = b = nullptr;
  }
};

}  // namespace

// Timing scopes for kernels launched from other files of the library.
namespace wiu {
void* prof_open(int id, hipStream_t st) {
  if (!g_prof_on) return nullptr;
  return new ProfScope(id, st);
}
void prof_close(void* h) { delete static_cast<ProfScope*>(h); }
}  // namespace wiu

namespace {

// Tile shape of each sweep direction (index into the compiled variants).
int g_variant[2] = {0, 2};  // xi 128 x 1, eta 32 x 8 (measured at 2048^2)

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Workspace layout (byte offsets):
//   0            header: int status, padding
//   HDR          lam_xi[ny], lam_eta[nx], cfl_max[1], cfl per eta line[nx]
//                (uint64 bit patterns)
//   lam2         a second such set (maxima of an RK stage state)
//   off_scratch  R^xi[4 np], U1[4 np], U2[4 np]  -- or the metric band temp
//   then the adjoint region: Ubar2, Ubar1 (4 planes each), eigenvalue
//   partials [max lines x segments] (double) and first maximal nodes (int),
//   off-line contributions [max lines][2][6][4]
struct WsLayout {
  size_t lam, lam2, scratch, rxi, u1, u2, ub2, ub1, lpx, lpe, apx, ape, ghx, ghe, total;
};

WsLayout layout(const wiu_grid* g) {
  WsLayout L;
  const size_t np = (size_t)g->nx * g->ny;
  const int B = GHOST + 4;  // widest nodal-metric band (eight-point interpolation)
  const size_t band = 5 * (size_t)(g->nx + 2 * B) * (g->ny + 2 * B);
  const size_t plane4 = align_up(4 * np * 8);
  // a maxima set: lam_xi[ny], lam_eta[nx], cfl[1], then per eta line the
  // CFL maxima[nx] that wiu_rk3_steps_cfl accumulates in a step's last stage
  const size_t set = align_up(((size_t)2 * g->nx + g->ny + 1) * 8);
  L.lam = ALIGN;
  L.lam2 = L.lam + set;
  L.scratch = L.lam2 + set;
  L.rxi = L.scratch;
  L.u1 = L.rxi + plane4;
  L.u2 = L.u1 + plane4;
  const size_t end_rk = L.u2 + plane4;
  const size_t end_met = L.scratch + align_up(band * 8);
  L.ub2 = end_rk > end_met ? end_rk : end_met;
  L.ub1 = L.ub2 + plane4;
  const size_t lp_xi = (size_t)g->ny * adj_nseg(0, g->nx), lp_eta = (size_t)g->nx * adj_nseg(1, g->ny);
  L.lpx = L.ub1 + plane4;
  L.lpe = L.lpx + align_up(lp_xi * 8);
  L.apx = L.lpe + align_up(lp_eta * 8);
  L.ape = L.apx + align_up(lp_xi * 4);
  L.ghx = L.ape + align_up(lp_eta * 4);
  L.ghe = L.ghx + align_up((size_t)g->ny * 2 * 6 * 4 * 8);
  L.total = L.ghe + align_up((size_t)g->nx * 2 * 6 * 4 * 8);
  return L;
}

bool grid_ok(const wiu_grid* g) {
  if (!g) return false;
  if (g->nx < 1 || g->ny < 1) return false;
  if (g->bc_x < 0 || g->bc_x > 1 || g->bc_y < 0 || g->bc_y > 1) return false;
  if (g->bc_x == WIU_BC_TRANSMISSIVE && g->nx < 2) return false;
  if (g->bc_y == WIU_BC_TRANSMISSIVE && g->ny < 2) return false;
  if (g->bc_x == WIU_BC_PERIODIC && !(g->period_x > 0.0)) return false;
  if (g->bc_y == WIU_BC_PERIODIC && !(g->period_y > 0.0)) return false;
  // side rules of non-periodic directions; fixed states must be physical
  for (int k = 0; k < 4; ++k) {
    const bool periodic = (k < 2 ? g->bc_x : g->bc_y) == WIU_BC_PERIODIC;
    if (periodic) continue;
    if (g->side[k] < WIU_SIDE_TRANSMISSIVE || g->side[k] > WIU_SIDE_FIXED) return false;
    if (g->side[k] == WIU_SIDE_FIXED) {
      const double* q = g->fixed[k];
      const double rho = q[0];
      if (!(rho > 0.0) || !(rho < 1.0e300)) return false;
      const double p = q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / rho;  // (gamma - 1) p
      if (!(p > 0.0) || !(p < 1.0e300)) return false;
    }
  }
  // launch geometry limits (grid.y <= 65535 for the row-wise launches)
  if (g->ny > 65535 * 4 || g->nx > (1 << 28)) return false;
  return true;
}

bool alpha_h_ok(int scheme, double a) {
  // the free parameter exists for the one-midpoint schemes only
  return a > 0.0 && a < 1.0e300 && (a == 1.0 || scheme == WIU_3_1MP || scheme == WIU_5_1MP || scheme == WIU_7_1MP);
}

bool params_ok(const wiu_params* p) {
  return p && p->gamma > 1.0 && p->alpha_lf > 0.0 && p->eps >= 0.0 && (p->ppm == 0 || p->ppm == 1) &&
         p->vars >= WIU_VARS_CHARACTERISTIC && p->vars <= WIU_VARS_PRIMITIVE &&
         (p->weights == WIU_WEIGHTS_JS || p->weights == WIU_WEIGHTS_Z) && p->split >= WIU_SPLIT_LF &&
         p->split <= WIU_SPLIT_VL;
}

bool scheme_ok(int s) { return s >= 0 && s <= 7; }

// scheme and parameters together
bool options_ok(int s, const wiu_params* p) { return scheme_ok(s) && params_ok(p) && alpha_h_ok(s, p->alpha_h); }

// The adjoint covers the third- and fifth-order schemes with the paper's
// configuration (characteristic variables, alpha_h = 1) on periodic or
// transmissive sides.
bool adjoint_ok(int s, const wiu_params* p, const wiu_grid* g) {
  if (!(s >= 0 && s <= 3 && params_ok(p) && p->vars == WIU_VARS_CHARACTERISTIC && p->alpha_h == 1.0 &&
        p->weights == WIU_WEIGHTS_JS && p->split == WIU_SPLIT_LF))
    return false;
  for (int k = 0; k < 4; ++k)
    if ((k < 2 ? g->bc_x : g->bc_y) != WIU_BC_PERIODIC && g->side[k] != WIU_SIDE_TRANSMISSIVE) return false;
  return true;
}

Dims dims(const wiu_grid* g) {
  Dims d;
  d.nx = g->nx; d.ny = g->ny; d.bcx = g->bc_x; d.bcy = g->bc_y;
  d.mpitch = g->nx + 2 * GHOST;
  d.mplane = (long long)(g->nx + 2 * GHOST) * (g->ny + 2 * GHOST);
  d.np = (long long)g->nx * g->ny;
  d.Lx = g->period_x; d.Ly = g->period_y;
  return d;
}

struct Ws {
  int* status;
  unsigned long long *lx, *le, *cfl;
  unsigned long long *lx2, *le2;  // maxima of an RK stage state, from the previous stage
  double *rxi, *u1, *u2, *band;
  double *ub2, *ub1, *lpx, *lpe, *ghx, *ghe;  // adjoint: per direction, eigenvalue partials and ghosts
  int *apx, *ape;                            //   and first maximal nodes
};

Ws carve(const wiu_grid* g, void* ws) {
  WsLayout L = layout(g);
  char* b = (char*)ws;
  Ws w;
  w.status = (int*)b;
  w.lx = (unsigned long long*)(b + L.lam);
  w.le = w.lx + g->ny;
  w.cfl = w.le + g->nx;
  w.lx2 = (unsigned long long*)(b + L.lam2);
  w.le2 = w.lx2 + g->ny;
  w.rxi = (double*)(b + L.rxi);
  w.u1 = (double*)(b + L.u1);
  w.u2 = (double*)(b + L.u2);
  w.band = (double*)(b + L.scratch);
  w.ub2 = (double*)(b + L.ub2);
  w.ub1 = (double*)(b + L.ub1);
  w.lpx = (double*)(b + L.lpx);
  w.lpe = (double*)(b + L.lpe);
  w.apx = (int*)(b + L.apx);
  w.ape = (int*)(b + L.ape);
  w.ghx = (double*)(b + L.ghx);
  w.ghe = (double*)(b + L.ghe);
  return w;
}

// Output of a residual adjoint: Ubar = sum_k a[k] x[k] + c dt (d rhs / dU)^T Gbar
// (dt the device scalar if given, else 1; null x[k] skipped).
struct VjpOut {
  double c = 1.0;
  const double* dt = nullptr;
  const double* x[3] = {nullptr, nullptr, nullptr};
  double a[3] = {0.0, 0.0, 0.0};
};

// lam (optional): the line maxima of U (lam_xi[ny], lam_eta[nx]) from a step
// record; otherwise they are computed here.
int residual_vjp(const wiu_grid* g, int scheme, const wiu_params* p, const double* U, const double* M,
                 const double* Gbar, double* Ubar, const Ws& w, hipStream_t st, const VjpOut& vo = VjpOut(),
                 const unsigned long long* lam = nullptr) {
  Dims d = dims(g);
  if (!lam) {
    if (launch_wave_max(d, U, M, p->gamma, w.lx, w.le, w.cfl, w.status, st) != hipSuccess) return WIU_EHIP;
    lam = w.lx;
  }
  AdjArgs a;
  a.d = d; a.U = U; a.M = M; a.Gbar = Gbar; a.Ubar = Ubar; a.lam_xi = lam; a.lam_eta = lam + d.ny;
  a.gamma = p->gamma; a.alpha = p->alpha_lf; a.eps = p->eps; a.ppm = p->ppm;
  a.status = w.status;
  a.coef_c = vo.c; a.coef_dt = vo.dt;
  for (int k = 0; k < 3; ++k) { a.base_x[k] = vo.x[k]; a.base_a[k] = vo.a[k]; }
  // xi sweep: writes Ubar, its eigenvalue partials and ghost contributions
  a.lam_part = w.lpx; a.arg_part = w.apx; a.ghost = w.ghx;
  a.x_lam_part = nullptr; a.x_arg_part = nullptr; a.x_ghost = nullptr; a.x_nseg = 0;
  a.accumulate = 0;
  if (launch_adj_sweep(scheme, 0, a, st, false) != hipSuccess) return WIU_EHIP;
  // eta sweep: adds its part and, node by node, the xi fix-up; then the eta fix-up
  a.lam_part = w.lpe; a.arg_part = w.ape; a.ghost = w.ghe;
  a.x_lam_part = w.lpx; a.x_arg_part = w.apx; a.x_ghost = w.ghx; a.x_nseg = adj_nseg(0, g->nx);
  a.accumulate = 1;
  return launch_adj_sweep(scheme, 1, a, st, true) == hipSuccess ? WIU_OK : WIU_EHIP;
}

int hip_rc(hipError_t e) { return e == hipSuccess ? WIU_OK : WIU_EHIP; }

// Residual pieces shared by rhs and the RK stages: line maxima, then the xi
// sweep into R^xi, then the eta sweep with the requested epilogue.  The
// maxima are computed here unless given (lx_in/le_in, accumulated by the
// previous stage); with nlx/nle (mode 2 only) the eta sweep accumulates the
// maxima of the new stage state there.
struct Maxima {
  const unsigned long long *lx_in = nullptr, *le_in = nullptr;
  unsigned long long *nlx = nullptr, *nle = nullptr;
  unsigned long long* ncfl = nullptr;  // with nlx: per eta line CFL maxima of the new state (nlx + nx + ny + 1)
  unsigned long long* wm = nullptr;  // target of the separate pass (lx[ny], le[nx], cfl[1]); default the workspace's
};

int residual(const wiu_grid* g, int scheme, const wiu_params* p, const double* U, const double* M, const Ws& w,
             int mode, double* out, const double* U0, const double* dt, double ca, double cb, hipStream_t st,
             const Maxima& mx = Maxima()) {
  Dims d = dims(g);
  hipError_t e = hipSuccess;
  SweepArgs a;
  a.lam_xi = mx.lx_in; a.lam_eta = mx.le_in;
  if (!mx.lx_in) {
    ProfScope ps(WIU_K_WAVE_MAX, st);
    unsigned long long* lx = mx.wm ? mx.wm : w.lx;
    e = launch_wave_max(d, U, M, p->gamma, lx, lx + d.ny, lx + d.ny + d.nx, w.status, st);
    a.lam_xi = lx; a.lam_eta = lx + d.ny;
  }
  if (e != hipSuccess) return WIU_EHIP;
  a.d = d; a.U = U; a.M = M;
  a.gamma = p->gamma; a.alpha = p->alpha_lf; a.eps = p->eps; a.ppm = p->ppm;
  a.vars = p->vars; a.ah = p->alpha_h; a.weights = p->weights; a.split = p->split;
  for (int k = 0; k < 4; ++k) {
    const bool periodic = (k < 2 ? g->bc_x : g->bc_y) == WIU_BC_PERIODIC;
    a.side[k] = periodic ? WIU_SIDE_TRANSMISSIVE : g->side[k];
    for (int c = 0; c < 4; ++c) a.fixed[k][c] = g->fixed[k][c];
  }
  a.mode = mode == 2 ? 3 : 0; a.Rxi = w.rxi; a.out = out; a.U0 = U0; a.dt = dt; a.ca = ca; a.cb = cb;
  a.status = w.status;
  a.nlam_xi = nullptr; a.nlam_eta = nullptr; a.ncfl = nullptr;
  {
    ProfScope ps(WIU_K_SWEEP_XI, st);
    e = launch_sweep(scheme, 0, g_variant[0], a, st);
  }
  if (e != hipSuccess) return WIU_EHIP;
  a.mode = mode;
  if (mode == 2 && mx.nlx) {
    // one set is contiguous: lam_xi[ny], lam_eta[nx], cfl[1] (and the per-line
    // CFL maxima[nx] when they are accumulated too)
    const long long len = (long long)d.nx + d.ny + 1 + (mx.ncfl ? d.nx : 0);
    if (launch_fill_u64(mx.nlx, len, st) != hipSuccess) return WIU_EHIP;
    a.nlam_xi = mx.nlx; a.nlam_eta = mx.nle; a.ncfl = mx.ncfl;
  }
  {
    ProfScope ps(WIU_K_SWEEP_ETA, st);
    e = launch_sweep(scheme, 1, g_variant[1], a, st);
  }
  return hip_rc(e);
}

// The three Shu-Osher TVD-RK3 stages (Sec. 4.2):
//   U1 = U + dt L(U); U2 = 3/4 U + 1/4 (U1 + dt L(U1)); U <- 1/3 U + 2/3 (U2 + dt L(U2)).
// The first stage's line maxima are computed from U (or taken from a
// preceding CFL evaluation of the same state, have_max); stages 1 and 2
// accumulate the maxima of U1 and U2 in their eta sweeps.
// rec (optional, a step record): the three maxima sets go there instead of
// the workspace, U's at rec[0], U1's at rec[1], U2's at rec[2].
//
// inplace: two buffers instead of three.  The eta sweep of a stage reads
// the partial update P only at its own output node, so it may write the new
// stage state over P: stage 1 puts P and then U1 in U1's buffer, stage 2 P
// and U2 in U2's, and stage 3 its P in U1's buffer (U1 is no longer read).
int rk3_stages(const wiu_grid* g, int scheme, const wiu_params* p, double* U, const double* M, const double* dt,
               double* U1, double* U2, const Ws& w, hipStream_t st, bool have_max,
               unsigned long long* rec = nullptr, bool inplace = false) {
  const long long ns = (long long)g->nx + g->ny + 1;
  unsigned long long* m0 = rec ? rec : w.lx;              // maxima of U
  unsigned long long* mA = rec ? rec + ns : w.lx2;        // of U1
  unsigned long long* mB = rec ? rec + 2 * ns : w.lx;     // of U2
  Ws w1 = w, w2 = w, w3 = w;
  if (inplace) { w1.rxi = U1; w2.rxi = U2; w3.rxi = U1; }
  Maxima m1;
  if (have_max) { m1.lx_in = w.lx; m1.le_in = w.le; }
  m1.wm = m0;
  m1.nlx = mA; m1.nle = mA + g->ny;
  int rc = residual(g, scheme, p, U, M, w1, 2, U1, U, dt, 0.0, 1.0, st, m1);
  if (rc) return rc;
  Maxima m2;
  m2.lx_in = mA; m2.le_in = mA + g->ny; m2.nlx = mB; m2.nle = mB + g->ny;
  rc = residual(g, scheme, p, U1, M, w2, 2, U2, U, dt, 0.75, 0.25, st, m2);
  if (rc) return rc;
  Maxima m3;
  m3.lx_in = mB; m3.le_in = mB + g->ny;
  return residual(g, scheme, p, U2, M, w3, 2, U, U, dt, 1.0 / 3.0, 2.0 / 3.0, st, m3);
}

// ---- allocation-free RK3 step ------------------------------------------------
// Scratch of wiu_rk3_step_noalloc: one array per device, resident from the
// library's first use on that device until the process ends.  Host code never
// uses the array's name as an address (it is a host-side stand-in): the
// device address is taken once per device with hipGetSymbolAddress.
constexpr size_t NOALLOC_BYTES = WIU_NOALLOC_SCRATCH_BYTES;
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Layout in the scratch: two sets of line maxima, then the two stage
// buffers (P / U1 and P / U2, see rk3_stages).
struct NoallocLayout {
  size_t lam, lam2, a, b, total;
};
NoallocLayout noalloc_layout(const wiu_grid* g) {
  NoallocLayout L;
  const size_t np = (size_t)g->nx * g->ny;
  const size_t lam = align_up(((size_t)g->nx + g->ny + 1) * 8);
  L.lam = 0;
  L.lam2 = lam;
  L.a = 2 * lam;
  L.b = L.a + align_up(4 * np * 8);
  L.total = L.b + align_up(4 * np * 8);
  return L;
}

}  // namespace

static __device__ __align__(256) unsigned char scratch[WIU_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of this device's scratch (the current device), taken on
// the first call on the device; WIU_EHIP when the runtime cannot give it.
int noalloc_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return WIU_EHIP;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return WIU_EINVAL;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return WIU_EHIP;
    g_noalloc_ptr[dev] = ptr;
  }
  *out = g_noalloc_ptr[dev];
  return WIU_OK;
}

}  // namespace

extern "C" {

size_t wiu_metrics_size(const wiu_grid* g) {
  if (!grid_ok(g)) return 0;
  return (9 * (size_t)(g->nx + 2 * GHOST) * (g->ny + 2 * GHOST) + 8) * sizeof(double);
}

size_t wiu_workspace_bytes(const wiu_grid* g) {
  if (!grid_ok(g)) return 0;
  return layout(g).total;
}

int wiu_workspace_init(void* ws, wiu_stream_t stream) {
  if (!ws) return WIU_EINVAL;
  return hip_rc(launch_zero_header((int*)ws, 64, (hipStream_t)stream));
}

int wiu_metrics(const wiu_grid* g, int scheme, const wiu_params* p, const double* x, const double* y, double* M,
                void* ws, wiu_stream_t stream) {
  const double ah = p ? p->alpha_h : 1.0;
  if (!grid_ok(g) || !scheme_ok(scheme) || !alpha_h_ok(scheme, ah) || !x || !y || !M || !ws) return WIU_EINVAL;
  Ws w = carve(g, ws);
  ProfScope ps(WIU_K_METRICS, (hipStream_t)stream);
  return hip_rc(launch_metrics(dims(g), scheme, ah, x, y, M, w.band, w.status, (hipStream_t)stream));
}

int wiu_set_metrics_tag(const wiu_grid* g, int scheme, const wiu_params* p, double* M, wiu_stream_t stream) {
  const double ah = p ? p->alpha_h : 1.0;
  if (!grid_ok(g) || !scheme_ok(scheme) || !alpha_h_ok(scheme, ah) || !M) return WIU_EINVAL;
  return hip_rc(launch_set_tag(dims(g), scheme, ah, M, (hipStream_t)stream));
}

int wiu_line_eigenvalues(const wiu_grid* g, const wiu_params* p, const double* U, const double* M, double* lam_xi,
                         double* lam_eta, void* ws, wiu_stream_t stream) {
  if (!grid_ok(g) || !params_ok(p) || !U || !M || !lam_xi || !lam_eta || !ws) return WIU_EINVAL;
  Ws w = carve(g, ws);
  Dims d = dims(g);
  hipStream_t st = (hipStream_t)stream;
  if (launch_wave_max(d, U, M, p->gamma, w.lx, w.le, w.cfl, w.status, st) != hipSuccess) return WIU_EHIP;
  return hip_rc(launch_lambda_out(d, p->alpha_lf, w.lx, w.le, lam_xi, lam_eta, st));
}

int wiu_rhs(const wiu_grid* g, int scheme, const wiu_params* p, const double* U, const double* M, double* dUdt,
            void* ws, wiu_stream_t stream) {
  if (!grid_ok(g) || !options_ok(scheme, p) || !U || !M || !dUdt || !ws) return WIU_EINVAL;
  if (dUdt == U) return WIU_EINVAL;
  Ws w = carve(g, ws);
  return residual(g, scheme, p, U, M, w, 1, dUdt, U, nullptr, 0.0, 0.0, (hipStream_t)stream);
}

int wiu_cfl_dt(const wiu_grid* g, const wiu_params* p, const double* U, const double* M, double cfl, double* dt_dev,
               void* ws, wiu_stream_t stream) {
  if (!grid_ok(g) || !params_ok(p) || !U || !M || !dt_dev || !ws || !(cfl > 0.0)) return WIU_EINVAL;
  Ws w = carve(g, ws);
  hipStream_t st = (hipStream_t)stream;
  if (launch_wave_max(dims(g), U, M, p->gamma, w.lx, w.le, w.cfl, w.status, st) != hipSuccess) return WIU_EHIP;
  return hip_rc(launch_cfl_dt(w.cfl, cfl, dt_dev, st));
}

int wiu_rk3_step(const wiu_grid* g, int scheme, const wiu_params* p, double* U, const double* M,
                 const double* dt_dev, void* ws, wiu_stream_t stream) {
  if (!grid_ok(g) || !options_ok(scheme, p) || !U || !M || !dt_dev || !ws) return WIU_EINVAL;
  Ws w = carve(g, ws);
  return rk3_stages(g, scheme, p, U, M, dt_dev, w.u1, w.u2, w, (hipStream_t)stream, false);
}

int wiu_rk3_step_cfl(const wiu_grid* g, int scheme, const wiu_params* p, double* U, const double* M, double cfl,
                     double* dt_dev, void* ws, wiu_stream_t stream) {
  if (!grid_ok(g) || !options_ok(scheme, p) || !U || !M || !dt_dev || !ws || !(cfl > 0.0))
    return WIU_EINVAL;
  Ws w = carve(g, ws);
  hipStream_t st = (hipStream_t)stream;
  {
    ProfScope ps(WIU_K_WAVE_MAX, st);
    if (launch_wave_max(dims(g), U, M, p->gamma, w.lx, w.le, w.cfl, w.status, st) != hipSuccess) return WIU_EHIP;
  }
  if (launch_cfl_dt(w.cfl, cfl, dt_dev, st) != hipSuccess) return WIU_EHIP;
  return rk3_stages(g, scheme, p, U, M, dt_dev, w.u1, w.u2, w, st, true);
}

int wiu_rk3_steps_cfl(const wiu_grid* g, int scheme, const wiu_params* p, double* U, const double* M, double cfl,
                      int nsteps, double* dt_dev, void* ws, wiu_stream_t stream) {
  if (!grid_ok(g) || !options_ok(scheme, p) || !U || !M || !dt_dev || !ws || !(cfl > 0.0) || nsteps < 1)
    return WIU_EINVAL;
  Ws w = carve(g, ws);
  hipStream_t st = (hipStream_t)stream;
  const long long ny = g->ny, nxy = (long long)g->nx + g->ny;
  // two maxima sets (lam_xi[ny], lam_eta[nx], cfl[1], cfl per eta line[nx]):
  // sa holds the current state's, sb receives the next stage's; they swap
  // roles stage by stage.  The first step's come from the separate pass (one
  // CFL maximum), later steps' from the step before (per-line CFL maxima).
  unsigned long long* sa = w.lx;
  unsigned long long* sb = w.lx2;
  {
    ProfScope ps(WIU_K_WAVE_MAX, st);
    if (launch_wave_max(dims(g), U, M, p->gamma, sa, sa + ny, sa + nxy, w.status, st) != hipSuccess) return WIU_EHIP;
  }
  for (int s = 0; s < nsteps; ++s) {
    double* dt = dt_dev + s;
    if ((s == 0 ? launch_cfl_dt(sa + nxy, cfl, dt, st) : launch_cfl_dt_lines(sa + nxy + 1, g->nx, cfl, dt, st)) !=
        hipSuccess)
      return WIU_EHIP;
    Maxima m1;  // U in, U1 out
    m1.lx_in = sa; m1.le_in = sa + ny; m1.nlx = sb; m1.nle = sb + ny;
    int rc = residual(g, scheme, p, U, M, w, 2, w.u1, U, dt, 0.0, 1.0, st, m1);
    if (rc) return rc;
    Maxima m2;  // U1 in, U2 out
    m2.lx_in = sb; m2.le_in = sb + ny; m2.nlx = sa; m2.nle = sa + ny;
    rc = residual(g, scheme, p, w.u1, M, w, 2, w.u2, U, dt, 0.75, 0.25, st, m2);
    if (rc) return rc;
    Maxima m3;  // U2 in; the new state's maxima and CFL maximum out, unless last
    m3.lx_in = sa; m3.le_in = sa + ny;
    if (s + 1 < nsteps) { m3.nlx = sb; m3.nle = sb + ny; m3.ncfl = sb + nxy + 1; }
    rc = residual(g, scheme, p, w.u2, M, w, 2, U, U, dt, 1.0 / 3.0, 2.0 / 3.0, st, m3);
    if (rc) return rc;
    std::swap(sa, sb);
  }
  return WIU_OK;
}

size_t wiu_noalloc_bytes(const wiu_grid* g) {
  if (!grid_ok(g)) return 0;
  return noalloc_layout(g).total;
}

int wiu_rk3_step_noalloc(const wiu_grid* g, int scheme, const wiu_params* p, double* U, const double* M,
                         const double* dt_dev, int* status_dev, wiu_stream_t stream) {
  if (!grid_ok(g) || !options_ok(scheme, p) || !U || !M || !dt_dev || !status_dev) return WIU_EINVAL;
  const NoallocLayout L = noalloc_layout(g);
  if (L.total > NOALLOC_BYTES) return WIU_EINVAL;  // beyond the scratch, checked before any device call
  void* base = nullptr;
  if (const int rc = noalloc_scratch(&base)) return rc;
  char* b = (char*)base;
  Ws w{};
  w.status = status_dev;
  w.lx = (unsigned long long*)(b + L.lam);
  w.le = w.lx + g->ny;
  w.cfl = w.le + g->nx;
  w.lx2 = (unsigned long long*)(b + L.lam2);
  w.le2 = w.lx2 + g->ny;
  double* A = (double*)(b + L.a);
  double* B = (double*)(b + L.b);
  // every maxima set is cleared by a fill kernel before it is accumulated,
  // and both stage buffers are written before they are read
  return rk3_stages(g, scheme, p, U, M, dt_dev, A, B, w, (hipStream_t)stream, false, nullptr, true);
}

int wiu_rhs_vjp(const wiu_grid* g, int scheme, const wiu_params* p, const double* U, const double* M,
                const double* Gbar, double* Ubar, void* ws, wiu_stream_t stream) {
  if (!grid_ok(g) || !adjoint_ok(scheme, p, g) || !U || !M || !Gbar || !Ubar || !ws)
    return WIU_EINVAL;
  if (Ubar == U || Ubar == Gbar) return WIU_EINVAL;
  Ws w = carve(g, ws);
  return residual_vjp(g, scheme, p, U, M, Gbar, Ubar, w, (hipStream_t)stream);
}

size_t wiu_step_record_bytes(const wiu_grid* g) {
  if (!grid_ok(g)) return 0;
  return 3 * ((size_t)g->nx + g->ny + 1) * sizeof(unsigned long long);
}

int wiu_rk3_step_stages(const wiu_grid* g, int scheme, const wiu_params* p, double* U, const double* M,
                        const double* dt_dev, double* U1, double* U2, void* rec, void* ws, wiu_stream_t stream) {
  if (!grid_ok(g) || !options_ok(scheme, p) || !U || !M || !dt_dev || !U1 || !U2 || !ws)
    return WIU_EINVAL;
  Ws w = carve(g, ws);
  return rk3_stages(g, scheme, p, U, M, dt_dev, U1, U2, w, (hipStream_t)stream, false, (unsigned long long*)rec);
}

int wiu_rk3_steps_stages(const wiu_grid* g, int scheme, const wiu_params* p, double* U, const double* M,
                         const double* dt_dev, int nsteps, double* stages, void* recs, void* ws, wiu_stream_t stream) {
  if (!grid_ok(g) || !options_ok(scheme, p) || !U || !M || !dt_dev || nsteps < 1 || !stages || !recs || !ws)
    return WIU_EINVAL;
  Ws w = carve(g, ws);
  hipStream_t st = (hipStream_t)stream;
  const long long ny = g->ny, ns = (long long)g->nx + g->ny + 1;
  const size_t plane4 = (size_t)4 * g->nx * g->ny;
  unsigned long long* r = (unsigned long long*)recs;
  // the first step's maxima of U from a separate pass, into its record;
  // later steps' from the last stage of the step before
  {
    ProfScope ps(WIU_K_WAVE_MAX, st);
    if (launch_wave_max(dims(g), U, M, p->gamma, r, r + ny, r + ns - 1, w.status, st) != hipSuccess) return WIU_EHIP;
  }
  for (int s = 0; s < nsteps; ++s) {
    double* S0 = stages + (size_t)s * 3 * plane4;
    double* S1 = S0 + plane4;
    double* S2 = S1 + plane4;
    unsigned long long* rs = r + (long long)s * 3 * ns;
    if (hipMemcpyAsync(S0, U, plane4 * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess) return WIU_EHIP;
    Maxima m1;  // U in, U1 out
    m1.lx_in = rs; m1.le_in = rs + ny; m1.nlx = rs + ns; m1.nle = rs + ns + ny;
    int rc = residual(g, scheme, p, U, M, w, 2, S1, U, dt_dev, 0.0, 1.0, st, m1);
    if (rc) return rc;
    Maxima m2;  // U1 in, U2 out
    m2.lx_in = rs + ns; m2.le_in = rs + ns + ny; m2.nlx = rs + 2 * ns; m2.nle = rs + 2 * ns + ny;
    rc = residual(g, scheme, p, S1, M, w, 2, S2, U, dt_dev, 0.75, 0.25, st, m2);
    if (rc) return rc;
    Maxima m3;  // U2 in; the new state's maxima into the next step's record
    m3.lx_in = rs + 2 * ns; m3.le_in = rs + 2 * ns + ny;
    if (s + 1 < nsteps) { m3.nlx = rs + 3 * ns; m3.nle = rs + 3 * ns + ny; }
    rc = residual(g, scheme, p, S2, M, w, 2, U, U, dt_dev, 1.0 / 3.0, 2.0 / 3.0, st, m3);
    if (rc) return rc;
  }
  return WIU_OK;
}

int wiu_rk3_step_vjp(const wiu_grid* g, int scheme, const wiu_params* p, const double* U_n, const double* U1,
                     const double* U2, const void* rec, const double* M, const double* dt_dev,
                     const double* Ubar_np1, double* Ubar_n, void* ws, wiu_stream_t stream) {
  if (!grid_ok(g) || !adjoint_ok(scheme, p, g) || !U_n || !M || !dt_dev || !Ubar_np1 || !Ubar_n ||
      !ws)
    return WIU_EINVAL;
  if ((U1 == nullptr) != (U2 == nullptr)) return WIU_EINVAL;
  if (rec && !U1) return WIU_EINVAL;
  const long long ns = (long long)g->nx + g->ny + 1;
  const unsigned long long* r = (const unsigned long long*)rec;
  Ws w = carve(g, ws);
  hipStream_t st = (hipStream_t)stream;
  int rc;
  if (!U1) {  // recompute the stage states
    Maxima m1, m2;
    m1.nlx = w.lx2; m1.nle = w.le2;
    m2.lx_in = w.lx2; m2.le_in = w.le2;
    rc = residual(g, scheme, p, U_n, M, w, 2, w.u1, U_n, dt_dev, 0.0, 1.0, st, m1);
    if (rc) return rc;
    rc = residual(g, scheme, p, w.u1, M, w, 2, w.u2, U_n, dt_dev, 0.75, 0.25, st, m2);
    if (rc) return rc;
    U1 = w.u1;
    U2 = w.u2;
  }
  // U' = 1/3 U + 2/3 (U2 + dt L(U2)):  Ubar2 = 2/3 Ubar' + 2/3 dt L'(U2)^T Ubar'
  VjpOut o2;
  o2.c = 2.0 / 3.0; o2.dt = dt_dev; o2.x[0] = Ubar_np1; o2.a[0] = 2.0 / 3.0;
  if ((rc = residual_vjp(g, scheme, p, U2, M, Ubar_np1, w.ub2, w, st, o2, r ? r + 2 * ns : nullptr))) return rc;
  // U2 = 3/4 U + 1/4 (U1 + dt L(U1)):  Ubar1 = 1/4 Ubar2 + 1/4 dt L'(U1)^T Ubar2
  VjpOut o1;
  o1.c = 0.25; o1.dt = dt_dev; o1.x[0] = w.ub2; o1.a[0] = 0.25;
  if ((rc = residual_vjp(g, scheme, p, U1, M, w.ub2, w.ub1, w, st, o1, r ? r + ns : nullptr))) return rc;
  // U1 = U + dt L(U), and the direct U terms of U' and U2:
  //   Ubar_n = 1/3 Ubar' + 3/4 Ubar2 + Ubar1 + dt L'(U)^T Ubar1
  // (elementwise in Ubar', so Ubar_n may alias it)
  VjpOut o0;
  o0.c = 1.0; o0.dt = dt_dev;
  o0.x[0] = Ubar_np1; o0.a[0] = 1.0 / 3.0;
  o0.x[1] = w.ub2; o0.a[1] = 0.75;
  o0.x[2] = w.ub1; o0.a[2] = 1.0;
  return residual_vjp(g, scheme, p, U_n, M, w.ub1, Ubar_n, w, st, o0, r);
}

int wiu_status(void* ws, wiu_stream_t stream, int* status, int clear) {
  if (!ws || !status) return WIU_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (hipStreamSynchronize(st) != hipSuccess) return WIU_EHIP;
  int v = 0;
  if (hipMemcpy(&v, ws, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return WIU_EHIP;
  *status = v;
  if (clear) {
    if (launch_zero_header((int*)ws, 1, st) != hipSuccess) return WIU_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) return WIU_EHIP;
  }
  return WIU_OK;
}

int wiu_tuning_variants(int dir) { return (dir == 0 || dir == 1) ? sweep_variants(dir) : WIU_EINVAL; }

int wiu_set_tuning(int dir, int variant) {
  if ((dir != 0 && dir != 1) || variant < 0 || variant >= sweep_variants(dir)) return WIU_EINVAL;
  g_variant[dir] = variant;
  return WIU_OK;
}

int wiu_get_tuning(int dir) { return (dir == 0 || dir == 1) ? g_variant[dir] : WIU_EINVAL; }

int wiu_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  return WIU_OK;
}

int wiu_profile_read(int id, long long* count, double* mean_ms) {
  if (id < 0 || id >= WIU_K_COUNT || !count || !mean_ms) return WIU_EINVAL;
  if (hipDeviceSynchronize() != hipSuccess) return WIU_EHIP;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  long long n = 0;
  double tot = 0.0;
  std::vector<ProfRec> keep;
  for (auto& r : g_prof) {
    if (r.id != id) { keep.push_back(r); continue; }
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) { tot += ms; ++n; }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.swap(keep);
  *count = n;
  *mean_ms = n ? tot / n : 0.0;
  return WIU_OK;
}

const char* wiu_strerror(int code) {
  switch (code) {
    case WIU_OK: return "ok";
    case WIU_EINVAL: return "invalid argument";
    case WIU_EHIP: return "HIP runtime or launch failure";
    default: return "unknown error";
  }
}

}  // extern "C"
