// ---------------------------------------------------------------------------
// WENOIU reference oracle: C entry points -- TEST INFRASTRUCTURE ONLY.
// Called from the test suite, the smoke check and the CPU-baseline leg of the
// benchmark through ctypes.  Arrays are host memory, fp64, row-major with the
// i (xi) index fastest; conservative states are [4][ny][nx] = rho, rho u,
// rho v, e.  Metric arrays follow the layout documented in the header.
// ---------------------------------------------------------------------------
#include "wenoiu_oracle.hpp"
#include "multiblock.hpp"
#include "euler3d.hpp"
#include "flop_count.hpp"
#include "ad_types.hpp"

#include <cstring>
#ifdef _OPENMP
#include <omp.h>
#endif

using namespace orc;

namespace {

// side[4] (x lo, x hi, y lo, y hi; Side values) and fixed[4][4] may be null.
Grid make_grid(int nx, int ny, int bcx, int bcy, double Lx, double Ly, const int* side = nullptr,
               const double* fixed = nullptr) {
  Grid g;
  g.nx = nx; g.ny = ny; g.bcx = (Bc)bcx; g.bcy = (Bc)bcy; g.Lx = Lx; g.Ly = Ly;
  for (int k = 0; k < 4; ++k) {
    g.side[k] = side ? side[k] : SIDE_TRANSMISSIVE;
    for (int q = 0; q < 4; ++q) g.fixed[k][q] = fixed ? fixed[4 * k + q] : 0.0;
  }
  return g;
}

Params make_params(double gamma, double alpha, double eps, int ppm, int vars = 0, double alpha_h = 1.0,
                   int weights = 0, int split = 0) {
  Params p;
  p.gamma = gamma; p.alpha_lf = alpha; p.eps = eps; p.ppm = ppm; p.vars = vars; p.alpha_h = alpha_h;
  p.weights = weights; p.split = split;
  return p;
}

bool bad_scheme(int s) { return s < 0 || s > 7; }

// Multi-block descriptors, per block: idesc[16] = nx, ny, bcx, bcy, side[4],
// nbr[4], nbr_side[4]; fdesc[26] = Lx, Ly, shift[4][2], fixed[4][4].  X_all
// holds block b's x at offX[b] and y right after it (nx ny values each).
std::vector<Block> make_blocks(int nblocks, const int* idesc, const double* fdesc, const double* X_all,
                               const long long* offX) {
  std::vector<Block> B(nblocks);
  for (int b = 0; b < nblocks; ++b) {
    const int* I = idesc + 16 * b;
    const double* F = fdesc + 26 * b;
    B[b].g = make_grid(I[0], I[1], I[2], I[3], F[0], F[1], I + 4, F + 10);
    for (int s = 0; s < 4; ++s) {
      B[b].nbr[s] = I[8 + s];
      B[b].nbr_side[s] = I[12 + s];
      B[b].shift[s][0] = F[2 + 2 * s];
      B[b].shift[s][1] = F[3 + 2 * s];
    }
    if (X_all) {
      B[b].x = X_all + offX[b];
      B[b].y = X_all + offX[b] + (long long)I[0] * I[1];
    }
  }
  return B;
}

template <class P, class Q> std::vector<P> views(int n, Q* base, const long long* off) {
  std::vector<P> v(n);
  for (int b = 0; b < n; ++b) v[b] = base + off[b];
  return v;
}

// alpha_h other than 1 exists only for the one-midpoint schemes
bool bad_options(int s, int vars, double alpha_h, int weights, int split) {
  return bad_scheme(s) || vars < 0 || vars > 2 || (alpha_h != 1.0 && !one_midpoint(s)) || !(alpha_h > 0.0) ||
         weights < 0 || weights > 1 || split < 0 || split > 2;
}

}  // namespace

extern "C" {

void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// ---- component probes (used to pin the pieces against the paper) ----------

// WENO interpolation to k+1/2.  r = 4: v[0..6] = v_{k-3..k+3}; r = 3:
// v[0..4] = v_{k-2..k+2}; r = 2: v[0..3] = v_{k-2..k+1}.
double orc_weno(int r, const double* v, double eps, int ppm, int weights) {
  Params p = make_params(1.4, 1.1, eps, ppm, 0, 1.0, weights);
  if (r == 4) return weno_r4(v, p);
  if (r == 3) return weno_r3(v, p);
  return weno_r2(v, p);
}

double orc_ppm(int order, double w, double C) {
  return order == 4 ? ppm4(w, C) : (order == 3 ? ppm3(w, C) : ppm2(w, C));
}

// r = 4 indicator of stencil k on (a, b, c, d).
double orc_is4(int k, double a, double b, double c, double d) { return is_r4(k, a, b, c, d); }

double orc_is(int k, double a, double b, double c) {
  return k == 0 ? is_left(a, b, c) : (k == 1 ? is_mid(a, b, c) : is_right(a, b, c));
}

// h^+_{i+1/2} with nodal f[0..6] = f_{i-3..i+3} and midpoint
// F[0..5] = f_{i-5/2}, ..., f_{i+5/2} (F[m + 3] = f_{i+1/2+m}).
double orc_hplus(int scheme, double alpha_h, const double* f, const double* F) {
  auto fn = [&](int m) { return f[m + 3]; };
  auto Fm = [&](int m) { return F[m + 3]; };
  return h_plus<double>((Scheme)scheme, alpha_h, fn, Fm);
}

// delta^{c,(1)} at node i with nodal g[0..8] = g_{i-4..i+4} and midpoint
// gm[0..7] = g_{i-7/2}, ..., g_{i+7/2}.
double orc_delta_c(int scheme, double alpha_h, const double* g, const double* gm) {
  auto gn = [&](int m) { return g[m + 4]; };
  auto gmm = [&](int m) { return gm[m + 4]; };
  return delta_c((Scheme)scheme, alpha_h, gn, gmm);
}

// Midpoint interpolation from g[0..5] = g_{i-2..i+3} (npts = 6) or
// g[0..7] = g_{i-3..i+4} (npts = 8).
double orc_interp_mid(int npts, const double* g) {
  if (npts == 8) return interp_mid8([&](int l) { return g[l + 3]; });
  return interp_mid6([&](int l) { return g[l + 2]; });
}

// The combined metric operator on relative values r[0..16] = g_{i-8..i+8} - g_i.
double orc_metric_derivative(int scheme, double alpha_h, const double* r) {
  return metric_derivative((Scheme)scheme, alpha_h, r);
}

// delta^{c,(1)} built by Eq. 2.7 from h+ (at any alpha_h), for comparison
// with the printed operators.
double orc_delta_c_eq27(int scheme, double alpha_h, const double* g, const double* gm) {
  auto gn = [&](int m) { return g[m + 4]; };
  auto gmm = [&](int m) { return gm[m + 4]; };
  return delta_c_eq27((Scheme)scheme, alpha_h, gn, gmm);
}

void orc_eigenvectors(const double* Q, double gamma, double nx, double ny, double* L, double* R) {
  double LL[4][4], RR[4][4];
  eigenvectors(Q, gamma, nx, ny, LL, RR);
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) { L[a * 4 + b] = LL[a][b]; R[a * 4 + b] = RR[a][b]; }
}

void orc_flux_hat(const double* Q, double gamma, double kx, double ky, double* out) {
  flux_hat(Q, gamma, kx, ky, out);
}

// Midpoint split fluxes: Qs[8][4] = Q_{k-3..k+4}; k0 = (kx,ky) at k, k1 at k+1,
// mk = midpoint metric; lam = line eigenvalue.
int orc_midpoint_flux(int scheme, double gamma, double eps, int ppm, int vars, int weights, int split,
                      const double* Qs, const double* k0, const double* k1, const double* mk, double lam, double* Fp,
                      double* Fm) {
  if (bad_options(scheme, vars, 1.0, weights, split)) return -1;
  Params p = make_params(gamma, 1.1, eps, ppm, vars, 1.0, weights, split);
  double QQ[8][4];
  std::memcpy(QQ, Qs, sizeof(QQ));
  midpoint_flux((Scheme)scheme, p, QQ, k0[0], k0[1], k1[0], k1[1], mk[0], mk[1], lam, Fp, Fm);
  return 0;
}

// ---- 2-D Euler ----------------------------------------------------------------

long long orc_metrics_size(int nx, int ny) { return 9LL * (nx + 2 * G) * (ny + 2 * G); }
int orc_ghost(void) { return G; }

int orc_metrics(int scheme, double alpha_h, int nx, int ny, int bcx, int bcy, double Lx, double Ly, const double* x,
                const double* y, double* M) {
  if (bad_options(scheme, 0, alpha_h, 0, 0) || nx < 1 || ny < 1) return -1;
  if ((bcx == TRANSMISSIVE && nx < 2) || (bcy == TRANSMISSIVE && ny < 2)) return -1;
  Grid g = make_grid(nx, ny, bcx, bcy, Lx, Ly);
  compute_metrics((Scheme)scheme, alpha_h, g, x, y, M);
  return 0;
}

int orc_rhs(int scheme, int nx, int ny, int bcx, int bcy, const int* side, const double* fixed, double gamma, double alpha, double eps, int ppm, int vars,
         double alpha_h, int weights, int split,
            const double* U, const double* M, double* dUdt, double* lam_xi, double* lam_eta) {
  if (bad_options(scheme, vars, alpha_h, weights, split) || nx < 1 || ny < 1) return -1;
  Grid g = make_grid(nx, ny, bcx, bcy, 0.0, 0.0, side, fixed);
  Params p = make_params(gamma, alpha, eps, ppm, vars, alpha_h, weights, split);
  rhs<double>((Scheme)scheme, p, g, U, M, dUdt, lam_xi, lam_eta);
  return 0;
}

double orc_cfl_dt(int nx, int ny, double gamma, const double* U, const double* M, double cfl) {
  Grid g = make_grid(nx, ny, 0, 0, 0.0, 0.0);
  Params p = make_params(gamma, 1.1, 1e-40, 1);
  return cfl_dt(p, g, U, M, cfl);
}

int orc_rk3_step(int scheme, int nx, int ny, int bcx, int bcy, const int* side, const double* fixed, double gamma, double alpha, double eps, int ppm, int vars,
         double alpha_h, int weights, int split,
                 double* U, const double* M, double dt) {
  if (bad_options(scheme, vars, alpha_h, weights, split) || nx < 1 || ny < 1) return -1;
  Grid g = make_grid(nx, ny, bcx, bcy, 0.0, 0.0, side, fixed);
  Params p = make_params(gamma, alpha, eps, ppm, vars, alpha_h, weights, split);
  rk3_step<double>((Scheme)scheme, p, g, U, M, dt);
  return 0;
}

// Run nsteps TVD-RK3 steps at fixed dt.
int orc_rk3_run(int scheme, int nx, int ny, int bcx, int bcy, const int* side, const double* fixed, double gamma, double alpha, double eps, int ppm, int vars,
         double alpha_h, int weights, int split,
                double* U, const double* M, double dt, int nsteps) {
  for (int s = 0; s < nsteps; ++s) {
    int rc = orc_rk3_step(scheme, nx, ny, bcx, bcy, side, fixed, gamma, alpha, eps, ppm, vars, alpha_h, weights, split, U, M, dt);
    if (rc) return rc;
  }
  return 0;
}

// ---- Sec. 5.1: scalar linear advection u_t + u_x = 0 ---------------------------
// Semi-discrete WENOIU operator on a periodic uniform grid of N points with
// spacing dx (Eq. 3.2).  split = 0: upwind split f+ = u, f- = 0;
// split = 1: Lax-Friedrichs split f+- = (u +- alpha u)/2.  Midpoint values
// interpolate u and form the flux from it (Sec. 2.4).
void orc_adv1d_rhs(int scheme, int N, double dx, int split, double alpha, double eps, int ppm, double alpha_h,
                   int weights, const double* u, double* dudt) {
  Params p = make_params(1.4, alpha, eps, ppm, 0, alpha_h, weights);
  Scheme sc = (Scheme)scheme;
  auto U = [&](int k) { return u[wrap(k, N)]; };
  double cp = split == 0 ? 1.0 : 0.5 * (1.0 + alpha);
  double cm = split == 0 ? 0.0 : 0.5 * (1.0 - alpha);
  std::vector<double> H(N + 1);
  for (int i = -1; i < N; ++i) {
    auto fp = [&](int m) { return cp * U(i + m); };
    auto fm = [&](int m) { return cm * U(i + 1 - m); };
    auto Fp = [&](int m) {  // f^+ at i+1/2+m
      int k = i + m;
      double s[8];
      for (int l = 0; l < 8; ++l) s[l] = U(k - 3 + l);
      return cp * weno_left(sc, s, p);
    };
    auto Fm = [&](int m) {  // f^- at i+1/2-m
      int k = i - m;
      double s[8];
      for (int l = 0; l < 8; ++l) s[l] = U(k - 3 + l);
      return cm * weno_right(sc, s, p);
    };
    H[i + 1] = h_plus<double>(sc, alpha_h, fp, Fp) + h_plus<double>(sc, alpha_h, fm, Fm);
  }
  for (int k = 0; k < N; ++k) dudt[k] = -(H[k + 1] - H[k]) / dx;
}

// Table 3 experiment: u0 = sin(pi x - sin(pi x)/pi) on [-1, 1), classical RK4
// with dt = dx^dtpow (5/4 in Table 3; 7/4 keeps RK4's error below a
// seventh-order spatial one), shortened to land on tend, errors against the
// exact translated solution.
int orc_adv1d_run(int scheme, int N, int split, double alpha, double eps, int ppm, double alpha_h, int weights,
                  double tend, double dtpow, double* l2, double* linf) {
  if (bad_options(scheme, 0, alpha_h, weights, 0) || N < 8) return -1;
  const double PI = 3.14159265358979323846;
  double dx = 2.0 / N;
  auto u0 = [&](double x) { return std::sin(PI * x - std::sin(PI * x) / PI); };
  std::vector<double> u(N), k1(N), k2(N), k3(N), k4(N), tmp(N);
  for (int i = 0; i < N; ++i) u[i] = u0(-1.0 + i * dx);
  int nsteps = (int)std::ceil(tend / std::pow(dx, dtpow) - 1e-12);
  double dt = tend / nsteps;
  for (int s = 0; s < nsteps; ++s) {
    orc_adv1d_rhs(scheme, N, dx, split, alpha, eps, ppm, alpha_h, weights, u.data(), k1.data());
    for (int i = 0; i < N; ++i) tmp[i] = u[i] + 0.5 * dt * k1[i];
    orc_adv1d_rhs(scheme, N, dx, split, alpha, eps, ppm, alpha_h, weights, tmp.data(), k2.data());
    for (int i = 0; i < N; ++i) tmp[i] = u[i] + 0.5 * dt * k2[i];
    orc_adv1d_rhs(scheme, N, dx, split, alpha, eps, ppm, alpha_h, weights, tmp.data(), k3.data());
    for (int i = 0; i < N; ++i) tmp[i] = u[i] + dt * k3[i];
    orc_adv1d_rhs(scheme, N, dx, split, alpha, eps, ppm, alpha_h, weights, tmp.data(), k4.data());
    for (int i = 0; i < N; ++i) u[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
  }
  double s2 = 0.0, smax = 0.0;
  for (int i = 0; i < N; ++i) {
    double x = -1.0 + i * dx - tend;
    x = x - 2.0 * std::floor((x + 1.0) / 2.0);
    double e = u[i] - u0(x);
    s2 += e * e;
    smax = std::max(smax, std::fabs(e));
  }
  *l2 = std::sqrt(s2 / N);
  *linf = smax;
  return 0;
}

// ---- tangents and adjoints (metrics held fixed) ------------------------------------
// Single-threaded: the reverse-mode tape is one global record.
struct SingleThread {
#ifdef _OPENMP
  int nt;
  SingleThread() : nt(omp_get_max_threads()) { omp_set_num_threads(1); }
  ~SingleThread() { omp_set_num_threads(nt); }
#endif
};

// out_val = rhs(U), out_tan = (d rhs / dU) V (forward mode).
int orc_rhs_jvp(int scheme, int nx, int ny, int bcx, int bcy, const int* side, const double* fixed, double gamma, double alpha, double eps, int ppm, int vars,
         double alpha_h, int weights, int split,
                const double* U, const double* V, const double* M, double* out_val, double* out_tan) {
  if (bad_options(scheme, vars, alpha_h, weights, split) || nx < 1 || ny < 1) return -1;
  SingleThread guard;
  Grid g = make_grid(nx, ny, bcx, bcy, 0.0, 0.0, side, fixed);
  Params p = make_params(gamma, alpha, eps, ppm, vars, alpha_h, weights, split);
  const size_t N = 4 * (size_t)nx * ny;
  std::vector<Dual> Ud(N), out(N);
  for (size_t e = 0; e < N; ++e) Ud[e] = Dual(U[e], V[e]);
  rhs<Dual>((Scheme)scheme, p, g, Ud.data(), M, out.data());
  for (size_t e = 0; e < N; ++e) { out_val[e] = out[e].v; out_tan[e] = out[e].d; }
  return 0;
}

// Ubar = (d rhs / dU)^T Gbar (reverse mode on a tape).
int orc_rhs_vjp(int scheme, int nx, int ny, int bcx, int bcy, const int* side, const double* fixed, double gamma, double alpha, double eps, int ppm, int vars,
         double alpha_h, int weights, int split,
                const double* U, const double* M, const double* Gbar, double* Ubar) {
  if (bad_options(scheme, vars, alpha_h, weights, split) || nx < 1 || ny < 1) return -1;
  SingleThread guard;
  Grid g = make_grid(nx, ny, bcx, bcy, 0.0, 0.0, side, fixed);
  Params p = make_params(gamma, alpha, eps, ppm, vars, alpha_h, weights, split);
  const size_t N = 4 * (size_t)nx * ny;
  Tape& tape = Tape::get();
  tape.clear();
  std::vector<Var> Uv(N), out(N);
  for (size_t e = 0; e < N; ++e) Uv[e] = Var::leaf(U[e]);
  rhs<Var>((Scheme)scheme, p, g, Uv.data(), M, out.data());
  tape.adj.assign(tape.nodes.size(), 0.0);
  for (size_t e = 0; e < N; ++e)
    if (out[e].id >= 0) tape.adj[out[e].id] += Gbar[e];
  tape.backward();
  for (size_t e = 0; e < N; ++e) Ubar[e] = tape.adj[Uv[e].id];
  tape.clear();
  return 0;
}

// Tangent of one TVD-RK3 step at fixed dt: (U_out, dU_out) from (U, V).
int orc_rk3_step_jvp(int scheme, int nx, int ny, int bcx, int bcy, const int* side, const double* fixed, double gamma, double alpha, double eps, int ppm, int vars,
         double alpha_h, int weights, int split,
                     const double* U, const double* V, const double* M, double dt, double* out_val,
                     double* out_tan) {
  if (bad_options(scheme, vars, alpha_h, weights, split) || nx < 1 || ny < 1) return -1;
  SingleThread guard;
  Grid g = make_grid(nx, ny, bcx, bcy, 0.0, 0.0, side, fixed);
  Params p = make_params(gamma, alpha, eps, ppm, vars, alpha_h, weights, split);
  const size_t N = 4 * (size_t)nx * ny;
  std::vector<Dual> Ud(N);
  for (size_t e = 0; e < N; ++e) Ud[e] = Dual(U[e], V[e]);
  rk3_step<Dual>((Scheme)scheme, p, g, Ud.data(), M, dt);
  for (size_t e = 0; e < N; ++e) { out_val[e] = Ud[e].v; out_tan[e] = Ud[e].d; }
  return 0;
}

// Adjoint of one TVD-RK3 step at fixed dt: Ubar_n = (dU^{n+1}/dU^n)^T Ubar_np1,
// composed from the stage adjoints:
//   U1 = U + dt L(U);  U2 = 3/4 U + 1/4 (U1 + dt L(U1));  U' = 1/3 U + 2/3 (U2 + dt L(U2))
int orc_rk3_step_vjp(int scheme, int nx, int ny, int bcx, int bcy, const int* side, const double* fixed, double gamma, double alpha, double eps, int ppm, int vars,
         double alpha_h, int weights, int split,
                     const double* U, const double* M, double dt, const double* Ubar_np1, double* Ubar_n) {
  if (bad_options(scheme, vars, alpha_h, weights, split) || nx < 1 || ny < 1) return -1;
  Grid g = make_grid(nx, ny, bcx, bcy, 0.0, 0.0, side, fixed);
  Params p = make_params(gamma, alpha, eps, ppm, vars, alpha_h, weights, split);
  const size_t N = 4 * (size_t)nx * ny;
  std::vector<double> L(N), U1(N), U2(N), w(N), a(N), u2b(N), u1b(N);
  rhs<double>((Scheme)scheme, p, g, U, M, L.data());
  for (size_t e = 0; e < N; ++e) U1[e] = U[e] + dt * L[e];
  rhs<double>((Scheme)scheme, p, g, U1.data(), M, L.data());
  for (size_t e = 0; e < N; ++e) U2[e] = 0.75 * U[e] + 0.25 * (U1[e] + dt * L[e]);
  // stage 3
  orc_rhs_vjp(scheme, nx, ny, bcx, bcy, side, fixed, gamma, alpha, eps, ppm, vars, alpha_h, weights, split, U2.data(), M, Ubar_np1, a.data());
  for (size_t e = 0; e < N; ++e) {
    u2b[e] = (2.0 / 3.0) * (Ubar_np1[e] + dt * a[e]);
    Ubar_n[e] = (1.0 / 3.0) * Ubar_np1[e];
  }
  // stage 2
  orc_rhs_vjp(scheme, nx, ny, bcx, bcy, side, fixed, gamma, alpha, eps, ppm, vars, alpha_h, weights, split, U1.data(), M, u2b.data(), a.data());
  for (size_t e = 0; e < N; ++e) {
    u1b[e] = 0.25 * (u2b[e] + dt * a[e]);
    Ubar_n[e] += 0.75 * u2b[e];
  }
  // stage 1
  orc_rhs_vjp(scheme, nx, ny, bcx, bcy, side, fixed, gamma, alpha, eps, ppm, vars, alpha_h, weights, split, U, M, u1b.data(), a.data());
  for (size_t e = 0; e < N; ++e) Ubar_n[e] += u1b[e] + dt * a[e];
  return 0;
}

// ---- operation count of one rhs evaluation ---------------------------------------
// counts[0]: xi sweep (all rows), counts[1]: eta sweep (all columns),
// counts[2]: final combination; single-threaded.
static long long g_marks[4];
static void mark(int ph) { g_marks[ph] = Counted::n(); }

int orc_count_rhs_flops(int scheme, int nx, int ny, int bcx, int bcy, const int* side, const double* fixed, double gamma, double alpha, double eps,
                        int ppm, int vars, double alpha_h, int weights, int split, const double* U, const double* M, long long* counts) {
  if (bad_options(scheme, vars, alpha_h, weights, split) || nx < 1 || ny < 1) return -1;
  Grid g = make_grid(nx, ny, bcx, bcy, 0.0, 0.0, side, fixed);
  Params p = make_params(gamma, alpha, eps, ppm, vars, alpha_h, weights, split);
  const size_t N = 4 * (size_t)nx * ny;
  std::vector<Counted> Uc(U, U + N), out(N);
#ifdef _OPENMP
  int nt = omp_get_max_threads();
  omp_set_num_threads(1);
#endif
  Counted::n() = 0;
  rhs<Counted>((Scheme)scheme, p, g, Uc.data(), M, out.data(), nullptr, nullptr, mark);
#ifdef _OPENMP
  omp_set_num_threads(nt);
#endif
  counts[0] = g_marks[0];
  counts[1] = g_marks[1] - g_marks[0];
  counts[2] = g_marks[2] - g_marks[1];
  return 0;
}

// ---- multi-block grids (multiblock.hpp) ----------------------------------
// All return 0, or -1 for an invalid scheme, option or connectivity.

int orc_mb_metrics(int scheme, double alpha_h, int nblocks, const int* idesc, const double* fdesc,
                   const double* X_all, const long long* offX, double* M_all, const long long* offM) {
  if (bad_scheme(scheme) || (alpha_h != 1.0 && !one_midpoint(scheme))) return -1;
  std::vector<Block> B = make_blocks(nblocks, idesc, fdesc, X_all, offX);
  if (!mb_valid(B)) return -1;
  for (int b = 0; b < nblocks; ++b) mb_metrics((Scheme)scheme, alpha_h, B, b, M_all + offM[b]);
  return 0;
}

int orc_mb_rhs(int scheme, int nblocks, const int* idesc, const double* fdesc, double gamma, double alpha,
               double eps, int ppm, int vars, double alpha_h, int weights, int split, const double* U_all,
               const long long* offU, const double* M_all, const long long* offM, double* out_all) {
  if (bad_options(scheme, vars, alpha_h, weights, split)) return -1;
  std::vector<Block> B = make_blocks(nblocks, idesc, fdesc, nullptr, nullptr);
  if (!mb_valid(B)) return -1;
  Params p = make_params(gamma, alpha, eps, ppm, vars, alpha_h, weights, split);
  mb_rhs<double>((Scheme)scheme, p, B, views<const double*>(nblocks, U_all, offU),
                 views<const double*>(nblocks, M_all, offM), views<double*>(nblocks, out_all, offU));
  return 0;
}

int orc_mb_rk3_step(int scheme, int nblocks, const int* idesc, const double* fdesc, double gamma, double alpha,
                    double eps, int ppm, int vars, double alpha_h, int weights, int split, double* U_all,
                    const long long* offU, const double* M_all, const long long* offM, const double* dt) {
  if (bad_options(scheme, vars, alpha_h, weights, split)) return -1;
  std::vector<Block> B = make_blocks(nblocks, idesc, fdesc, nullptr, nullptr);
  if (!mb_valid(B)) return -1;
  Params p = make_params(gamma, alpha, eps, ppm, vars, alpha_h, weights, split);
  mb_rk3_step((Scheme)scheme, p, B, views<double*>(nblocks, U_all, offU), views<const double*>(nblocks, M_all, offM),
              dt);
  return 0;
}

int orc_mb_cfl_dt(int nblocks, const int* idesc, const double* fdesc, double gamma, const double* U_all,
                  const long long* offU, const double* M_all, const long long* offM, double cfl, double* dt) {
  std::vector<Block> B = make_blocks(nblocks, idesc, fdesc, nullptr, nullptr);
  if (!mb_valid(B)) return -1;
  Params p = make_params(gamma, 1.1, 1e-40, 1);
  mb_cfl_dt(p, B, views<const double*>(nblocks, U_all, offU), views<const double*>(nblocks, M_all, offM), cfl, dt);
  return 0;
}

// ---- three-dimensional grids (euler3d.hpp) ---------------------------------
// n[3], bc[3] (0 periodic, 1 transmissive), L[3] periods; x, y, z nodes
// [nz][ny][nx]; states [5][nz][ny][nx]; metrics as MetricView3.  The paper's
// configuration only (characteristic variables, Lax-Friedrichs, alpha = 1).

namespace {
// side[6] and fixed[6][5] may be null (all transmissive)
Grid3 make_grid3(const int* n, const int* bc, const double* L, const int* side = nullptr,
                 const double* fixed = nullptr) {
  Grid3 g;
  for (int d = 0; d < 3; ++d) { g.n[d] = n[d]; g.bc[d] = (Bc)bc[d]; g.L[d] = L[d]; }
  for (int k = 0; k < 6; ++k) {
    g.side[k] = side ? side[k] : SIDE_TRANSMISSIVE;
    for (int q = 0; q < 5; ++q) g.fixed[k][q] = fixed ? fixed[5 * k + q] : 0.0;
  }
  return g;
}
const double kNoPeriod[3] = {0.0, 0.0, 0.0};  // rhs3 reads no coordinates
bool bad_grid3(const int* n, const int* bc) {
  for (int d = 0; d < 3; ++d)
    if (n[d] < 1 || bc[d] < 0 || bc[d] > 1 || (bc[d] == 1 && n[d] < 2)) return true;
  return false;
}
}  // namespace

long long orc3_metrics_size(const int* n) {
  return (long long)NPLANES3 * (n[0] + 2 * G) * (n[1] + 2 * G) * (n[2] + 2 * G);
}

int orc3_metrics(int scheme, const int* n, const int* bc, const double* L, const double* x, const double* y,
                 const double* z, double* M, int jform, double alpha_h) {
  if (bad_options(scheme, 0, alpha_h, 0, 0) || bad_grid3(n, bc) || (jform != 5 && jform != 6)) return -1;
  compute_metrics3((Scheme)scheme, make_grid3(n, bc, L), x, y, z, M, jform, alpha_h);
  return 0;
}

int orc3_rhs(int scheme, const int* n, const int* bc, const int* side, const double* fixed, double gamma,
             double alpha, double eps, int ppm, int vars, double alpha_h, int weights, int split, const double* U,
             const double* M, double* out) {
  if (bad_options(scheme, vars, alpha_h, weights, split) || bad_grid3(n, bc)) return -1;
  rhs3((Scheme)scheme, make_params(gamma, alpha, eps, ppm, vars, alpha_h, weights, split),
       make_grid3(n, bc, kNoPeriod, side, fixed), U, M, out);
  return 0;
}

double orc3_cfl_dt(const int* n, double gamma, const double* U, const double* M, double cfl) {
  const int bc[3] = {0, 0, 0};
  return cfl_dt3(make_params(gamma, 1.1, 1e-40, 1), make_grid3(n, bc, kNoPeriod), U, M, cfl);
}

int orc3_rk3_step(int scheme, const int* n, const int* bc, const int* side, const double* fixed, double gamma,
                  double alpha, double eps, int ppm, int vars, double alpha_h, int weights, int split, double* U,
                  const double* M, double dt) {
  if (bad_options(scheme, vars, alpha_h, weights, split) || bad_grid3(n, bc)) return -1;
  rk3_step3((Scheme)scheme, make_params(gamma, alpha, eps, ppm, vars, alpha_h, weights, split),
            make_grid3(n, bc, kNoPeriod, side, fixed), U, M, dt);
  return 0;
}

void orc3_eigenvectors(const double* Q, double gamma, const double* nvec, double* L, double* R) {
  double l[5][5], r[5][5];
  eigenvectors3(Q, gamma, nvec, l, r);
  for (int a = 0; a < 5; ++a)
    for (int b = 0; b < 5; ++b) { L[5 * a + b] = l[a][b]; R[5 * a + b] = r[a][b]; }
}

void orc3_flux_hat(const double* Q, double gamma, const double* k, double* out) { flux_hat3(Q, gamma, k, out); }

// Another split of the midpoint flux (split 1 Steger-Warming, 2 van Leer).
void orc3_midpoint_split(int split, double gamma, const double* Q, const double* k, int side, double* out) {
  midpoint_split3(split, gamma, Q, k, side, out);
}

// Operation counts of one 3-D grid line of n nodes (line_residual3 with the
// counting scalar), by phase: [0] line maximum, [1] nodal split fluxes
// (nodes -4 .. n+3), [2] midpoint split fluxes (midpoints -4 .. n+2),
// [3] upwind-biased combination and difference.  Q [5][n] (the ends repeat
// the boundary node), K [6][n+8] (nodal and midpoint metric of the
// direction at positions -4 .. n+3).
int orc3_count_line_flops(int scheme, int n, double gamma, const double* Q, const double* K, long long* counts) {
  if (bad_scheme(scheme) || n < 2) return -1;
  Params p = make_params(gamma, 1.1, 1e-40, 1);
  std::vector<Counted> R(5 * (size_t)n);
  auto Qf = [&](int k, int q) { return Counted(Q[(size_t)q * n + std::min(std::max(k, 0), n - 1)]); };
  auto Kf = [&](int w, int k) { return K[(size_t)w * (n + 8) + (k + 4)]; };
  Counted::n() = 0;
  line_residual3<Counted>((Scheme)scheme, p, n, Qf, Kf, R.data(), nullptr, mark);
  counts[0] = g_marks[0];
  for (int k = 1; k < 4; ++k) counts[k] = g_marks[k] - g_marks[k - 1];
  return 0;
}

}  // extern "C"
