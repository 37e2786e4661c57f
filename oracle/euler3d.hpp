// ---------------------------------------------------------------------------
// Three-dimensional Euler equations on curvilinear grids in the reference
// oracle -- TEST INFRASTRUCTURE ONLY.
//
// The paper states the method in three dimensions (Sec. 2.1, Eq. 2.2) and
// the 2-D path is its z-independent reduction.  Here:
//   * metrics in the symmetric conservative form (Eq. 2.4, all nine
//     components by cyclic permutation), every derivative the scheme's own
//     central operator in its direction (Sec. 2.3); Jacobian by Eq. 2.5;
//     midpoint metrics by the same linear interpolation as in 2-D (Sec. 2.4);
//   * Q = (rho, rho u, rho v, rho w, e), E^ = k_x E + k_y F + k_z G;
//   * the characteristic projection of Sec. 3.4 with the five eigenvectors
//     along the unit direction n; the two shear waves need a tangent basis,
//     which the paper does not fix (reading): t1 is the Cartesian axis along
//     which n has its smallest component (ties to the later axis), made
//     orthogonal to n and normalised, and t2 = t1 x n; for n in the x-y
//     plane t1 = z and t2 = (-n_y, n_x, 0), the 2-D tangent, so z-uniform data
//     reproduce the 2-D scheme;
//   * the scheme options of Secs. 2.4 and 3.2-3.3 and Sec. 7 as in 2-D:
//     interpolation in characteristic, conservative or primitive variables
//     (component-wise on deviations from the reference node), the free
//     parameter alpha of the one-midpoint families (in h+ and, through
//     Eq. 2.7, in the metric operator), Jiang-Shu (PPM-mapped) or WENO-Z
//     weights, and the Steger-Warming or van Leer split of the leading
//     midpoint flux (Sec. 7, reading as in 2-D: H gains (F~+ - F+) +
//     (F~- - F-) at its own midpoint, the other terms keep Lax-Friedrichs).
// Arrays are [c][nz][ny][nx] with i fastest.
// ---------------------------------------------------------------------------
#pragma once

#include "wenoiu_oracle.hpp"

namespace orc {

struct Grid3 {
  int n[3];
  Bc bc[3];
  double L[3];  // periods of periodic directions
  // rules beyond the sides of non-periodic directions (x lo, x hi, y lo,
  // y hi, z lo, z hi), as in 2-D: transmissive, reflecting slip wall (mirror
  // image about the boundary node, momentum along the boundary node's unit
  // metric direction reversed) or a fixed state
  int side[6] = {SIDE_TRANSMISSIVE, SIDE_TRANSMISSIVE, SIDE_TRANSMISSIVE,
                 SIDE_TRANSMISSIVE, SIDE_TRANSMISSIVE, SIDE_TRANSMISSIVE};
  double fixed[6][5] = {};
};

// Extended coordinates X_c(i, j, k) for any integers, in extended precision:
// periodic directions repeat the grid shifted by the period, transmissive
// ones extend it linearly from the last two nodes, direction by direction
// (tensor-product extension at edges and corners).
struct Coords3 {
  const Grid3& g;
  const double* x[3];
  long double ext(int c, int i, int j, int k, int d) const {
    if (d == 3) return x[c][((size_t)k * g.n[1] + j) * g.n[0] + i];
    int p[3] = {i, j, k};
    const int n = g.n[d];
    if (g.bc[d] == PERIODIC) {
      const int m = floordiv(p[d], n);
      p[d] = wrap(p[d], n);
      return ext(c, p[0], p[1], p[2], d + 1) + (c == d ? (long double)m * (long double)g.L[d] : 0.0L);
    }
    if (p[d] >= 0 && p[d] < n) return ext(c, p[0], p[1], p[2], d + 1);
    int q[3] = {p[0], p[1], p[2]}, r[3] = {p[0], p[1], p[2]};
    long double e;
    if (p[d] < 0) { q[d] = 0; r[d] = 1; e = (long double)(-p[d]); }
    else { q[d] = n - 1; r[d] = n - 2; e = (long double)(p[d] - (n - 1)); }
    const long double a = ext(c, q[0], q[1], q[2], d + 1), b = ext(c, r[0], r[1], r[2], d + 1);
    return a + e * (a - b);
  }
  long double at(int c, int i, int j, int k) const { return ext(c, i, j, k, 0); }
};

// Metric storage: 19 planes of (nx+2G)(ny+2G)(nz+2G) doubles, node (i, j, k)
// at ((k+G)(ny+2G) + j+G)(nx+2G) + i+G:
//   0-2 xi^ (x, y, z), 3-5 eta^, 6-8 zeta^, 9 J^{-1}       at nodes
//   10-12 xi^ at (i+1/2), 13-15 eta^ at (j+1/2), 16-18 zeta^ at (k+1/2)
constexpr int NPLANES3 = 19;
struct MetricView3 {
  int n[3];
  const double* M;
  size_t plane() const { return (size_t)(n[0] + 2 * G) * (n[1] + 2 * G) * (n[2] + 2 * G); }
  size_t off(int i, int j, int k) const {
    return ((size_t)(k + G) * (n[1] + 2 * G) + (j + G)) * (n[0] + 2 * G) + (i + G);
  }
  double operator()(int p, int i, int j, int k) const { return M[p * plane() + off(i, j, k)]; }
};

// A box of values over [-E, n+E) in every direction.
struct Box3 {
  int n[3], E;
  std::vector<long double> v;
  Box3(const int nn[3], int e) : E(e) {
    for (int d = 0; d < 3; ++d) n[d] = nn[d];
    v.assign((size_t)(n[0] + 2 * E) * (n[1] + 2 * E) * (n[2] + 2 * E), 0.0L);
  }
  long double& operator()(int i, int j, int k) {
    return v[((size_t)(k + E) * (n[1] + 2 * E) + (j + E)) * (n[0] + 2 * E) + (i + E)];
  }
};

inline void step3(int d, int m, int& i, int& j, int& k) {
  if (d == 0) i += m; else if (d == 1) j += m; else k += m;
}

// Fill all 19 metric planes, ghost band included.  jform selects the
// Jacobian: 5 for Eq. 2.5, J^{-1} = 1/3 sum_{m,l} n^_{m,l} D_m x_l, or 6 for
// Eq. 2.6, J^{-1} = 1/3 sum_{m,l} D_m(n^_{m,l} x_l), with x_l taken relative
// to the node (sum_m D_m n^_{m,l} = 0 holds discretely for Eq. 2.4, so the
// shift changes only the rounding).
inline void compute_metrics3(Scheme sc, const Grid3& g, const double* x, const double* y, const double* z,
                             double* M, int jform = 5, double alpha_h = 1.0) {
  Coords3 C{g, {x, y, z}};
  // nodal band for the midpoint interpolation, or for Eq. 2.6 around the
  // ghost band (the operator below is evaluated on 8 nodes each side)
  const int B = jform == 6 ? G + 8 : G + (seventh_order(sc) ? 4 : 3);
  const int EI = B + 8;                           // inner derivatives: the outer operator's reach
  // the scheme's operator along d at (i, j, k) of a function f given on nodes
  auto D = [&](int d, int i, int j, int k, auto f) {
    const long double f0 = f(i, j, k);
    double r[17];
    for (int m = -8; m <= 8; ++m) {
      int a = i, b = j, c = k;
      step3(d, m, a, b, c);
      r[m + 8] = (double)(f(a, b, c) - f0);
    }
    return (long double)metric_derivative(sc, alpha_h, r);
  };
  // inner derivatives D_d x_c on [-EI, n+EI)
  std::vector<Box3> Dx;
  for (int d = 0; d < 3; ++d)
    for (int c = 0; c < 3; ++c) Dx.emplace_back(g.n, EI);
#pragma omp parallel for schedule(static)
  for (int k = -EI; k < g.n[2] + EI; ++k)
    for (int j = -EI; j < g.n[1] + EI; ++j)
      for (int i = -EI; i < g.n[0] + EI; ++i)
        for (int d = 0; d < 3; ++d)
          for (int c = 0; c < 3; ++c)
            Dx[3 * d + c](i, j, k) = D(d, i, j, k, [&](int a, int b, int e) { return C.at(c, a, b, e); });
  // nodal metrics on [-B, n+B): for direction m with (a, b) the next two
  // directions cyclically and component l with (p, q) the next two
  // coordinates cyclically, Eq. 2.4:
  //   n^_{m,l} = 1/2 [D_b(q D_a p) - D_a(q D_b p) + D_a(p D_b q) - D_b(p D_a q)],
  // evaluated with p, q taken relative to the node (the bracket annihilates
  // constants, the operators along a and b commuting).  Periodic directions
  // evaluate at the wrapped node, so band copies equal the interior values.
  std::vector<Box3> T;
  for (int p = 0; p < 10; ++p) T.emplace_back(g.n, B);
#pragma omp parallel for schedule(static)
  for (int k = -B; k < g.n[2] + B; ++k)
    for (int j = -B; j < g.n[1] + B; ++j)
      for (int i = -B; i < g.n[0] + B; ++i) {
        int w[3] = {i, j, k};
        for (int d = 0; d < 3; ++d)
          if (g.bc[d] == PERIODIC) w[d] = wrap(w[d], g.n[d]);
        long double J = 0.0L;
        for (int m = 0; m < 3; ++m) {
          const int a = (m + 1) % 3, b = (m + 2) % 3;
          for (int l = 0; l < 3; ++l) {
            const int p = (l + 1) % 3, q = (l + 2) % 3;
            const long double p0 = C.at(p, w[0], w[1], w[2]), q0 = C.at(q, w[0], w[1], w[2]);
            auto term = [&](int outer, int cv, long double c0, int inner, int cd) {
              // D_outer((X_cv - c0) D_inner X_cd)
              Box3& Di = Dx[3 * inner + cd];
              return D(outer, w[0], w[1], w[2],
                       [&](int ii, int jj, int kk) { return (C.at(cv, ii, jj, kk) - c0) * Di(ii, jj, kk); });
            };
            const long double v = 0.5L * (term(b, q, q0, a, p) - term(a, q, q0, b, p) + term(a, p, p0, b, q) -
                                          term(b, p, p0, a, q));
            T[3 * m + l](i, j, k) = v;
            J += v * Dx[3 * m + l](w[0], w[1], w[2]);  // Eq. 2.5
          }
        }
        T[9](i, j, k) = J / 3.0L;
      }
  MetricView3 mv{{g.n[0], g.n[1], g.n[2]}, M};
  const size_t P = mv.plane();
  for (int k = -G; k < g.n[2] + G; ++k)
    for (int j = -G; j < g.n[1] + G; ++j)
      for (int i = -G; i < g.n[0] + G; ++i) {
        const size_t o = mv.off(i, j, k);
        for (int p = 0; p < 10; ++p) M[p * P + o] = (double)T[p](i, j, k);
        if (jform == 6) {
          int w[3] = {i, j, k};
          for (int d = 0; d < 3; ++d)
            if (g.bc[d] == PERIODIC) w[d] = wrap(w[d], g.n[d]);
          long double J = 0.0L;
          for (int m = 0; m < 3; ++m)
            for (int l = 0; l < 3; ++l) {
              const long double x0 = C.at(l, w[0], w[1], w[2]);
              J += D(m, w[0], w[1], w[2], [&](int a, int b, int e) {
                return T[3 * m + l](a, b, e) * (C.at(l, a, b, e) - x0);
              });
            }
          M[9 * P + o] = (double)(J / 3.0L);
        }
        for (int m = 0; m < 3; ++m)
          for (int l = 0; l < 3; ++l)
            M[(10 + 3 * m + l) * P + o] = interp_mid(sc, [&](int s) {
              int a = i, b = j, c = k;
              step3(m, s, a, b, c);
              return (double)T[3 * m + l](a, b, c);
            });
      }
}

// ===========================================================================
// Sec. 2.1 in three dimensions: pressure, contravariant flux, wave speed and
// the eigenvectors of the flux Jacobian along n (Sec. 3.4).
// ===========================================================================
template <class T> T pressure3(const T Q[5], double gam) {
  return (gam - 1.0) * (Q[4] - 0.5 * (Q[1] * Q[1] + Q[2] * Q[2] + Q[3] * Q[3]) / Q[0]);
}

template <class T> void flux_hat3(const T Q[5], double gam, const double k[3], T out[5]) {
  const T u = Q[1] / Q[0], v = Q[2] / Q[0], w = Q[3] / Q[0];
  const T p = (gam - 1.0) * (Q[4] - 0.5 * Q[0] * (u * u + v * v + w * w));
  const T U = k[0] * u + k[1] * v + k[2] * w;
  out[0] = Q[0] * U;
  out[1] = Q[1] * U + k[0] * p;
  out[2] = Q[2] * U + k[1] * p;
  out[3] = Q[3] * U + k[2] * p;
  out[4] = (Q[4] + p) * U;
}

template <class T> T wave_speed3(const T Q[5], double gam, const double k[3]) {
  const T u = Q[1] / Q[0], v = Q[2] / Q[0], w = Q[3] / Q[0];
  const T p = (gam - 1.0) * (Q[4] - 0.5 * Q[0] * (u * u + v * v + w * w));
  const T c = sqrt(gam * p / Q[0]);
  return fabs(k[0] * u + k[1] * v + k[2] * w) + c * std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
}

// Tangent basis of the unit direction n (the reading stated above).
inline void tangents3(const double n[3], double t1[3], double t2[3]) {
  int e = 2;
  for (int c = 1; c >= 0; --c)
    if (std::fabs(n[c]) < std::fabs(n[e])) e = c;
  double a[3] = {0.0, 0.0, 0.0};
  a[e] = 1.0;
  const double an = a[0] * n[0] + a[1] * n[1] + a[2] * n[2];
  for (int c = 0; c < 3; ++c) t1[c] = a[c] - an * n[c];
  const double tn = std::sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
  for (int c = 0; c < 3; ++c) t1[c] /= tn;
  t2[0] = t1[1] * n[2] - t1[2] * n[1];
  t2[1] = t1[2] * n[0] - t1[0] * n[2];
  t2[2] = t1[0] * n[1] - t1[1] * n[0];
}

// Right eigenvectors (columns) for q_n - c, q_n (entropy), q_n (shear along
// t2), q_n (shear along t1), q_n + c and the matching left eigenvectors
// (rows), b1 = (gamma-1)/c^2, b2 = b1 q^2 / 2.
template <class T> void eigenvectors3(const T Q[5], double gam, const double n[3], T L[5][5], T R[5][5]) {
  double t1[3], t2[3];
  tangents3(n, t1, t2);
  const T rho = Q[0];
  const T V[3] = {Q[1] / rho, Q[2] / rho, Q[3] / rho};
  const T q2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
  const T p = (gam - 1.0) * (Q[4] - 0.5 * rho * q2);
  const T c = sqrt(gam * p / rho);
  const T Hh = (Q[4] + p) / rho;
  const T qn = V[0] * n[0] + V[1] * n[1] + V[2] * n[2];
  const T q1 = V[0] * t1[0] + V[1] * t1[1] + V[2] * t1[2];
  const T qt = V[0] * t2[0] + V[1] * t2[1] + V[2] * t2[2];
  const T b1 = (gam - 1.0) / (c * c);
  const T b2 = 0.5 * b1 * q2;
  R[0][0] = T(1.0); R[0][1] = T(1.0); R[0][2] = T(0.0); R[0][3] = T(0.0); R[0][4] = T(1.0);
  for (int d = 0; d < 3; ++d) {
    R[1 + d][0] = V[d] - c * n[d];
    R[1 + d][1] = V[d];
    R[1 + d][2] = T(t2[d]);
    R[1 + d][3] = T(t1[d]);
    R[1 + d][4] = V[d] + c * n[d];
  }
  R[4][0] = Hh - c * qn; R[4][1] = 0.5 * q2; R[4][2] = qt; R[4][3] = q1; R[4][4] = Hh + c * qn;
  L[0][0] = 0.5 * (b2 + qn / c);
  L[1][0] = 1.0 - b2;
  L[2][0] = -qt;
  L[3][0] = -q1;
  L[4][0] = 0.5 * (b2 - qn / c);
  for (int d = 0; d < 3; ++d) {
    L[0][1 + d] = 0.5 * (-b1 * V[d] - n[d] / c);
    L[1][1 + d] = b1 * V[d];
    L[2][1 + d] = T(t2[d]);
    L[3][1 + d] = T(t1[d]);
    L[4][1 + d] = 0.5 * (-b1 * V[d] + n[d] / c);
  }
  L[0][4] = 0.5 * b1; L[1][4] = -b1; L[2][4] = T(0.0); L[3][4] = T(0.0); L[4][4] = 0.5 * b1;
}

// Another split of the midpoint flux at the interpolated state Q with the
// midpoint metric k (Sec. 7 names them; the 3-D forms of the 2-D ones):
//   split 1 (Steger-Warming): F+- = R diag(l+-) L Q along n = k/|k|,
//     l = |k| (q_n - c, q_n, q_n, q_n, q_n + c), l+- = (l +- |l|)/2;
//   split 2 (van Leer): M = q_n / c; F+ = E^, F- = 0 for M >= 1 (mirrored for
//     M <= -1), else F+- = +-|k| rho c (M +- 1)^2 / 4 (1, u + n (-q_n +- 2c)/gamma,
//     ((gamma-1) q_n +- 2c)^2 / (2(gamma^2-1)) + (q^2 - q_n^2)/2).
template <class T>
void midpoint_split3(int split, double gam, const T Q[5], const double k[3], int side, T out[5]) {
  const double kn = std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
  const double n[3] = {k[0] / kn, k[1] / kn, k[2] / kn};
  const T rho = Q[0];
  const T V[3] = {Q[1] / rho, Q[2] / rho, Q[3] / rho};
  const T p = pressure3(Q, gam);
  const T c = sqrt(gam * p / rho);
  const T qn = V[0] * n[0] + V[1] * n[1] + V[2] * n[2];
  if (split == 1) {
    T L[5][5], R[5][5];
    eigenvectors3(Q, gam, n, L, R);
    const T lam5[5] = {kn * (qn - c), kn * qn, kn * qn, kn * qn, kn * (qn + c)};
    T w[5];
    for (int a = 0; a < 5; ++a) {
      T lq = T(0.0);
      for (int b = 0; b < 5; ++b) lq = lq + L[a][b] * Q[b];
      const T part = side == 0 ? 0.5 * (lam5[a] + fabs(lam5[a])) : 0.5 * (lam5[a] - fabs(lam5[a]));
      w[a] = part * lq;
    }
    for (int a = 0; a < 5; ++a) {
      out[a] = T(0.0);
      for (int b = 0; b < 5; ++b) out[a] = out[a] + R[a][b] * w[b];
    }
    return;
  }
  const T M = qn / c;
  if ((side == 0 && T(1.0) <= M) || (side == 1 && M <= T(-1.0))) {
    flux_hat3(Q, gam, k, out);
    return;
  }
  if ((side == 0 && M <= T(-1.0)) || (side == 1 && T(1.0) <= M)) {
    for (int q = 0; q < 5; ++q) out[q] = T(0.0);
    return;
  }
  const double sg = side == 0 ? 1.0 : -1.0;
  const T fm = sg * kn * rho * c * (M + sg) * (M + sg) / 4.0;
  const T vt = -qn + sg * 2.0 * c;
  const T e2 = (gam - 1.0) * qn + sg * 2.0 * c;
  out[0] = fm;
  for (int a = 0; a < 3; ++a) out[1 + a] = fm * (V[a] + n[a] * vt / gam);
  out[4] = fm * (e2 * e2 / (2.0 * (gam * gam - 1.0)) + 0.5 * (V[0] * V[0] + V[1] * V[1] + V[2] * V[2] - qn * qn));
}

// Midpoint split fluxes F^+-_{k+1/2} (Secs. 2.3, 2.4, 3.4), as in 2-D: the
// eight states Q_{k-3..k+4}, nodal metrics at k and k+1 (their normalised
// mean is the eigenvector direction), the interpolated midpoint metric and
// the line eigenvalue; reference state Q_k for F+, Q_{k+1} for F-, projected
// deviations.
// With another split (pr.split != 0) Dalt receives (F~+ - F+) + (F~- - F-).
template <class T>
void midpoint_flux3(Scheme sc, const Params& pr, const T Qs[8][5], const double k0[3], const double k1[3],
                    const double mk[3], const T& lam, T Fp[5], T Fm[5], T* Dalt = nullptr) {
  if (Dalt)
    for (int q = 0; q < 5; ++q) Dalt[q] = T(0.0);
  double n[3] = {0.5 * (k0[0] + k1[0]), 0.5 * (k0[1] + k1[1]), 0.5 * (k0[2] + k1[2])};
  const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int d = 0; d < 3; ++d) n[d] /= nn;
  const int m0 = seventh_order(sc) ? 0 : 1, m1 = seventh_order(sc) ? 8 : 7;
  for (int side = 0; side < 2; ++side) {
    const T* Qref = Qs[3 + side];
    // the entries this side's interpolation reads, each deviation formed once
    int lo, hi;
    side_window(sc, side, lo, hi);
    T Qm[5];
    if (pr.vars == 0) {
      T L[5][5], R[5][5];
      eigenvectors3(Qref, pr.gamma, n, L, R);
      T dQ[8][5];
      for (int m = lo; m < hi; ++m)
        for (int q = 0; q < 5; ++q) dQ[m][q] = m == 3 + side ? T(0.0) : Qs[m][q] - Qref[q];
      T W[5];
      for (int c = 0; c < 5; ++c) {
        T s[8];
        for (int m = 0; m < 8; ++m) {
          s[m] = T(0.0);
          // the reference node's own deviation is zero, and so is its projection
          if (m < lo || m >= hi || m == 3 + side) continue;
          s[m] = L[c][0] * dQ[m][0];
          for (int q = 1; q < 5; ++q) s[m] = s[m] + L[c][q] * dQ[m][q];
        }
        W[c] = side == 0 ? weno_left(sc, s, pr) : weno_right(sc, s, pr);
      }
      for (int q = 0; q < 5; ++q) {
        Qm[q] = R[q][0] * W[0];
        for (int c = 1; c < 5; ++c) Qm[q] = Qm[q] + R[q][c] * W[c];
        Qm[q] = Qref[q] + Qm[q];
      }
    } else {
      // Sec. 2.4: component by component in conservative (vars 1) or
      // primitive (vars 2: rho, u, v, w, p) variables, on deviations from
      // the reference node's values
      auto prim = [&](const T Q[5], T V[5]) {
        V[0] = Q[0];
        V[1] = Q[1] / Q[0]; V[2] = Q[2] / Q[0]; V[3] = Q[3] / Q[0];
        V[4] = pressure3(Q, pr.gamma);
      };
      T V[8][5];
      for (int m = 0; m < 8; ++m) {
        if (m < m0 || m >= m1)
          for (int q = 0; q < 5; ++q) V[m][q] = T(0.0);
        else if (pr.vars == 1)
          for (int q = 0; q < 5; ++q) V[m][q] = Qs[m][q];
        else
          prim(Qs[m], V[m]);
      }
      T Vm[5];
      for (int c = 0; c < 5; ++c) {
        T s[8];
        for (int m = 0; m < 8; ++m)
          s[m] = (m < lo || m >= hi || m == 3 + side) ? T(0.0) : V[m][c] - V[3 + side][c];
        Vm[c] = V[3 + side][c] + (side == 0 ? weno_left(sc, s, pr) : weno_right(sc, s, pr));
      }
      if (pr.vars == 1) {
        for (int q = 0; q < 5; ++q) Qm[q] = Vm[q];
      } else {
        Qm[0] = Vm[0];
        for (int a = 0; a < 3; ++a) Qm[1 + a] = Vm[0] * Vm[1 + a];
        Qm[4] = Vm[4] / (pr.gamma - 1.0) + 0.5 * Vm[0] * (Vm[1] * Vm[1] + Vm[2] * Vm[2] + Vm[3] * Vm[3]);
      }
    }
    T E[5];
    flux_hat3(Qm, pr.gamma, mk, E);
    const double sgn = side == 0 ? 1.0 : -1.0;
    T* out = side == 0 ? Fp : Fm;
    for (int q = 0; q < 5; ++q) out[q] = 0.5 * (E[q] + sgn * lam * Qm[q]);
    if (Dalt && pr.split != 0) {
      T G[5];
      midpoint_split3(pr.split, pr.gamma, Qm, mk, side, G);
      for (int q = 0; q < 5; ++q) Dalt[q] = Dalt[q] + (G[q] - out[q]);
    }
  }
}

// One grid line: R_k = H_{k+1/2} - H_{k-1/2} (Eq. 3.2), the 3-D counterpart
// of line_residual.  Q(k, q): state at line index k (boundary rule applied);
// K(w, k): w = 0..2 nodal metric of this direction, 3..5 midpoint metric at
// k+1/2.  The Lax-Friedrichs eigenvalue is alpha * max over the line's nodes.
template <class T, class QF, class KF>
void line_residual3(Scheme sc, const Params& pr, int n, QF Q, KF K, T* R, T* lam_out,
                    void (*phase_end)(int) = nullptr) {
  T lam = T(0.0);
  for (int k = 0; k < n; ++k) {
    T Qk[5] = {Q(k, 0), Q(k, 1), Q(k, 2), Q(k, 3), Q(k, 4)};
    const double kk[3] = {K(0, k), K(1, k), K(2, k)};
    T s = wave_speed3(Qk, pr.gamma, kk);
    if (k == 0 || s > lam) lam = s;
  }
  lam = pr.alpha_lf * lam;
  if (lam_out) *lam_out = lam;
  if (phase_end) phase_end(0);
  const int off = 4, len = n + 8;
  std::vector<T> fp(5 * len), fm(5 * len), Fp(5 * len), Fm(5 * len);
  for (int k = -4; k < n + 4; ++k) {
    T Qk[5] = {Q(k, 0), Q(k, 1), Q(k, 2), Q(k, 3), Q(k, 4)}, E[5];
    const double kk[3] = {K(0, k), K(1, k), K(2, k)};
    flux_hat3(Qk, pr.gamma, kk, E);
    for (int q = 0; q < 5; ++q) {
      fp[q * len + k + off] = 0.5 * (E[q] + lam * Qk[q]);
      fm[q * len + k + off] = 0.5 * (E[q] - lam * Qk[q]);
    }
  }
  if (phase_end) phase_end(1);
  std::vector<T> Dv(pr.split != 0 ? 5 * len : 0);
  for (int k = -4; k < n + 3; ++k) {
    T Qs[8][5];
    for (int m = 0; m < 8; ++m)
      for (int q = 0; q < 5; ++q) Qs[m][q] = Q(k - 3 + m, q);
    const double k0[3] = {K(0, k), K(1, k), K(2, k)}, k1[3] = {K(0, k + 1), K(1, k + 1), K(2, k + 1)};
    const double mk[3] = {K(3, k), K(4, k), K(5, k)};
    T a[5], b[5], Da[5];
    midpoint_flux3(sc, pr, Qs, k0, k1, mk, lam, a, b, pr.split != 0 ? Da : nullptr);
    for (int q = 0; q < 5; ++q) { Fp[q * len + k + off] = a[q]; Fm[q * len + k + off] = b[q]; }
    if (pr.split != 0)
      for (int q = 0; q < 5; ++q) Dv[q * len + k + off] = Da[q];
  }
  if (phase_end) phase_end(2);
  std::vector<T> H(5 * (n + 1));
  for (int i = -1; i < n; ++i)
    for (int q = 0; q < 5; ++q) {
      auto fpn = [&](int m) { return fp[q * len + i + m + off]; };
      auto Fpm = [&](int m) { return Fp[q * len + i + m + off]; };
      auto fmn = [&](int m) { return fm[q * len + i + 1 - m + off]; };
      auto Fmm = [&](int m) { return Fm[q * len + i - m + off]; };
      H[q * (n + 1) + i + 1] = h_plus<T>(sc, pr.alpha_h, fpn, Fpm) + h_plus<T>(sc, pr.alpha_h, fmn, Fmm);
      if (pr.split != 0) H[q * (n + 1) + i + 1] = H[q * (n + 1) + i + 1] + Dv[q * len + i + off];
    }
  for (int k = 0; k < n; ++k)
    for (int q = 0; q < 5; ++q) R[q * n + k] = H[q * (n + 1) + k + 1] - H[q * (n + 1) + k];
  if (phase_end) phase_end(3);
}

// Eq. 2.2: dQ/dt = -[sum over the three directions of H_{+1/2} - H_{-1/2}] / J^{-1};
// beyond a transmissive end the boundary node's state.
inline void rhs3(Scheme sc, const Params& pr, const Grid3& g, const double* U, const double* M, double* dUdt) {
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const size_t NP = (size_t)nx * ny * nz;
  MetricView3 mv{{nx, ny, nz}, M};
  std::vector<double> Rs(5 * NP, 0.0);
  auto idx = [&](int i, int j, int k) { return ((size_t)k * ny + j) * nx + i; };
  for (int d = 0; d < 3; ++d) {
    const int n = g.n[d];
    const int a = (d + 1) % 3, b = (d + 2) % 3;  // the two directions across the line
#pragma omp parallel for schedule(dynamic)
    for (int lb = 0; lb < g.n[b]; ++lb)
      for (int la = 0; la < g.n[a]; ++la) {
        auto node = [&](int k, int& i, int& j, int& kk) {
          int p[3];
          p[d] = k; p[a] = la; p[b] = lb;
          i = p[0]; j = p[1]; kk = p[2];
        };
        auto at = [&](int k, int q) {
          int i, j, kz;
          node(k, i, j, kz);
          return U[q * NP + idx(i, j, kz)];
        };
        auto K = [&](int w, int k) {
          int i, j, kz;
          node(k, i, j, kz);
          return w < 3 ? mv(3 * d + w, i, j, kz) : mv(10 + 3 * d + (w - 3), i, j, kz);
        };
        auto Q = [&](int k, int q) -> double {
          if (g.bc[d] == PERIODIC) return at(wrap(k, n), q);
          if (k >= 0 && k < n) return at(k, q);
          const int sd = 2 * d + (k < 0 ? 0 : 1);
          const int kb = k < 0 ? 0 : n - 1;
          if (g.side[sd] == SIDE_FIXED) return g.fixed[sd][q];
          if (g.side[sd] == SIDE_WALL) {
            const int km = std::min(std::max(2 * kb - k, 0), n - 1);
            if (q == 0 || q == 4) return at(km, q);
            double nv[3] = {K(0, kb), K(1, kb), K(2, kb)};
            const double nn = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
            for (int c = 0; c < 3; ++c) nv[c] /= nn;
            const double mn = at(km, 1) * nv[0] + at(km, 2) * nv[1] + at(km, 3) * nv[2];
            return at(km, q) - 2.0 * mn * nv[q - 1];
          }
          return at(kb, q);
        };
        std::vector<double> R(5 * n);
        line_residual3<double>(sc, pr, n, Q, K, R.data(), nullptr);
        for (int k = 0; k < n; ++k) {
          int i, j, kz;
          node(k, i, j, kz);
          for (int q = 0; q < 5; ++q) Rs[q * NP + idx(i, j, kz)] += R[q * n + k];
        }
      }
  }
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        for (int q = 0; q < 5; ++q) dUdt[q * NP + idx(i, j, k)] = -Rs[q * NP + idx(i, j, k)] / mv(9, i, j, k);
}

// dt = CFL / max over nodes of sum_d (|U^_d| + c|k_d|) / J^{-1}.
inline double cfl_dt3(const Params& pr, const Grid3& g, const double* U, const double* M, double cfl) {
  const size_t NP = (size_t)g.n[0] * g.n[1] * g.n[2];
  MetricView3 mv{{g.n[0], g.n[1], g.n[2]}, M};
  double smax = 0.0;
  for (int k = 0; k < g.n[2]; ++k)
    for (int j = 0; j < g.n[1]; ++j)
      for (int i = 0; i < g.n[0]; ++i) {
        const size_t o = ((size_t)k * g.n[1] + j) * g.n[0] + i;
        const double Q[5] = {U[o], U[NP + o], U[2 * NP + o], U[3 * NP + o], U[4 * NP + o]};
        double s = 0.0;
        for (int d = 0; d < 3; ++d) {
          const double kk[3] = {mv(3 * d, i, j, k), mv(3 * d + 1, i, j, k), mv(3 * d + 2, i, j, k)};
          s += wave_speed3(Q, pr.gamma, kk);
        }
        s /= mv(9, i, j, k);
        if (s > smax) smax = s;
      }
  return cfl / smax;
}

// TVD-RK3 (Sec. 6), Shu-Osher form.
inline void rk3_step3(Scheme sc, const Params& pr, const Grid3& g, double* U, const double* M, double dt) {
  const size_t N = 5 * (size_t)g.n[0] * g.n[1] * g.n[2];
  std::vector<double> L(N), U1(N), U2(N);
  rhs3(sc, pr, g, U, M, L.data());
  for (size_t e = 0; e < N; ++e) U1[e] = U[e] + dt * L[e];
  rhs3(sc, pr, g, U1.data(), M, L.data());
  for (size_t e = 0; e < N; ++e) U2[e] = 0.75 * U[e] + 0.25 * (U1[e] + dt * L[e]);
  rhs3(sc, pr, g, U2.data(), M, L.data());
  for (size_t e = 0; e < N; ++e) U[e] = (1.0 / 3.0) * U[e] + (2.0 / 3.0) * (U2[e] + dt * L[e]);
}

}  // namespace orc
