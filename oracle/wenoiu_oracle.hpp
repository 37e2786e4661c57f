// ---------------------------------------------------------------------------
// WENOIU reference oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, scalar CPU implementation of the WENO interpolation-based,
// upwind-biased (WENOIU) schemes of Li & Sun, "WENO interpolation-based and
// upwind-biased schemes with free-stream preservation" (arXiv 1810.11103),
// applied to the 2-D Euler equations in curvilinear coordinates.
//
// Only the test suite, the smoke check and the CPU-baseline leg of the
// benchmark may call this code.  It shares no source with the HIP library and
// must never be used as a fallback for it.  Every step follows the paper's
// order; where the paper is silent the reading adopted is stated at the spot.
//
// Everything is templated on the scalar type T of the flow state so that the
// same code yields forward values (T = double), tangents (dual numbers) and
// adjoints (a tape).  Grid coordinates and metrics are plain doubles.
// ---------------------------------------------------------------------------
#pragma once

#include <cmath>
#include <cstdint>
#include <functional>
#include <vector>
#include <algorithm>

namespace orc {

enum Scheme { W3_1MP = 0, W3_2MP = 1, W5_1MP = 2, W5_2MP = 3, W7_1MP = 4, W7_2MP = 5, W7_4MP = 6, W7_6MP = 7 };
enum Bc { PERIODIC = 0, TRANSMISSIVE = 1 };

// Width of the metric ghost band stored around the grid (each side).
constexpr int G = 4;

struct Params {
  double gamma = 1.4;     // ratio of specific heats (Sec. 6.3(1))
  double alpha_lf = 1.1;  // alpha of the Lax-Friedrichs eigenvalue, 1.1-1.2 (Sec. 2.3)
  double eps = 1e-40;     // WENO epsilon when the PPM mapping is used (Sec. 3.2(3))
  int ppm = 1;            // apply the piecewise-polynomial mapping (Eqs. 3.15/3.23)
  // Variables the midpoint values are interpolated in (Sec. 2.4): 0
  // characteristic (the paper's choice, Sec. 3.4), 1 conservative, 2 primitive.
  int vars = 0;
  // Free parameter alpha of the one-midpoint families (Eqs. 3.5, 3.17 and
  // Appendix (1)); the paper tests alpha = 1 only.  Other schemes require 1.
  double alpha_h = 1.0;
  // Nonlinear weights: 0 Jiang-Shu (Eqs. 3.12-3.13, the paper's), 1 WENO-Z
  // (named in Sec. 7 as a possible alternative).
  int weights = 0;
  // Splitting of the midpoint flux: 0 Lax-Friedrichs with the line
  // eigenvalue (Sec. 2.3, the paper's), 1 Steger-Warming, 2 van Leer (named
  // in Sec. 7 as possible alternatives for the midpoint flux only).
  int split = 0;
};

inline bool one_midpoint(int s) { return s == 0 || s == 2 || s == 4; }

inline bool fifth_order(Scheme s) { return s == W5_1MP || s == W5_2MP; }
inline bool seventh_order(Scheme s) { return s >= W7_1MP; }
inline bool two_midpoints(Scheme s) { return s == W3_2MP || s == W5_2MP; }

// Overloads that AD scalar types also provide.
using std::sqrt;
using std::fabs;

// ===========================================================================
// Sec. 3.2(3), Eqs. 3.10-3.15 and Sec. 3.3(3), Eqs. 3.22-3.23, Table 1:
// WENO interpolation of a nodal sequence to the midpoint x_{k+1/2}.
// ===========================================================================

// Smoothness indicators of Eq. 3.22 on the three-point stencil (a, b, c).
// Eq. 3.22 prints them as quadratic forms; the same forms written as sums of
// squares (the Jiang-Shu indicators, 13/12 (a-2b+c)^2 + 1/4 (...)^2) are used
// here because they cannot turn negative through rounding.  The equality of
// the two is checked by the test suite against the printed coefficients.
template <class T> T is_left(const T& a, const T& b, const T& c) {   // IS_0
  T d2 = a - 2.0 * b + c, d1 = a - 4.0 * b + 3.0 * c;
  return (13.0 / 12.0) * d2 * d2 + 0.25 * d1 * d1;
}
template <class T> T is_mid(const T& a, const T& b, const T& c) {    // IS_1
  T d2 = a - 2.0 * b + c, d1 = a - c;
  return (13.0 / 12.0) * d2 * d2 + 0.25 * d1 * d1;
}
template <class T> T is_right(const T& a, const T& b, const T& c) {  // IS_2
  T d2 = a - 2.0 * b + c, d1 = 3.0 * a - 4.0 * b + c;
  return (13.0 / 12.0) * d2 * d2 + 0.25 * d1 * d1;
}

// Second-order piecewise-polynomial mapping, Eq. 3.15.
template <class T> T ppm2(const T& w, double C) {
  if (w <= C) { T t = w / C - 1.0; return C * (1.0 - t * t); }
  T d = w - C;
  return C - d * d / (C - 1.0);
}
// Third-order piecewise-polynomial mapping, Eq. 3.23.
template <class T> T ppm3(const T& w, double C) {
  if (w <= C) { T t = w / C - 1.0; return C * (1.0 + t * t * t); }
  T d = w - C;
  return C + d * d * d / ((C - 1.0) * (C - 1.0));
}

// Nonlinear weights from the indicators IS_k and linear weights C_k.
//   weights 0: Eqs. 3.12-3.13, alpha_k = C_k / (eps + IS_k)^2, w = alpha /
//     sum alpha; with the mapping (ppm), g_k = map(w_k; C_k) re-normalised.
//   weights 1 (WENO-Z; Sec. 7 names it, gives no details; reading): alpha_k =
//     C_k (1 + (tau / (eps + IS_k))^2) with the global indicator tau passed
//     in, w = alpha / sum alpha, no mapping.
template <class T, int N, class Map>
void nonlinear_weights(const T (&IS)[N], const double (&C)[N], const T& tau, const Params& pr, Map map, T (&w)[N]) {
  T a[N], sa = T(0.0);
  for (int k = 0; k < N; ++k) {
    T d = pr.eps + IS[k];
    if (pr.weights == 1) {
      T q = tau / d;
      a[k] = C[k] * (1.0 + q * q);
    } else {
      a[k] = C[k] / (d * d);
    }
    sa = sa + a[k];
  }
  for (int k = 0; k < N; ++k) w[k] = a[k] / sa;
  if (pr.weights == 0 && pr.ppm) {
    T g[N], sg = T(0.0);
    for (int k = 0; k < N; ++k) { g[k] = map(w[k], C[k]); sg = sg + g[k]; }
    for (int k = 0; k < N; ++k) w[k] = g[k] / sg;
  }
}

// r = 3 (fifth-order schemes).  v[0..4] = v_{k-2}, ..., v_{k+2}; returns the
// left-biased value at k+1/2.  Candidates p_k^3 from Eq. 3.11 with the b_{k,l}
// of Table 1, linear weights C = (1, 10, 5)/16, weights Eqs. 3.12-3.13,
// indicators Eq. 3.22, mapping Eq. 3.23 followed by re-normalisation.
template <class T> T weno_r3(const T v[5], const Params& pr) {
  const double C[3] = {1.0 / 16.0, 10.0 / 16.0, 5.0 / 16.0};
  T p[3];
  p[0] = (3.0 / 8.0) * v[0] - (10.0 / 8.0) * v[1] + (15.0 / 8.0) * v[2];
  p[1] = (-1.0 / 8.0) * v[1] + (6.0 / 8.0) * v[2] + (3.0 / 8.0) * v[3];
  p[2] = (3.0 / 8.0) * v[2] + (6.0 / 8.0) * v[3] - (1.0 / 8.0) * v[4];
  T IS[3] = {is_left(v[0], v[1], v[2]), is_mid(v[1], v[2], v[3]), is_right(v[2], v[3], v[4])};
  T w[3];
  // WENO-Z global indicator for r = 3: |IS_0 - IS_2|
  nonlinear_weights(IS, C, fabs(IS[0] - IS[2]), pr, [](const T& x, double c) { return ppm3(x, c); }, w);
  return w[0] * p[0] + w[1] * p[1] + w[2] * p[2];
}

// r = 2 (third-order schemes).  v[0..3] = v_{k-2}, ..., v_{k+1}.  Candidates
// from Table 1 (C = (1, 3)/4); the indicators are IS_0 and IS_1 of Eq. 3.22 on
// the three-point stencils {k-2,k-1,k} and {k-1,k,k+1} in place of Eq. 3.14,
// as Sec. 5.1 prescribes for the third-order schemes; mapping Eq. 3.15.
template <class T> T weno_r2(const T v[4], const Params& pr) {
  const double C[2] = {1.0 / 4.0, 3.0 / 4.0};
  T p[2];
  p[0] = (-1.0 / 2.0) * v[1] + (3.0 / 2.0) * v[2];
  p[1] = (1.0 / 2.0) * v[2] + (1.0 / 2.0) * v[3];
  T IS[2] = {is_left(v[0], v[1], v[2]), is_mid(v[1], v[2], v[3])};
  T w[2];
  // WENO-Z global indicator for r = 2: |IS_0 - IS_1|
  nonlinear_weights(IS, C, fabs(IS[0] - IS[1]), pr, [](const T& x, double c) { return ppm2(x, c); }, w);
  return w[0] * p[0] + w[1] * p[1];
}

// Fourth-order piecewise-polynomial mapping (Appendix), for r = 4.
template <class T> T ppm4(const T& w, double C) {
  if (w <= C) { T t = w / C - 1.0; T t2 = t * t; return C * (1.0 - t2 * t2); }
  T d = w - C; T d2 = d * d;
  return C - d2 * d2 / ((C - 1.0) * (C - 1.0) * (C - 1.0));
}

// Smoothness indicators for r = 4 on the four-point stencil (a, b, c, d)
// counted from the left: the paper gives none; the Jiang-Shu definition that
// yields the printed r = 3 ones (Eqs. 3.14, 3.22) gives these quadratic forms
// (coefficients / 240), derived exactly by oracle/derive_weno_is.py and
// re-derived by the test suite.  k is the stencil's position (0: leftmost).
template <class T> T is_r4(int k, const T& a, const T& b, const T& c, const T& d) {
  static const double Q[4][10] = {
      // a^2, ab, ac, ad, b^2, bc, bd, c^2, cd, d^2 (cross terms doubled)
      {547, -3882, 4642, -1854, 7043, -17246, 7042, 11003, -9402, 2107},
      {267, -1642, 1602, -494, 2843, -5966, 1922, 3443, -2522, 547},
      {547, -2522, 1922, -494, 3443, -5966, 1602, 2843, -1642, 267},
      {2107, -9402, 7042, -1854, 11003, -17246, 4642, 7043, -3882, 547}};
  const double* q = Q[k];
  T s = a * (q[0] * a + q[1] * b + q[2] * c + q[3] * d) + b * (q[4] * b + q[5] * c + q[6] * d) +
        c * (q[7] * c + q[8] * d) + q[9] * d * d;
  return s / 240.0;
}

// r = 4 (seventh-order schemes, Appendix).  v[0..6] = v_{k-3}, ..., v_{k+3};
// left-biased value at k+1/2.  Candidates and linear weights of Table A1
// (C = (1, 21, 35, 7)/64), weights Eqs. 3.12-3.13, indicators is_r4, the
// fourth-order mapping followed by re-normalisation.
template <class T> T weno_r4(const T v[7], const Params& pr) {
  const double C[4] = {1.0 / 64.0, 21.0 / 64.0, 35.0 / 64.0, 7.0 / 64.0};
  T p[4];
  p[0] = (-5.0 * v[0] + 21.0 * v[1] - 35.0 * v[2] + 35.0 * v[3]) / 16.0;
  p[1] = (1.0 * v[1] - 5.0 * v[2] + 15.0 * v[3] + 5.0 * v[4]) / 16.0;
  p[2] = (-1.0 * v[2] + 9.0 * v[3] + 9.0 * v[4] - 1.0 * v[5]) / 16.0;
  p[3] = (5.0 * v[3] + 15.0 * v[4] - 5.0 * v[5] + 1.0 * v[6]) / 16.0;
  T IS[4];
  for (int k = 0; k < 4; ++k) IS[k] = is_r4(k, v[k], v[k + 1], v[k + 2], v[k + 3]);
  T w[4];
  // WENO-Z global indicator for r = 4: |IS_0 + 3 IS_1 - 3 IS_2 - IS_3|
  nonlinear_weights(IS, C, fabs(IS[0] + 3.0 * IS[1] - 3.0 * IS[2] - IS[3]), pr,
                    [](const T& x, double c) { return ppm4(x, c); }, w);
  return w[0] * p[0] + w[1] * p[1] + w[2] * p[2] + w[3] * p[3];
}

// Left-biased value at k+1/2 from the window s[0..7] = v_{k-3..k+4}.
template <class T> T weno_left(Scheme sc, const T s[8], const Params& pr) {
  if (seventh_order(sc)) return weno_r4(s, pr);
  if (fifth_order(sc)) return weno_r3(s + 1, pr);
  return weno_r2(s + 1, pr);
}
// Right-biased value at k+1/2: the same interpolation applied to the sequence
// mirrored about k+1/2, i.e. v_{k+4}, v_{k+3}, ..., v_{k-3}.
template <class T> T weno_right(Scheme sc, const T s[8], const Params& pr) {
  T m[8];
  for (int i = 0; i < 8; ++i) m[i] = s[7 - i];
  return weno_left(sc, m, pr);
}

// Window entries [lo, hi) of Q_{k-3..k+4} that the interpolation of one side
// reads: k-2..k+2 (r = 3), k-2..k+1 (r = 2), k-3..k+3 (r = 4) for the
// left-biased side, the mirror images about k+1/2 for the right-biased one.
inline void side_window(Scheme sc, int side, int& lo, int& hi) {
  const int r4 = seventh_order(sc), r3 = fifth_order(sc);
  if (side == 0) { lo = r4 ? 0 : 1; hi = r4 ? 7 : (r3 ? 6 : 5); }
  else { lo = r4 ? 1 : (r3 ? 2 : 3); hi = r4 ? 8 : 7; }
}

// ===========================================================================
// Sec. 3.2 / 3.3: upwind-biased numerical flux h^+_{i+1/2} from nodal values
// f(m) = f_{i+m} and midpoint values F(m) = f_{i+1/2+m}, with alpha = 1
// (the only member of the families 3.5 / 3.17 that the paper tests).
// ===========================================================================
template <class T, class NodeF, class MidF>
T h_plus(Scheme sc, double a, NodeF f, MidF F) {
  if (a != 1.0) {
    // the general one-midpoint forms; sc is W3_1MP, W5_1MP or W7_1MP
    switch (sc) {
      case W3_1MP:  // Eq. 3.5
        return a * F(0) + (a / 8.0 - 1.0 / 6.0) * f(-1) + (-3.0 * a / 4.0 + 5.0 / 6.0) * f(0) +
               (-3.0 * a / 8.0 + 1.0 / 3.0) * f(1);
      case W5_1MP:  // Eq. 3.17
        return a * F(0) + (-3.0 * a / 128.0 + 1.0 / 30.0) * f(-2) + (5.0 * a / 32.0 - 13.0 / 60.0) * f(-1) +
               (-45.0 * a / 64.0 + 47.0 / 60.0) * f(0) + (-15.0 * a / 32.0 + 9.0 / 20.0) * f(1) +
               (5.0 * a / 128.0 - 1.0 / 20.0) * f(2);
      default:  // Appendix (1), general form
        return a * F(0) + (5.0 * a / 1024.0 - 1.0 / 140.0) * f(-3) + (-21.0 * a / 512.0 + 5.0 / 84.0) * f(-2) +
               (175.0 * a / 1024.0 - 101.0 / 420.0) * f(-1) + (-175.0 * a / 256.0 + 319.0 / 420.0) * f(0) +
               (-525.0 * a / 1024.0 + 107.0 / 210.0) * f(1) + (35.0 * a / 512.0 - 19.0 / 210.0) * f(2) +
               (-7.0 * a / 1024.0 + 1.0 / 105.0) * f(3);
    }
  }
  switch (sc) {
    case W3_1MP:  // Eq. 3.4
      return F(0) + (1.0 / 24.0) * (-f(-1) + 2.0 * f(0) - f(1));
    case W3_2MP:  // Eq. 3.8
      return F(0) + (1.0 / 6.0) * (-F(-1) + 2.0 * f(0) - F(0));
    case W5_1MP:  // Eq. 3.16
      return F(0) + (19.0 / 1920.0) * f(-2) - (29.0 / 480.0) * f(-1) + (77.0 / 960.0) * f(0) -
             (3.0 / 160.0) * f(1) - (7.0 / 640.0) * f(2);
    case W5_2MP:  // Eq. 3.20
      return F(0) + (1.0 / 30.0) * ((-4.0 * f(1) + f(0) + f(-1)) + (6.0 * F(0) - 4.0 * F(-1)));
    case W7_1MP:  // Appendix (1), alpha = 1
      return F(0) + (1.0 / 107520.0) * (-243.0 * f(-3) + 1990.0 * f(-2) - 7481.0 * f(-1) + 8164.0 * f(0) -
                                        341.0 * f(1) - 2378.0 * f(2) + 289.0 * f(3));
    case W7_2MP:  // Appendix (2); its f_j coefficient -92 is read as -93 (consistency)
      return F(0) + (1.0 / 1260.0) * ((-128.0 * F(-1) + 404.0 * F(0)) +
                                      (-2.0 * f(-2) + 47.0 * f(-1) - 93.0 * f(0) - 233.0 * f(1) + 5.0 * f(2)));
    case W7_4MP:  // Appendix (3)
      return F(0) + (1.0 / 420.0) * ((18.0 * f(-1) - 66.0 * f(0) - 108.0 * f(1)) +
                                     (-3.0 * F(-2) - 31.0 * F(-1) + 179.0 * F(0) + 11.0 * F(1)));
    case W7_6MP:  // Appendix (4); its node term 3840 f_{j-1} is read as 3840 f_j
    default:
      return F(0) + (1.0 / 26880.0) * (3840.0 * f(0) + (-45.0 * F(-3) + 501.0 * F(-2) - 3874.0 * F(-1) +
                                                         746.0 * F(0) - 1249.0 * F(1) + 81.0 * F(2)));
  }
}

// ===========================================================================
// Sec. 2.3, Eq. 2.7 and Eqs. 3.7, 3.9, 3.19, 3.21: the central operator
// delta^{c,(1)} of each scheme, used for the grid metrics.  g(m) = g_{i+m} at
// nodes, gm(m) = g_{i+1/2+m} at midpoints (so g_{i-1/2} = gm(-1)).
// ===========================================================================
template <class NodeF, class MidF>
double delta_c(Scheme sc, NodeF g, MidF gm);

// The central operator of a one-midpoint scheme with free parameter a != 1,
// for which the paper prints none: Eq. 2.7 itself, half the sum of the
// upwind-biased difference and its mirror image,
//   delta g_i = [(h+_{i+1/2} - h+_{i-1/2}) + (h-_{i+1/2} - h-_{i-1/2})] / 2,
// with h- the mirror of h+ about the midpoint.  At a = 1 this reproduces the
// printed operators (Eqs. 3.7, 3.19, Appendix (1)).
template <class NodeF, class MidF>
double delta_c_eq27(Scheme sc, double a, NodeF g, MidF gm) {
  auto hp = [&](int s) {  // h+_{i+1/2+s}
    return h_plus<double>(sc, a, [&](int m) { return g(s + m); }, [&](int m) { return gm(s + m); });
  };
  auto hm = [&](int s) {  // h-_{i+1/2+s}
    return h_plus<double>(sc, a, [&](int m) { return g(s + 1 - m); }, [&](int m) { return gm(s - m); });
  };
  return 0.5 * ((hp(0) - hp(-1)) + (hm(0) - hm(-1)));
}

template <class NodeF, class MidF>
double delta_c(Scheme sc, double a, NodeF g, MidF gm) {
  return a == 1.0 ? delta_c(sc, g, gm) : delta_c_eq27(sc, a, g, gm);
}

template <class NodeF, class MidF>
double delta_c(Scheme sc, NodeF g, MidF gm) {
  switch (sc) {
    case W3_1MP:  // Eq. 3.7
      return (gm(0) - gm(-1)) + (1.0 / 48.0) * (-g(2) + 2.0 * g(1) - 2.0 * g(-1) + g(-2));
    case W3_2MP:  // Eq. 3.9
      return (1.0 / 12.0) * (2.0 * (g(1) - g(-1)) + (-gm(1) + 11.0 * gm(0) - 11.0 * gm(-1) + gm(-2)));
    case W5_1MP:  // Eq. 3.19
      return (gm(0) - gm(-1)) + (19.0 / 3840.0) * (g(3) - g(-3)) - (13.0 / 320.0) * (g(2) - g(-2)) +
             (17.0 / 256.0) * (g(1) - g(-1));
    case W5_2MP:  // Eq. 3.21 (its "f_{i+2}" is f_{j+2})
      return (1.0 / 60.0) * (g(2) - 4.0 * g(1) + 4.0 * g(-1) - g(-2)) +
             (1.0 / 15.0) * (-gm(1) + 19.0 * gm(0) - 19.0 * gm(-1) + gm(-2));
    case W7_1MP:  // Appendix (1)
      return (gm(0) - gm(-1)) + (1.0 / 107520.0) * (-121.5 * (g(4) - g(-4)) + 1261.0 * (g(3) - g(-3)) -
                                                    6069.0 * (g(2) - g(-2)) + 8841.0 * (g(1) - g(-1)));
    case W7_2MP:  // Appendix (2)
      return (1.0 / 315.0) * (-16.0 * (gm(1) - gm(-2)) + 432.0 * (gm(0) - gm(-1))) +
             (1.0 / 1260.0) * (-(g(3) - g(-3)) + 27.0 * (g(2) - g(-2)) - 189.0 * (g(1) - g(-1)));
    case W7_4MP:  // Appendix (3) (its "f_{i-2}", "f_{i-5/2}" are f_{j-2}, f_{j-5/2})
      return (1.0 / 140.0) * (3.0 * (g(2) - g(-2)) - 32.0 * (g(1) - g(-1))) +
             (1.0 / 840.0) * (-3.0 * (gm(2) - gm(-3)) - 17.0 * (gm(1) - gm(-2)) + 1218.0 * (gm(0) - gm(-1)));
    case W7_6MP:  // Appendix (4)
    default:
      return (1.0 / 14.0) * (g(1) - g(-1)) - (3.0 / 3584.0) * (gm(3) - gm(-4)) +
             (209.0 / 17920.0) * (gm(2) - gm(-3)) - (163.0 / 1536.0) * (gm(1) - gm(-2)) +
             (575.0 / 512.0) * (gm(0) - gm(-1));
  }
}

// Linear interpolation to the midpoint g_{i+1/2}.  The paper asks only for a
// "directionally consistent" linear interpolation, the same in the metrics
// and in the midpoint fluxes (Sec. 2.4).  The reading adopted is the central
// Lagrange interpolation one order above the scheme: six points g_{i-2..i+3}
// (sixth order) for the third- and fifth-order schemes, eight points
// g_{i-3..i+4} (eighth order) for the seventh-order ones, so the metrics keep
// the order of the scheme's central operator (Sec. 2.3, Appendix).
template <class NodeF> double interp_mid6(NodeF g) {
  return (3.0 * g(-2) - 25.0 * g(-1) + 150.0 * g(0) + 150.0 * g(1) - 25.0 * g(2) + 3.0 * g(3)) / 256.0;
}
template <class NodeF> double interp_mid8(NodeF g) {
  return (-5.0 * g(-3) + 49.0 * g(-2) - 245.0 * g(-1) + 1225.0 * g(0) + 1225.0 * g(1) - 245.0 * g(2) +
          49.0 * g(3) - 5.0 * g(4)) / 2048.0;
}
template <class NodeF> double interp_mid(Scheme sc, NodeF g) {
  return seventh_order(sc) ? interp_mid8(g) : interp_mid6(g);
}

// The scheme's metric derivative at a node, evaluated on the local relative
// values r[m + 8] = g_{i+m} - g_i, m = -8..8 (the operator annihilates
// constants, so subtracting g_i changes nothing but the rounding).
inline double metric_derivative(Scheme sc, double a, const double r[17]) {
  auto g = [&](int m) { return r[m + 8]; };
  auto gm = [&](int m) {  // g_{i+1/2+m}
    return interp_mid(sc, [&](int l) { return r[m + l + 8]; });
  };
  return delta_c(sc, a, g, gm);
}

// ===========================================================================
// Grid description and coordinate extension.
// ===========================================================================
// Rule of one side of a non-periodic direction for the states outside the
// grid (the paper fixes none; these are the library's): transmissive (copy
// of the boundary node), a reflecting slip wall (mirror image about the
// boundary node with the momentum's component along the boundary's metric
// direction reversed), or a fixed state (e.g. supersonic inflow).
// A side of a multi-block grid may instead be an interface to another block
// (multiblock.hpp), whose states continue the lines across it.
enum Side { SIDE_TRANSMISSIVE = 0, SIDE_WALL = 1, SIDE_FIXED = 2, SIDE_INTERFACE = 3 };

struct Grid {
  int nx, ny;
  Bc bcx, bcy;
  double Lx, Ly;  // period lengths of periodic directions
  int side[4] = {SIDE_TRANSMISSIVE, SIDE_TRANSMISSIVE, SIDE_TRANSMISSIVE, SIDE_TRANSMISSIVE};  // x lo, x hi, y lo, y hi
  double fixed[4][4] = {};  // conservative state outside a SIDE_FIXED side
};

inline int wrap(int a, int n) { int r = a % n; return r < 0 ? r + n : r; }
inline int floordiv(int a, int n) { return (a - wrap(a, n)) / n; }

// Extended coordinates X(a, b) for any integer (a, b), in extended precision.
// Periodic directions repeat the grid shifted by the period; transmissive
// directions extend it linearly from the last two nodes.  (The paper states
// no boundary rule; this is the reading adopted here.)
struct Coords {
  const Grid& g;
  const double* x;
  const double* y;
  void row(int a, int jr, long double& X, long double& Y) const {  // jr in [0, ny)
    if (g.bcx == PERIODIC) {
      int ar = wrap(a, g.nx), k = floordiv(a, g.nx);
      X = (long double)x[(size_t)jr * g.nx + ar] + (long double)k * (long double)g.Lx;
      Y = (long double)y[(size_t)jr * g.nx + ar];
      return;
    }
    auto at = [&](int i, long double& XX, long double& YY) {
      XX = x[(size_t)jr * g.nx + i]; YY = y[(size_t)jr * g.nx + i];
    };
    long double X0, Y0, X1, Y1;
    if (a < 0) {
      at(0, X0, Y0); at(1, X1, Y1);
      X = X0 + (long double)a * (X1 - X0); Y = Y0 + (long double)a * (Y1 - Y0);
    } else if (a >= g.nx) {
      at(g.nx - 1, X0, Y0); at(g.nx - 2, X1, Y1);
      long double s = (long double)(a - g.nx + 1);
      X = X0 + s * (X0 - X1); Y = Y0 + s * (Y0 - Y1);
    } else {
      at(a, X, Y);
    }
  }
  void at(int a, int b, long double& X, long double& Y) const {
    if (g.bcy == PERIODIC) {
      int br = wrap(b, g.ny), k = floordiv(b, g.ny);
      row(a, br, X, Y);
      Y += (long double)k * (long double)g.Ly;
      return;
    }
    long double X0, Y0, X1, Y1;
    if (b < 0) {
      row(a, 0, X0, Y0); row(a, 1, X1, Y1);
      X = X0 + (long double)b * (X1 - X0); Y = Y0 + (long double)b * (Y1 - Y0);
    } else if (b >= g.ny) {
      row(a, g.ny - 1, X0, Y0); row(a, g.ny - 2, X1, Y1);
      long double s = (long double)(b - g.ny + 1);
      X = X0 + s * (X0 - X1); Y = Y0 + s * (Y0 - Y1);
    } else {
      row(a, b, X, Y);
    }
  }
};

// Nodal metrics at (i, j) (any integers): Sec. 2.2 in two dimensions, where the
// conservative forms 2.3/2.4 reduce to xi_x^ = y_eta, xi_y^ = -x_eta,
// eta_x^ = -y_xi, eta_y^ = x_xi, and the Jacobian 2.5 to
// J^{-1} = x_xi y_eta - x_eta y_xi.  Each derivative is the scheme's own
// central operator (Sec. 2.3), evaluated on coordinate differences.
struct NodalMetric { double xix, xiy, etx, ety, jinv; };

template <class CoordSrc>
NodalMetric nodal_metric(Scheme sc, double a, const CoordSrc& C, int i, int j) {
  long double X0, Y0;
  C.at(i, j, X0, Y0);
  double rx[17], ry[17];
  for (int m = -8; m <= 8; ++m) {
    long double X, Y;
    C.at(i + m, j, X, Y);
    rx[m + 8] = (double)(X - X0); ry[m + 8] = (double)(Y - Y0);
  }
  double x_xi = metric_derivative(sc, a, rx), y_xi = metric_derivative(sc, a, ry);
  for (int m = -8; m <= 8; ++m) {
    long double X, Y;
    C.at(i, j + m, X, Y);
    rx[m + 8] = (double)(X - X0); ry[m + 8] = (double)(Y - Y0);
  }
  double x_eta = metric_derivative(sc, a, rx), y_eta = metric_derivative(sc, a, ry);
  NodalMetric nm;
  nm.xix = y_eta; nm.xiy = -x_eta; nm.etx = -y_xi; nm.ety = x_xi;
  nm.jinv = x_xi * y_eta - x_eta * y_xi;
  return nm;
}

// Metric storage: nine planes of (ny + 2G) x (nx + 2G) doubles, i fastest,
// node (i, j) at (j + G) * (nx + 2G) + (i + G):
//   0 xi_x^, 1 xi_y^, 2 eta_x^, 3 eta_y^, 4 J^{-1}            at nodes (i, j)
//   5 xi_x^, 6 xi_y^ at (i + 1/2, j);  7 eta_x^, 8 eta_y^ at (i, j + 1/2)
struct MetricView {
  int nx, ny;
  const double* M;
  size_t plane() const { return (size_t)(nx + 2 * G) * (ny + 2 * G); }
  double operator()(int p, int i, int j) const {
    return M[p * plane() + (size_t)(j + G) * (nx + 2 * G) + (i + G)];
  }
};

// Fill all nine metric planes, ghost band included.  Periodic directions copy
// the metrics of the wrapped node; transmissive ones evaluate them on the
// extended coordinates.  Midpoint metrics are the interpolation of the nodal
// ones in the same direction (Sec. 2.4, directionally consistent).
template <class CoordSrc>
void compute_metrics_from(Scheme sc, double alpha_h, const Grid& g, const CoordSrc& C, double* M) {
  const int W = g.nx + 2 * G, H = g.ny + 2 * G;
  const size_t P = (size_t)W * H;
  // Nodal metrics on a band wide enough for the midpoint interpolation.
  const int B = G + (seventh_order(sc) ? 4 : 3);
  const int WB = g.nx + 2 * B, HB = g.ny + 2 * B;
  std::vector<NodalMetric> nm((size_t)WB * HB);
  auto wr = [&](int a, int n, Bc bc) { return bc == PERIODIC ? wrap(a, n) : a; };
#pragma omp parallel for schedule(static)
  for (int b = -B; b < g.ny + B; ++b)
    for (int a = -B; a < g.nx + B; ++a)
      nm[(size_t)(b + B) * WB + (a + B)] = nodal_metric(sc, alpha_h, C, wr(a, g.nx, g.bcx), wr(b, g.ny, g.bcy));
  auto N = [&](int a, int b) -> const NodalMetric& {
    // for periodic directions use the wrapped node so copies are bitwise equal
    int aa = g.bcx == PERIODIC ? wrap(a, g.nx) : a;
    int bb = g.bcy == PERIODIC ? wrap(b, g.ny) : b;
    return nm[(size_t)(bb + B) * WB + (aa + B)];
  };
  for (int b = -G; b < g.ny + G; ++b)
    for (int a = -G; a < g.nx + G; ++a) {
      size_t o = (size_t)(b + G) * W + (a + G);
      const NodalMetric& n0 = N(a, b);
      M[0 * P + o] = n0.xix; M[1 * P + o] = n0.xiy;
      M[2 * P + o] = n0.etx; M[3 * P + o] = n0.ety; M[4 * P + o] = n0.jinv;
      M[5 * P + o] = interp_mid(sc, [&](int l) { return N(a + l, b).xix; });
      M[6 * P + o] = interp_mid(sc, [&](int l) { return N(a + l, b).xiy; });
      M[7 * P + o] = interp_mid(sc, [&](int l) { return N(a, b + l).etx; });
      M[8 * P + o] = interp_mid(sc, [&](int l) { return N(a, b + l).ety; });
    }
}

inline void compute_metrics(Scheme sc, double alpha_h, const Grid& g, const double* x, const double* y,
                            double* M) {
  compute_metrics_from(sc, alpha_h, g, Coords{g, x, y}, M);
}

// ===========================================================================
// Sec. 2.1: state, pressure and the contravariant flux of Eq. 2.2 in 2-D,
// E^ = k_x E + k_y F for the hatted metric direction (k_x, k_y).
// ===========================================================================
template <class T> T pressure(const T Q[4], double gam) {
  T u = Q[1] / Q[0], v = Q[2] / Q[0];
  return (gam - 1.0) * (Q[3] - 0.5 * Q[0] * (u * u + v * v));
}

// Primitive variables (rho, u, v, p) of a conservative state and back.
template <class T> void to_primitive(const T Q[4], double gam, T P[4]) {
  P[0] = Q[0];
  P[1] = Q[1] / Q[0];
  P[2] = Q[2] / Q[0];
  P[3] = pressure(Q, gam);
}
template <class T> void to_conservative(const T P[4], double gam, T Q[4]) {
  Q[0] = P[0];
  Q[1] = P[0] * P[1];
  Q[2] = P[0] * P[2];
  Q[3] = P[3] / (gam - 1.0) + 0.5 * P[0] * (P[1] * P[1] + P[2] * P[2]);
}

template <class T> void flux_hat(const T Q[4], double gam, double kx, double ky, T out[4]) {
  T rho = Q[0], u = Q[1] / Q[0], v = Q[2] / Q[0];
  T p = (gam - 1.0) * (Q[3] - 0.5 * rho * (u * u + v * v));
  T U = kx * u + ky * v;
  out[0] = rho * U;
  out[1] = Q[1] * U + kx * p;
  out[2] = Q[2] * U + ky * p;
  out[3] = (Q[3] + p) * U;
}

// Wave speed |U^| + c |k^| of Sec. 2.3 (the absolute value is the reading
// adopted for "MAX(U^ + c|k^|)").
template <class T> T wave_speed(const T Q[4], double gam, double kx, double ky) {
  T u = Q[1] / Q[0], v = Q[2] / Q[0];
  T p = (gam - 1.0) * (Q[3] - 0.5 * Q[0] * (u * u + v * v));
  T c = sqrt(gam * p / Q[0]);
  T U = kx * u + ky * v;
  return fabs(U) + c * std::sqrt(kx * kx + ky * ky);
}

// ===========================================================================
// Sec. 3.4: eigenvectors of the flux Jacobian in the unit direction n at the
// reference state.  Right eigenvectors (columns) for q_n - c, q_n, q_n, q_n + c
// and the matching left eigenvectors (rows), with b1 = (gamma-1)/c^2 and
// b2 = b1 q^2 / 2.  (The paper fixes no basis; this one is the reading
// adopted.)
// ===========================================================================
template <class T> void eigenvectors(const T Q[4], double gam, double nx_, double ny_, T L[4][4], T R[4][4]) {
  T rho = Q[0], u = Q[1] / rho, v = Q[2] / rho;
  T q2 = u * u + v * v;
  T p = (gam - 1.0) * (Q[3] - 0.5 * rho * q2);
  T c = sqrt(gam * p / rho);
  T Hh = (Q[3] + p) / rho;
  T qn = u * nx_ + v * ny_;
  T qt = -u * ny_ + v * nx_;
  T b1 = (gam - 1.0) / (c * c);
  T b2 = 0.5 * b1 * q2;
  // columns of R
  R[0][0] = T(1.0);        R[0][1] = T(1.0);  R[0][2] = T(0.0);  R[0][3] = T(1.0);
  R[1][0] = u - c * nx_;   R[1][1] = u;       R[1][2] = T(-ny_); R[1][3] = u + c * nx_;
  R[2][0] = v - c * ny_;   R[2][1] = v;       R[2][2] = T(nx_);  R[2][3] = v + c * ny_;
  R[3][0] = Hh - c * qn;   R[3][1] = 0.5 * q2; R[3][2] = qt;     R[3][3] = Hh + c * qn;
  // rows of L
  L[0][0] = 0.5 * (b2 + qn / c); L[0][1] = 0.5 * (-b1 * u - nx_ / c);
  L[0][2] = 0.5 * (-b1 * v - ny_ / c); L[0][3] = 0.5 * b1;
  L[1][0] = 1.0 - b2; L[1][1] = b1 * u; L[1][2] = b1 * v; L[1][3] = -b1;
  L[2][0] = -qt; L[2][1] = T(-ny_); L[2][2] = T(nx_); L[2][3] = T(0.0);
  L[3][0] = 0.5 * (b2 - qn / c); L[3][1] = 0.5 * (-b1 * u + nx_ / c);
  L[3][2] = 0.5 * (-b1 * v + ny_ / c); L[3][3] = 0.5 * b1;
}

// ===========================================================================
// Split of the midpoint flux at the interpolated state Q (side 0: F^+, side
// 1: F^-) with the midpoint metric k = (kx, ky).
//   split 0 (the paper's, Sec. 2.3): Lax-Friedrichs, F+- = (E^(Q; k) +- lam Q)/2
//     with the line eigenvalue lam.
//   split 1 (Steger-Warming; Sec. 7 names it): F+- = R diag(l+-) L Q with the
//     eigen-decomposition of the flux Jacobian along n = k/|k| at Q,
//     l = |k| (q_n - c, q_n, q_n, q_n + c), l+- = (l +- |l|)/2.  Since E^ is
//     homogeneous of degree one in Q, F+ + F- = E^(Q; k).
//   split 2 (van Leer; Sec. 7 names it): the Mach-number split along n,
//     M = q_n / c; F+ = E^, F- = 0 for M >= 1 (mirrored for M <= -1), else
//     F+- = +-|k| rho c (M +- 1)^2 / 4 (1, u + n_x (-q_n +- 2c)/gamma,
//     v + n_y (-q_n +- 2c)/gamma, ((gamma-1) q_n +- 2c)^2 / (2(gamma^2-1)) +
//     (q^2 - q_n^2)/2).
// Only the midpoint flux is split differently; the nodal fluxes keep the
// Lax-Friedrichs split, so FSP is unaffected (at a uniform state every split
// sums to E^ with the same midpoint metric).
// ===========================================================================
template <class T>
void midpoint_split(const Params& pr, const T Q[4], double kx, double ky, const T& lam, int side, T out[4]) {
  const double gam = pr.gamma;
  if (pr.split == 0) {
    T E[4];
    flux_hat(Q, gam, kx, ky, E);
    const double sgn = side == 0 ? 1.0 : -1.0;
    for (int q = 0; q < 4; ++q) out[q] = 0.5 * (E[q] + sgn * lam * Q[q]);
    return;
  }
  const double kn = std::sqrt(kx * kx + ky * ky);
  const double nx_ = kx / kn, ny_ = ky / kn;
  const T rho = Q[0], u = Q[1] / rho, v = Q[2] / rho;
  const T p = pressure(Q, gam);
  const T c = sqrt(gam * p / rho);
  const T qn = u * nx_ + v * ny_;
  if (pr.split == 1) {
    T L[4][4], R[4][4];
    eigenvectors(Q, gam, nx_, ny_, L, R);
    const T lam4[4] = {kn * (qn - c), kn * qn, kn * qn, kn * (qn + c)};
    T w[4];
    for (int a = 0; a < 4; ++a) {
      T lq = T(0.0);
      for (int b = 0; b < 4; ++b) lq = lq + L[a][b] * Q[b];
      const T part = side == 0 ? 0.5 * (lam4[a] + fabs(lam4[a])) : 0.5 * (lam4[a] - fabs(lam4[a]));
      w[a] = part * lq;
    }
    for (int a = 0; a < 4; ++a) {
      out[a] = T(0.0);
      for (int b = 0; b < 4; ++b) out[a] = out[a] + R[a][b] * w[b];
    }
    return;
  }
  const T M = qn / c;
  if ((side == 0 && T(1.0) <= M) || (side == 1 && M <= T(-1.0))) {
    flux_hat(Q, gam, kx, ky, out);
    return;
  }
  if ((side == 0 && M <= T(-1.0)) || (side == 1 && T(1.0) <= M)) {
    for (int q = 0; q < 4; ++q) out[q] = T(0.0);
    return;
  }
  const double s = side == 0 ? 1.0 : -1.0;
  const T fm = s * kn * rho * c * (M + s) * (M + s) / 4.0;
  const T vt = -qn + s * 2.0 * c;
  const T e2 = (gam - 1.0) * qn + s * 2.0 * c;
  out[0] = fm;
  out[1] = fm * (u + nx_ * vt / gam);
  out[2] = fm * (v + ny_ * vt / gam);
  out[3] = fm * (e2 * e2 / (2.0 * (gam * gam - 1.0)) + 0.5 * (u * u + v * v - qn * qn));
}

// ===========================================================================
// Midpoint split fluxes F^+_{k+1/2}, F^-_{k+1/2} (Secs. 2.3, 2.4, 3.4).
// Inputs: the eight states Q_{k-3..k+4}, the nodal hatted metrics at k and k+1
// (their mean gives the eigenvector direction), the midpoint metric (I xi^)_{k+1/2},
// and the line eigenvalue lambda.
//   + side: reference state Q_k, left-biased interpolation of L Q over
//           k-2..k+2 (k-1..k+1 for r = 2, k-3..k+3 for r = 4)
//   - side: reference state Q_{k+1}, the mirror image about k+1/2
// Each midpoint is evaluated once and reused by every h that needs it.
//
// The projection is applied to the deviations Q_m - Q_ref and Q_ref is added
// back after R: since R L = I and the WENO interpolation commutes with adding
// a constant (the indicators see only differences and each candidate's
// coefficients sum to one), this is the same map as R WENO(L Q); it only
// removes the rounding of the round trip, so a uniform state comes back
// bitwise (the reading adopted for free-stream preservation at round-off).
// ===========================================================================
template <class T>
void midpoint_flux(Scheme sc, const Params& pr, const T Qs[8][4], double kx0, double ky0, double kx1,
                   double ky1, double mkx, double mky, const T& lam, T Fp[4], T Fm[4]) {
  double nbx = 0.5 * (kx0 + kx1), nby = 0.5 * (ky0 + ky1);
  double nn = std::sqrt(nbx * nbx + nby * nby);
  double nx_ = nbx / nn, ny_ = nby / nn;
  // window entries either side reads: Q_{k-3..k+4} for r = 4, Q_{k-2..k+3}
  // otherwise (the others are left out, and set to zero where passed on)
  const int m0 = seventh_order(sc) ? 0 : 1, m1 = seventh_order(sc) ? 8 : 7;
  for (int side = 0; side < 2; ++side) {
    const T* Qref = Qs[3 + side];  // Q_k for +, Q_{k+1} for -
    // the entries this side's interpolation reads, each deviation formed once
    int lo, hi;
    side_window(sc, side, lo, hi);
    T Qm[4];
    if (pr.vars == 0) {
      T L[4][4], R[4][4];
      eigenvectors(Qref, pr.gamma, nx_, ny_, L, R);
      T dQ[8][4];
      for (int m = lo; m < hi; ++m)
        for (int q = 0; q < 4; ++q) dQ[m][q] = m == 3 + side ? T(0.0) : Qs[m][q] - Qref[q];
      T W[4];
      for (int c = 0; c < 4; ++c) {
        T s[8];
        for (int m = 0; m < 8; ++m) {
          s[m] = T(0.0);
          // the reference node's own deviation is zero, and so is its projection
          if (m < lo || m >= hi || m == 3 + side) continue;
          s[m] = L[c][0] * dQ[m][0];
          for (int q = 1; q < 4; ++q) s[m] = s[m] + L[c][q] * dQ[m][q];
        }
        W[c] = side == 0 ? weno_left(sc, s, pr) : weno_right(sc, s, pr);
      }
      for (int q = 0; q < 4; ++q) {
        Qm[q] = R[q][0] * W[0];
        for (int c = 1; c < 4; ++c) Qm[q] = Qm[q] + R[q][c] * W[c];
        Qm[q] = Qref[q] + Qm[q];
      }
    } else {
      // Sec. 2.4: component by component in conservative (vars 1) or
      // primitive (vars 2) variables, on deviations from the reference
      // node's values as above
      T V[8][4];
      for (int m = 0; m < 8; ++m) {
        if (m < m0 || m >= m1)
          for (int q = 0; q < 4; ++q) V[m][q] = T(0.0);
        else if (pr.vars == 1)
          for (int q = 0; q < 4; ++q) V[m][q] = Qs[m][q];
        else
          to_primitive(Qs[m], pr.gamma, V[m]);
      }
      T Vm[4];
      for (int c = 0; c < 4; ++c) {
        T s[8];
        for (int m = 0; m < 8; ++m)
          s[m] = (m < lo || m >= hi || m == 3 + side) ? T(0.0) : V[m][c] - V[3 + side][c];
        Vm[c] = V[3 + side][c] + (side == 0 ? weno_left(sc, s, pr) : weno_right(sc, s, pr));
      }
      if (pr.vars == 1)
        for (int q = 0; q < 4; ++q) Qm[q] = Vm[q];
      else
        to_conservative(Vm, pr.gamma, Qm);
    }
    midpoint_split(pr, Qm, mkx, mky, lam, side, side == 0 ? Fp : Fm);
  }
}

// ===========================================================================
// One grid line: residual R_k = H_{k+1/2} - H_{k-1/2}, k = 0..n-1 (Eq. 3.2
// with unit spacing), H = h^+ + h^-.  Accessors:
//   Q(k, q)   conservative state at line index k (boundary rule applied)
//   K(0, k), K(1, k)  nodal hatted metric (k_x, k_y) of this direction
//   K(2, k), K(3, k)  midpoint metric at k+1/2
// The Lax-Friedrichs eigenvalue is alpha * max over the line's own nodes of
// the wave speed (Sec. 2.3); it is returned in *lam_out.
// ===========================================================================
template <class T, class QF, class KF>
void line_residual(Scheme sc, const Params& pr, int n, QF Q, KF K, T* R, T* lam_out, const T* smax_in = nullptr) {
  auto kx = [&](int k) { return K(0, k); };
  auto ky = [&](int k) { return K(1, k); };
  auto mkx = [&](int k) { return K(2, k); };
  auto mky = [&](int k) { return K(3, k); };
  // Sec. 2.3: A^ = alpha MAX(|U^| + c|k^|) over the full line.
  T lam = T(0.0);
  bool first = true;
  for (int k = 0; k < n; ++k) {
    T Qk[4] = {Q(k, 0), Q(k, 1), Q(k, 2), Q(k, 3)};
    T s = wave_speed(Qk, pr.gamma, kx(k), ky(k));
    if (first || s > lam) { lam = s; first = false; }
  }
  // on a line that continues into other blocks, the maximum over all of it
  if (smax_in) lam = *smax_in;
  lam = pr.alpha_lf * lam;
  if (lam_out) *lam_out = lam;

  // Indices a residual needs: nodes -4 .. n+3, midpoints -4 .. n+2 (the
  // widest stencils, of the seventh-order schemes; the metric ghost band
  // reaches exactly that far).
  const int off = 4;  // arrays hold indices -4 .. n+3
  const int len = n + 8;
  std::vector<T> fp(4 * len), fm(4 * len), Fp(4 * len), Fm(4 * len);
  // Nodal split fluxes f^+- = (E^ +- lambda Q) / 2 (Sec. 2.3).
  for (int k = -4; k < n + 4; ++k) {
    T Qk[4] = {Q(k, 0), Q(k, 1), Q(k, 2), Q(k, 3)}, E[4];
    flux_hat(Qk, pr.gamma, kx(k), ky(k), E);
    for (int q = 0; q < 4; ++q) {
      fp[q * len + k + off] = 0.5 * (E[q] + lam * Qk[q]);
      fm[q * len + k + off] = 0.5 * (E[q] - lam * Qk[q]);
    }
  }
  // Midpoint split fluxes at k+1/2 (Lax-Friedrichs split).  With another
  // midpoint splitting (Sec. 7), only the leading f_{i+1/2} of each h, the
  // term Sec. 7 singles out, takes it: H_{i+1/2} gains D = (F~+ - F+) +
  // (F~- - F-) at its own midpoint, while the correction terms of the 2-, 4-
  // and 6-midpoint schemes keep the Lax-Friedrichs values.  (Splitting every
  // midpoint value would break FSP for those schemes: a lone F+ at another
  // midpoint is then not linear in the metric.)
  Params plf = pr;
  plf.split = 0;
  std::vector<T> D(pr.split != 0 ? 4 * len : 0);
  for (int k = -4; k < n + 3; ++k) {
    T Qs[8][4];
    for (int m = 0; m < 8; ++m)
      for (int q = 0; q < 4; ++q) Qs[m][q] = Q(k - 3 + m, q);
    T a[4], b[4];
    midpoint_flux(sc, plf, Qs, kx(k), ky(k), kx(k + 1), ky(k + 1), mkx(k), mky(k), lam, a, b);
    for (int q = 0; q < 4; ++q) { Fp[q * len + k + off] = a[q]; Fm[q * len + k + off] = b[q]; }
    if (pr.split != 0 && k >= -1 && k < n) {
      T ga[4], gb[4];
      midpoint_flux(sc, pr, Qs, kx(k), ky(k), kx(k + 1), ky(k + 1), mkx(k), mky(k), lam, ga, gb);
      for (int q = 0; q < 4; ++q) D[q * len + k + off] = (ga[q] - a[q]) + (gb[q] - b[q]);
    }
  }
  // H_{i+1/2} = h^+_{i+1/2} + h^-_{i+1/2}; h^- is h^+ mirrored about i+1/2
  // (node i+m <-> i+1-m, midpoint i+1/2+m <-> i+1/2-m).
  std::vector<T> H(4 * (n + 1));
  for (int i = -1; i < n; ++i)
    for (int q = 0; q < 4; ++q) {
      auto fpn = [&](int m) { return fp[q * len + i + m + off]; };
      auto Fpm = [&](int m) { return Fp[q * len + i + m + off]; };
      auto fmn = [&](int m) { return fm[q * len + i + 1 - m + off]; };
      auto Fmm = [&](int m) { return Fm[q * len + i - m + off]; };
      H[q * (n + 1) + i + 1] = h_plus<T>(sc, pr.alpha_h, fpn, Fpm) + h_plus<T>(sc, pr.alpha_h, fmn, Fmm);
      if (pr.split != 0) H[q * (n + 1) + i + 1] = H[q * (n + 1) + i + 1] + D[q * len + i + off];
    }
  for (int k = 0; k < n; ++k)
    for (int q = 0; q < 4; ++q) R[q * n + k] = H[q * (n + 1) + k + 1] - H[q * (n + 1) + k];
}

// ===========================================================================
// Eq. 2.2 / 3.2: dQ/dt = -[(H^xi_{i+1/2} - H^xi_{i-1/2}) + (H^eta_{j+1/2} - H^eta_{j-1/2})] / J^{-1}.
// U and dUdt: [4][ny][nx].  lam_xi[ny], lam_eta[nx] receive the line
// eigenvalues when non-null.
// ===========================================================================
// Coupling of one block to the others of a multi-block grid: the state at
// depth m >= 1 beyond interface side s on line `line` of the block, and the
// maximum wave speed of each of its lines over the whole line across the
// blocks it passes through (before the factor alpha).
template <class T> struct Coupling {
  std::function<T(int s, int m, int line, int q)> ghost;
  const T* smax_xi = nullptr;   // [ny]
  const T* smax_eta = nullptr;  // [nx]
};

template <class T>
void rhs(Scheme sc, const Params& pr, const Grid& g, const T* U, const double* M, T* dUdt,
         T* lam_xi = nullptr, T* lam_eta = nullptr, void (*phase_end)(int) = nullptr,
         const Coupling<T>* cp = nullptr) {
  const int nx = g.nx, ny = g.ny;
  const size_t NP = (size_t)nx * ny;
  MetricView mv{nx, ny, M};
  // State at line index k of a line of n nodes (at(m, q): node m of the line)
  // under the boundary rule: periodic wrap, or the side's rule beyond the
  // ends; kx, ky: the line direction's metric plane indices for a wall normal.
  auto line_state = [&](int n, bool periodic, int slo, int shi, int line, auto at, auto knode, int k, int q) -> T {
    if (periodic) return at(wrap(k, n), q);
    if (k >= 0 && k < n) return at(k, q);
    const int sd = k < 0 ? slo : shi;
    const int kb = k < 0 ? 0 : n - 1;  // boundary node
    if (g.side[sd] == SIDE_INTERFACE) return cp->ghost(sd, k < 0 ? -k : k - n + 1, line, q);
    if (g.side[sd] == SIDE_FIXED) return T(g.fixed[sd][q]);
    if (g.side[sd] == SIDE_WALL) {
      const int km = std::min(std::max(2 * kb - k, 0), n - 1);  // mirror node
      if (q == 0 || q == 3) return at(km, q);
      double nxb, nyb;
      knode(kb, nxb, nyb);
      const double nn = std::sqrt(nxb * nxb + nyb * nyb);
      nxb /= nn; nyb /= nn;
      const T mn = at(km, 1) * nxb + at(km, 2) * nyb;
      return at(km, q) - 2.0 * mn * (q == 1 ? nxb : nyb);
    }
    return at(kb, q);
  };
  std::vector<T> Rx(4 * NP), Ry(4 * NP);
  // xi sweep: one line per row j
#pragma omp parallel for schedule(dynamic)
  for (int j = 0; j < ny; ++j) {
    std::vector<T> R(4 * nx);
    auto at = [&](int m, int q) { return U[q * NP + (size_t)j * nx + m]; };
    auto kn = [&](int m, double& a, double& b) { a = mv(0, m, j); b = mv(1, m, j); };
    auto Q = [&](int k, int q) { return line_state(nx, g.bcx == PERIODIC, 0, 1, j, at, kn, k, q); };
    const int plane[4] = {0, 1, 5, 6};
    auto K = [&](int w, int k) { return mv(plane[w], k, j); };
    T lam;
    line_residual<T>(sc, pr, nx, Q, K, R.data(), &lam, cp && cp->smax_xi ? &cp->smax_xi[j] : nullptr);
    if (lam_xi) lam_xi[j] = lam;
    for (int q = 0; q < 4; ++q)
      for (int i = 0; i < nx; ++i) Rx[q * NP + (size_t)j * nx + i] = R[q * nx + i];
  }
  if (phase_end) phase_end(0);
  // eta sweep: one line per column i
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < nx; ++i) {
    std::vector<T> R(4 * ny);
    auto at = [&](int m, int q) { return U[q * NP + (size_t)m * nx + i]; };
    auto kn = [&](int m, double& a, double& b) { a = mv(2, i, m); b = mv(3, i, m); };
    auto Q = [&](int k, int q) { return line_state(ny, g.bcy == PERIODIC, 2, 3, i, at, kn, k, q); };
    const int plane[4] = {2, 3, 7, 8};
    auto K = [&](int w, int k) { return mv(plane[w], i, k); };
    T lam;
    line_residual<T>(sc, pr, ny, Q, K, R.data(), &lam, cp && cp->smax_eta ? &cp->smax_eta[i] : nullptr);
    if (lam_eta) lam_eta[i] = lam;
    for (int q = 0; q < 4; ++q)
      for (int j = 0; j < ny; ++j) Ry[q * NP + (size_t)j * nx + i] = R[q * ny + j];
  }
  if (phase_end) phase_end(1);
  for (int q = 0; q < 4; ++q)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t o = (size_t)j * nx + i;
        dUdt[q * NP + o] = -(Rx[q * NP + o] + Ry[q * NP + o]) / mv(4, i, j);
      }
  if (phase_end) phase_end(2);
}

// ===========================================================================
// Time step from the CFL number: dt = CFL / max_ij [(|U^| + c|xi^|) + (|V^| + c|eta^|)] / J^{-1}.
// (The paper uses fixed steps; this is the rule adopted for CFL-driven runs.)
// ===========================================================================
inline double cfl_dt(const Params& pr, const Grid& g, const double* U, const double* M, double cfl) {
  const size_t NP = (size_t)g.nx * g.ny;
  MetricView mv{g.nx, g.ny, M};
  double smax = 0.0;
  for (int j = 0; j < g.ny; ++j)
    for (int i = 0; i < g.nx; ++i) {
      size_t o = (size_t)j * g.nx + i;
      double Q[4] = {U[o], U[NP + o], U[2 * NP + o], U[3 * NP + o]};
      double s = wave_speed(Q, pr.gamma, mv(0, i, j), mv(1, i, j)) +
                 wave_speed(Q, pr.gamma, mv(2, i, j), mv(3, i, j));
      s = s / mv(4, i, j);
      if (s > smax) smax = s;
    }
  return cfl / smax;
}

// ===========================================================================
// Third-order TVD Runge-Kutta (Shu-Osher form), used in Sec. 6:
//   U1 = U + dt L(U);  U2 = 3/4 U + 1/4 (U1 + dt L(U1));  U = 1/3 U + 2/3 (U2 + dt L(U2)).
// ===========================================================================
template <class T>
void rk3_step(Scheme sc, const Params& pr, const Grid& g, T* U, const double* M, double dt) {
  const size_t N = 4 * (size_t)g.nx * g.ny;
  std::vector<T> L(N), U1(N), U2(N);
  rhs<T>(sc, pr, g, U, M, L.data());
  for (size_t e = 0; e < N; ++e) U1[e] = U[e] + dt * L[e];
  rhs<T>(sc, pr, g, U1.data(), M, L.data());
  for (size_t e = 0; e < N; ++e) U2[e] = 0.75 * U[e] + 0.25 * (U1[e] + dt * L[e]);
  rhs<T>(sc, pr, g, U2.data(), M, L.data());
  for (size_t e = 0; e < N; ++e) U[e] = (1.0 / 3.0) * U[e] + (2.0 / 3.0) * (U2[e] + dt * L[e]);
}

}  // namespace orc
