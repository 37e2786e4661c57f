// Device-side building blocks of libwenoiu (gfx950, fp64).
//
// Pointwise gas dynamics, the characteristic projection, the WENO
// interpolation with mapped weights and the upwind-biased flux combination of
// the WENOIU schemes (Li & Sun, arXiv 1810.11103).  Everything here is
// __device__ inline code used by the kernels in wiu_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <climits>

#define WIU_DEV __device__ __forceinline__

namespace wiu {

constexpr int GHOST = 4;              // metric ghost band
constexpr double TAG_MAGIC = 1810.11103;  // first word of the metric tag

// Grid description passed by value to every kernel.
struct Dims {
  int nx, ny;
  int bcx, bcy;        // 0 periodic, 1 transmissive
  int mpitch;          // nx + 2 GHOST
  long long mplane;    // (nx + 2 GHOST) (ny + 2 GHOST)
  long long np;        // nx ny
  double Lx, Ly;       // periods
};

// Status bits latched in the workspace header.
constexpr int ST_JACOBIAN = 1, ST_NONPHYS = 2, ST_SCHEME = 4, ST_ARGMAX = 8;

// Map a line index onto the grid: wrap for periodic lines, clamp (copy of the
// boundary node) for transmissive ones.  Loops run at most halo/n times.
// Error-free sum (Knuth's TwoSum): a + b = s + e exactly.
WIU_DEV void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  double aa = s - bb;
  e = (a - aa) + (b - bb);
}

WIU_DEV int bc_index(int k, int n, int bc) {
  if (bc == 0) {
    // one period covers every stencil reach on lines at least as long as
    // it; shorter periodic lines take the remainder
    k = k < 0 ? k + n : (k >= n ? k - n : k);
    if (k < 0 || k >= n) {
      k %= n;
      if (k < 0) k += n;
    }
    return k;
  }
  return k < 0 ? 0 : (k >= n ? n - 1 : k);
}

// XCD-aware block order.  The hardware hands consecutive workgroup ids to
// the eight XCDs in turn, and each XCD has its own L2.  Remapping the
// hardware id h so that XCD x receives one contiguous range of logical tiles
// keeps neighbouring tiles (which share cache lines and stencil halos) in the
// same L2.  Bijective for any total (the first `total % 8` XCDs get one extra).
WIU_DEV int xcd_remap(int h, int total) {
  const int q = total >> 3, r = total & 7;
  const int x = h & 7, local = h >> 3;
  return x * q + (x < r ? x : r) + local;
}

// Workgroup-uniform values read from global memory, moved into scalar
// registers (the compiler cannot prove such loads uniform and would
// otherwise hold them in vector registers).
WIU_DEV int ufirst(int x) { return __builtin_amdgcn_readfirstlane(x); }
WIU_DEV long long ufirst(long long x) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(x & 0xffffffffLL));
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)x >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
WIU_DEV double ufirst(double x) { return __longlong_as_double(ufirst((long long)__double_as_longlong(x))); }

WIU_DEV Dims ufirst(const Dims& g) {
  Dims d;
  d.nx = ufirst(g.nx); d.ny = ufirst(g.ny); d.bcx = ufirst(g.bcx); d.bcy = ufirst(g.bcy);
  d.mpitch = ufirst(g.mpitch); d.mplane = ufirst(g.mplane); d.np = ufirst(g.np);
  d.Lx = ufirst(g.Lx); d.Ly = ufirst(g.Ly);
  return d;
}

// Reciprocal and reciprocal square root: the hardware estimates refined by
// two Newton-Raphson steps (r <- r + r (1 - x r); y <- y + y (1 - x y^2) / 2),
// which leaves an error of about one ulp (measured on gfx950: 1.1e-16 and
// 1.4e-16 relative; one step leaves 2.2e-15) at a fraction of the cost of
// the correctly rounded division and square-root sequences.  Arguments here
// are positive, finite and well scaled (densities, sums of squared weights).
WIU_DEV double rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
// One Newton step only (about 2e-15 relative): for the normalisations of
// the WENO weights, where the error scales the interpolated deviation from
// the reference state and nothing else (that deviation is exactly zero for a
// uniform state, so free-stream preservation is untouched).
WIU_DEV double rcp_w(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}
WIU_DEV double rsqrt_(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * y;
  double e = fma(-(x * y), h, 0.5);
  y = fma(y, e, y);
  h = 0.5 * y;
  e = fma(-(x * y), h, 0.5);
  return fma(y, e, y);
}

// ---------------------------------------------------------------------------
// Scheme traits: order, midpoints, and the index ranges a tile needs.
//   node range of split fluxes f^+- : [o + NLO, o + out + NHI)
//   midpoint range F^+-_{k+1/2}     : [o + MLO, o + out + MHI)
// for outputs i in [o, o + out).
// ---------------------------------------------------------------------------
template <int SC> struct Traits;
template <> struct Traits<0> {  // WENOIU3-1MP, Eq. 3.4
  static constexpr bool fifth = false, two_mp = false;
  static constexpr int R = 2, NLO = -2, NHI = 2, MLO = -1, MHI = 0;
};
template <> struct Traits<1> {  // WENOIU3-2MP, Eq. 3.8
  static constexpr bool fifth = false, two_mp = true;
  static constexpr int R = 2, NLO = -1, NHI = 1, MLO = -2, MHI = 1;
};
template <> struct Traits<2> {  // WENOIU5-1MP, Eq. 3.16
  static constexpr bool fifth = true, two_mp = false;
  static constexpr int R = 3, NLO = -3, NHI = 3, MLO = -1, MHI = 0;
};
template <> struct Traits<3> {  // WENOIU5-2MP, Eq. 3.20
  static constexpr bool fifth = true, two_mp = true;
  static constexpr int R = 3, NLO = -2, NHI = 2, MLO = -2, MHI = 1;
};
// Seventh-order schemes of the Appendix (R = 4 interpolation, Table A1).
template <> struct Traits<4> {  // WENOIU7-1MP
  static constexpr bool fifth = false, two_mp = false;
  static constexpr int R = 4, NLO = -4, NHI = 4, MLO = -1, MHI = 0;
};
template <> struct Traits<5> {  // WENOIU7-2MP
  static constexpr bool fifth = false, two_mp = true;
  static constexpr int R = 4, NLO = -3, NHI = 3, MLO = -2, MHI = 1;
};
template <> struct Traits<6> {  // WENOIU7-4MP
  static constexpr bool fifth = false, two_mp = false;
  static constexpr int R = 4, NLO = -2, NHI = 2, MLO = -3, MHI = 2;
};
template <> struct Traits<7> {  // WENOIU7-6MP
  static constexpr bool fifth = false, two_mp = false;
  static constexpr int R = 4, NLO = -1, NHI = 1, MLO = -4, MHI = 3;
};
template <int SC> struct Range {
  static constexpr int LO = Traits<SC>::NLO < Traits<SC>::MLO ? Traits<SC>::NLO : Traits<SC>::MLO;
  static constexpr int HI = Traits<SC>::NHI > Traits<SC>::MHI ? Traits<SC>::NHI : Traits<SC>::MHI;
  static constexpr int EXTRA = HI - LO;
  // states a midpoint flux reads on each side of its item k: Q_{k-QL} ..
  // Q_{k+QL+1} (the R = 4 interpolation reaches one node further)
  static constexpr int QL = Traits<SC>::R == 4 ? 3 : 2;
};

// ---------------------------------------------------------------------------
// WENO interpolation to x_{k+1/2} with mapped weights.
// ---------------------------------------------------------------------------

// The interpolated sequences are characteristic deviations from the
// reference state, whose own entry (the centre v_k of the stencil) is exactly
// zero; the routines below take that zero into account.
//
// Mappings (Eqs. 3.15, 3.23) written as one polynomial in d = w - C:
//   third order:  g = C + K d^3, K = 1/C^2 for d <= 0, 1/(C-1)^2 above
//   second order: g = C + K d^2, K = -1/C for d <= 0, 1/(1-C) above
// (C[1 + (w/C - 1)^3] = C + d^3/C^2 and C[1 - (w/C - 1)^2] = C - d^2/C).
// K d without a branch or a select: the product with the constant of smaller
// magnitude is formed for either sign of d and the difference of the
// constants is applied to the part of d on the other side (min(d, 0) or
// max(d, 0), exact), so the result is exact on one side and within a few
// ulp on the other.  (Folding K into |d| as A d + B |d|, A, B =
// (K_hi +- K_lo)/2, cancels where |K_lo| >> |K_hi|: up to 2e5 times for the
// fourth-order mapping at C = 1/64.  A select costs the compare, two
// selects and VGPR copies of the 64-bit constants.)  The constants are
// literals, so the choice of form is made at compile time.
WIU_DEV double kd(double d, double Klo, double Khi) {
  if (fabs(Klo) >= fabs(Khi)) return fma(Klo - Khi, fmin(d, 0.0), Khi * d);
  return fma(Khi - Klo, fmax(d, 0.0), Klo * d);
}
// Each mapping returns C + K d^n as w + d (K d^(n-1) - 1), which needs no
// copy of C beside -C (the -1 is an inline constant).
WIU_DEV double map3(double w, double C, double Klo, double Khi) {
  const double d = w - C;
  return fma(d, fma(d, kd(d, Klo, Khi), -1.0), w);
}
WIU_DEV double map2(double w, double C, double Klo, double Khi) {
  const double d = w - C;
  return fma(d, kd(d, Klo, Khi) - 1.0, w);
}

// (K_lo, K_hi) of the mappings for the linear weights of Table 1.
//   r = 3: C = 1/16, 10/16, 5/16, K_lo = 1/C^2, K_hi = 1/(C-1)^2
//   r = 2: C = 1/4, 3/4,          K_lo = -1/C,  K_hi = 1/(1-C)
#define WIU_M3L0 256.0
#define WIU_M3H0 (256.0 / 225.0)
#define WIU_M3L1 2.56
#define WIU_M3H1 (64.0 / 9.0)
#define WIU_M3L2 10.24
#define WIU_M3H2 (256.0 / 121.0)
#define WIU_M2L0 (-4.0)
#define WIU_M2H0 (4.0 / 3.0)
#define WIU_M2L1 (-4.0 / 3.0)
#define WIU_M2H1 4.0

// r = 3: left-biased value at k+1/2 from v_{k-2}, v_{k-1}, v_k = 0, v_{k+1},
// v_{k+2} = (a, b, 0, d, e).  Candidates from Table 1 (b_{k,l}), linear
// weights (1, 10, 5)/16, Jiang-Shu indicators (Eq. 3.22)
//   IS = 13/12 t^2 + 1/4 s^2 = 13/12 t^2 + u^2,  u = s/2,
// with t, u formed directly from the values (t0 = a - 2b, u0 = a/2 - 2b
// = t0 - a/2; t1 = b + d, u1 = (b - d)/2; t2 = e - 2d, u2 = t2 - e/2), weights
// alpha_k / sum alpha with alpha_k = C_k / (eps + IS_k)^2 formed with one
// reciprocal (w_k = C_k prod_{l != k} D_l / sum_m C_m prod_{l != m} D_l; the
// common factor 1/16 of the C_k cancels), mapping Eq. 3.23 and
// re-normalisation.
// ZOK (compile time) admits ppm = 2, which selects WENO-Z weights (Sec. 7 names
// them; reading): alpha_k = C_k (1 + (tau / (eps + IS_k))^2) with the global
// indicator tau, no mapping, the q_k = tau / (eps + IS_k) from one reciprocal.
template <bool ZOK = false>
WIU_DEV double weno5(double a, double b, double d, double e, double eps, int ppm) {
  const double p0 = 0.375 * a - 1.25 * b;
  const double p1 = 0.375 * d - 0.125 * b;
  const double p2 = 0.75 * d - 0.125 * e;
  const double t0 = fma(-2.0, b, a), t1 = b + d, t2 = fma(-2.0, d, e);
  const double u0 = fma(-0.5, a, t0), u1 = 0.5 * (b - d), u2 = fma(-0.5, e, t2);
  double D0 = fma(13.0 / 12.0, t0 * t0, fma(u0, u0, eps));
  double D1 = fma(13.0 / 12.0, t1 * t1, fma(u1, u1, eps));
  double D2 = fma(13.0 / 12.0, t2 * t2, fma(u2, u2, eps));
  if constexpr (ZOK) {
    if (ppm == 2) {
      // tau = |IS_0 - IS_2|; q_k = tau / (eps + IS_k) from one reciprocal
      const double P01 = D0 * D1, R = rcp_w(P01 * D2), tau = fabs(D0 - D2);
      const double q0 = tau * (D1 * D2 * R), q1 = tau * (D0 * D2 * R), q2 = tau * (P01 * R);
      const double a0 = fma(q0, q0, 1.0), a1 = 10.0 * fma(q1, q1, 1.0), a2 = 5.0 * fma(q2, q2, 1.0);
      return (a0 * p0 + a1 * p1 + a2 * p2) * rcp_w(a0 + a1 + a2);
    }
  }
  D0 *= D0; D1 *= D1; D2 *= D2;
  const double a0 = D1 * D2, a1 = 10.0 * (D0 * D2), a2 = 5.0 * (D0 * D1);
  const double r = rcp_w(a0 + a1 + a2);
  double w0 = a0 * r, w1 = a1 * r, w2 = a2 * r;
  if (ppm) {
    w0 = map3(w0, 0.0625, WIU_M3L0, WIU_M3H0);
    w1 = map3(w1, 0.625, WIU_M3L1, WIU_M3H1);
    w2 = map3(w2, 0.3125, WIU_M3L2, WIU_M3H2);
  }
  return (w0 * p0 + w1 * p1 + w2 * p2) * rcp_w(w0 + w1 + w2);
}

// r = 2: left-biased value at k+1/2 from v_{k-2}, v_{k-1}, v_k = 0, v_{k+1}
// = (a, b, 0, d).  Candidates (-v_{k-1} + 3 v_k)/2 and (v_k + v_{k+1})/2,
// C = (1, 3)/4, with the three-point indicators IS_0, IS_1 of Eq. 3.22 in
// place of Eq. 3.14 (Sec. 5.1) and the mapping 3.15.
template <bool ZOK = false>
WIU_DEV double weno3(double a, double b, double d, double eps, int ppm) {
  const double p0 = -0.5 * b;
  const double p1 = 0.5 * d;
  // the first two r = 3 indicators, in the form of weno5
  const double t0 = fma(-2.0, b, a), t1 = b + d;
  const double u0 = fma(-0.5, a, t0), u1 = 0.5 * (b - d);
  double D0 = fma(13.0 / 12.0, t0 * t0, fma(u0, u0, eps));
  double D1 = fma(13.0 / 12.0, t1 * t1, fma(u1, u1, eps));
  if constexpr (ZOK) {
    if (ppm == 2) {  // WENO-Z, tau = |IS_0 - IS_1|
      const double R = rcp_w(D0 * D1), tau = fabs(D0 - D1);
      const double q0 = tau * (D1 * R), q1 = tau * (D0 * R);
      const double a0 = fma(q0, q0, 1.0), a1 = 3.0 * fma(q1, q1, 1.0);
      return (a0 * p0 + a1 * p1) * rcp_w(a0 + a1);
    }
  }
  D0 *= D0; D1 *= D1;
  const double a0 = D1, a1 = 3.0 * D0;
  const double r = rcp_w(a0 + a1);
  double w0 = a0 * r, w1 = a1 * r;
  if (ppm) {
    w0 = map2(w0, 0.25, WIU_M2L0, WIU_M2H0);
    w1 = map2(w1, 0.75, WIU_M2L1, WIU_M2H1);
  }
  return (w0 * p0 + w1 * p1) * rcp_w(w0 + w1);
}

// Fourth-order mapping of the Appendix, g = C (1 - (w/C - 1)^4) below C and
// C - (w - C)^4 / (C - 1)^3 above, i.e. g = C + K d^4 with K = -1/C^3 for
// d <= 0 and 1/(1-C)^3 above.
WIU_DEV double map4(double w, double C, double Klo, double Khi) {
  const double d = w - C;
  return fma(d, fma(d * d, kd(d, Klo, Khi), -1.0), w);
}
//   C = 1/64, 21/64, 35/64, 7/64: K_lo = -(64/(64 C))^3, K_hi = (64/(64 - 64 C))^3
#define WIU_M4L0 (-262144.0)
#define WIU_M4H0 (262144.0 / 250047.0)
#define WIU_M4L1 (-262144.0 / 9261.0)
#define WIU_M4H1 (262144.0 / 79507.0)
#define WIU_M4L2 (-262144.0 / 42875.0)
#define WIU_M4H2 (262144.0 / 24389.0)
#define WIU_M4L3 (-262144.0 / 343.0)
#define WIU_M4H3 (262144.0 / 185193.0)

// r = 4: left-biased value at k+1/2 from v_{k-3..k+3} = (a, b, c, 0, e, f, g)
// (seventh-order schemes, Appendix).  Candidates and linear weights
// (1, 21, 35, 7)/64 of Table A1.  The paper prints no r = 4 indicators; the
// Jiang-Shu definition that gives its r = 3 ones is used, written as a sum
// of squares: with p = c0 + c1 x + c2 x^2 + c3 x^3 the stencil's cubic on
// the unit cell around k,
//   IS = sum_{l=1..3} int (p^(l))^2 = (c1 + c3/4)^2 + 13/3 c2^2 + 781/20 c3^2,
// where c1 + c3/4, c2 and c3 are fixed differences of the stencil values.
// Weights as in weno5 (products of the squared denominators, one
// reciprocal), mapping map4, re-normalisation.
template <bool ZOK = false>
WIU_DEV double weno7(double a, double b, double c, double e, double f, double g, double eps, int ppm) {
  const double p0 = (-5.0 * a + 21.0 * b - 35.0 * c) * 0.0625;
  const double p1 = (b - 5.0 * c + 5.0 * e) * 0.0625;
  const double p2 = (-c + 9.0 * e - f) * 0.0625;
  const double p3 = (15.0 * e - 5.0 * f + g) * 0.0625;
  auto is = [&](double y1, double c2, double c3) {
    return fma(781.0 / 20.0, c3 * c3, fma(13.0 / 3.0, c2 * c2, fma(y1, y1, eps)));
  };
  const double ce = 0.5 * (c + e);  // c2 of the two central stencils
  double D0 = is(fma(1.5, b, fma(-1.0 / 3.0, a, -3.0 * c)), fma(2.0, b, fma(-0.5, a, -2.5 * c)),
                 (-a + 3.0 * (b - c)) * (1.0 / 6.0));
  double D1 = is(fma(1.0 / 6.0, b, fma(1.0 / 3.0, e, -c)), ce, (3.0 * c - b + e) * (1.0 / 6.0));
  double D2 = is(fma(-1.0 / 3.0, c, fma(-1.0 / 6.0, f, e)), ce, (f - c - 3.0 * e) * (1.0 / 6.0));
  double D3 = is(fma(3.0, e, fma(1.0 / 3.0, g, -1.5 * f)), fma(2.0, f, fma(-2.5, e, -0.5 * g)),
                 (3.0 * (e - f) + g) * (1.0 / 6.0));
  if constexpr (ZOK) {
    if (ppm == 2) {  // WENO-Z, tau = |IS_0 + 3 IS_1 - 3 IS_2 - IS_3|
      const double P01 = D0 * D1, P23 = D2 * D3, R = rcp_w(P01 * P23);
      const double tau = fabs(fma(3.0, D1 - D2, D0 - D3));
      const double q0 = tau * (D1 * P23 * R), q1 = tau * (D0 * P23 * R);
      const double q2 = tau * (D3 * P01 * R), q3 = tau * (D2 * P01 * R);
      const double a0 = fma(q0, q0, 1.0), a1 = 21.0 * fma(q1, q1, 1.0);
      const double a2 = 35.0 * fma(q2, q2, 1.0), a3 = 7.0 * fma(q3, q3, 1.0);
      return (a0 * p0 + a1 * p1 + a2 * p2 + a3 * p3) * rcp_w((a0 + a1) + (a2 + a3));
    }
  }
  D0 *= D0; D1 *= D1; D2 *= D2; D3 *= D3;
  const double P01 = D0 * D1, P23 = D2 * D3;
  const double a0 = (D1 * P23), a1 = 21.0 * (D0 * P23), a2 = 35.0 * (D3 * P01), a3 = 7.0 * (D2 * P01);
  const double r = rcp_w((a0 + a1) + (a2 + a3));
  double w0 = a0 * r, w1 = a1 * r, w2 = a2 * r, w3 = a3 * r;
  if (ppm) {
    w0 = map4(w0, 1.0 / 64.0, WIU_M4L0, WIU_M4H0);
    w1 = map4(w1, 21.0 / 64.0, WIU_M4L1, WIU_M4H1);
    w2 = map4(w2, 35.0 / 64.0, WIU_M4L2, WIU_M4H2);
    w3 = map4(w3, 7.0 / 64.0, WIU_M4L3, WIU_M4H3);
  }
  return (w0 * p0 + w1 * p1 + w2 * p2 + w3 * p3) * rcp_w((w0 + w1) + (w2 + w3));
}

// Steger-Warming (split 1) or van Leer (split 2) split of a midpoint flux at
// the interpolated state Q with the midpoint metric (mx, my); side 0 gives
// F^+, side 1 F^- (Sec. 7 names both for the midpoint flux; closed forms
// along n = k/|k|, scaled by |k|):
//   Steger-Warming: F = |k| rho/(2 gamma) [2(g-1) l2 + l1 + l3,
//     2(g-1) l2 u + l1 (u - c nx) + l3 (u + c nx), (same for v, ny),
//     (g-1) l2 q^2 + l1 |u - c n|^2/2 + l3 |u + c n|^2/2 + (3-g)(l1 + l3) c^2/(2(g-1))]
//     with l = (qn - c, qn, qn + c) reduced to its positive / negative parts;
//   van Leer: F = E^ / 0 beyond |M| = 1 (M = qn/c), else
//     +-|k| rho c (M +- 1)^2/4 [1, u + nx (-qn +- 2c)/g, v + ny (...)/g,
//     ((g-1) qn +- 2c)^2/(2(g^2-1)) + (q^2 - qn^2)/2].
WIU_DEV void mid_split_alt(int split, const double Q[4], double mx, double my, int side, double gam, double F[4]) {
  const double kn2 = mx * mx + my * my;
  const double rk = rsqrt_(kn2), kn = kn2 * rk;
  const double nx_ = mx * rk, ny_ = my * rk;
  const double ri = rcp(Q[0]);
  const double u = Q[1] * ri, v = Q[2] * ri;
  const double q2 = u * u + v * v;
  const double gm1 = gam - 1.0;
  const double p = gm1 * (Q[3] - 0.5 * Q[0] * q2);
  const double c2 = gam * p * ri;
  const double rc = rsqrt_(c2), c = c2 * rc;
  const double qn = u * nx_ + v * ny_;
  const double sg = side == 0 ? 1.0 : -1.0;
  if (split == 1) {
    auto part = [&](double l) { return 0.5 * fma(sg, fabs(l), l); };
    const double l1 = part(qn - c), l2 = part(qn), l3 = part(qn + c);
    const double f = kn * Q[0] * rcp(2.0 * gam);
    const double uc = c * nx_, vc = c * ny_;
    const double um = u - uc, up = u + uc, vm = v - vc, vp = v + vc;
    F[0] = f * (2.0 * gm1 * l2 + l1 + l3);
    F[1] = f * (2.0 * gm1 * l2 * u + l1 * um + l3 * up);
    F[2] = f * (2.0 * gm1 * l2 * v + l1 * vm + l3 * vp);
    F[3] = f * (gm1 * l2 * q2 + 0.5 * l1 * (um * um + vm * vm) + 0.5 * l3 * (up * up + vp * vp) +
                (3.0 - gam) * (l1 + l3) * c2 * rcp(2.0 * gm1));
    return;
  }
  const double M = qn * rc;
  if (sg * M >= 1.0) {
    const double U = mx * u + my * v;
    F[0] = Q[0] * U; F[1] = Q[1] * U + mx * p; F[2] = Q[2] * U + my * p; F[3] = (Q[3] + p) * U;
    return;
  }
  if (sg * M <= -1.0) {
    F[0] = F[1] = F[2] = F[3] = 0.0;
    return;
  }
  const double mp = M + sg;
  const double fm = sg * kn * Q[0] * c * mp * mp * 0.25;
  const double rg = rcp(gam);
  const double vt = fma(sg * 2.0, c, -qn), e2 = fma(sg * 2.0, c, gm1 * qn);
  F[0] = fm;
  F[1] = fm * fma(nx_ * vt, rg, u);
  F[2] = fm * fma(ny_ * vt, rg, v);
  F[3] = fm * (e2 * e2 * rcp(2.0 * (gam * gam - 1.0)) + 0.5 * (q2 - qn * qn));
}

// ---------------------------------------------------------------------------
// Characteristic midpoint flux, one side (Secs. 2.3, 2.4, 3.4).
//   q(m, c), m = 0..5: conservative states at k-2 .. k+3 (read through an
//   accessor so they can stay in LDS).
//   side 0: F^+_{k+1/2}, reference Q_k, left-biased over k-2..k+2
//   side 1: F^-_{k+1/2}, reference Q_{k+1}, right-biased over k+3..k-1
//   (nx_, ny_): unit normal of the averaged nodal metric; (mx, my): midpoint
//   metric; lam: line eigenvalue.
// The projection acts on deviations from the reference state (exact for a
// uniform state) with the left eigenvectors factored as
//   l_1 = (A + B)/2, l_2 = e_rho - A, l_4 = (A - B)/2 applied to dQ, with
//   A = b2 drho - b1 (u dm + v dn - de), B = (qn drho - nx dm - ny dn)/c.
// ---------------------------------------------------------------------------
template <bool FIFTH, bool ZOK = false, class QF>
WIU_DEV void side_flux(QF q, int side, double nx_, double ny_, double mx, double my, double lam, double gam,
                       double eps, int ppm, double F[4], int split = 0, double* Dacc = nullptr) {
  const double Qr[4] = {q(2 + side, 0), q(2 + side, 1), q(2 + side, 2), q(2 + side, 3)};
  const double gm1 = gam - 1.0;
  const double rr = rcp(Qr[0]);
  const double u = Qr[1] * rr, v = Qr[2] * rr;
  const double q2 = u * u + v * v;
  const double p = gm1 * (Qr[3] - 0.5 * Qr[0] * q2);
  const double c2 = gam * p * rr;
  const double rc = rsqrt_(c2);
  const double c = c2 * rc;
  const double H = (Qr[3] + p) * rr;
  const double qn = u * nx_ + v * ny_;
  const double qt = v * nx_ - u * ny_;
  const double b1 = gm1 * (rc * rc);
  const double b2 = 0.5 * b1 * q2;

  // stencil in sweep order: s = 0..4 (fifth) or 0..3 (third), left-biased
  // order for side 0, mirrored for side 1
  constexpr int NS = FIFTH ? 5 : 4;
  double w[4][NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (s == 2) continue;  // the reference node: zero deviation
    const int m = side == 0 ? s : 5 - s;
    const double dr = q(m, 0) - Qr[0], dm = q(m, 1) - Qr[1], dn = q(m, 2) - Qr[2], de = q(m, 3) - Qr[3];
    const double A = b2 * dr - b1 * (u * dm + v * dn - de);
    const double B = rc * (qn * dr - nx_ * dm - ny_ * dn);
    w[0][s] = 0.5 * (A + B);
    w[1][s] = dr - A;
    w[2][s] = nx_ * dn - ny_ * dm - qt * dr;
    w[3][s] = 0.5 * (A - B);
  }
  double W[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if constexpr (FIFTH) W[k] = weno5<ZOK>(w[k][0], w[k][1], w[k][3], w[k][4], eps, ppm);
    else W[k] = weno3<ZOK>(w[k][0], w[k][1], w[k][3], eps, ppm);
  }
  // back to conservative variables: Q = Q_ref + R W
  const double s03 = W[0] + W[3], d30 = W[3] - W[0];
  const double sum = s03 + W[1];
  const double r0 = Qr[0] + sum;
  const double r1 = Qr[1] + (u * sum + c * nx_ * d30 - ny_ * W[2]);
  const double r2 = Qr[2] + (v * sum + c * ny_ * d30 + nx_ * W[2]);
  const double r3 = Qr[3] + (H * s03 + c * qn * d30 + 0.5 * q2 * W[1] + qt * W[2]);
  // contravariant flux with the midpoint metric, then the split part
  const double ri = rcp(r0);
  const double ul = r1 * ri, vl = r2 * ri;
  const double pl = gm1 * (r3 - 0.5 * (r1 * ul + r2 * vl));
  const double Ul = mx * ul + my * vl;
  const double sl = side == 0 ? lam : -lam;
  F[0] = 0.5 * (r0 * Ul + sl * r0);
  F[1] = 0.5 * (r1 * Ul + mx * pl + sl * r1);
  F[2] = 0.5 * (r2 * Ul + my * pl + sl * r2);
  F[3] = 0.5 * ((r3 + pl) * Ul + sl * r3);
  if (split != 0) {
    // another split for the leading midpoint flux: accumulate its difference
    const double Qm[4] = {r0, r1, r2, r3};
    double G[4];
    mid_split_alt(split, Qm, mx, my, side, gam, G);
#pragma unroll
    for (int c = 0; c < 4; ++c) Dacc[c] += G[c] - F[c];
  }
}

// The same for the seventh-order schemes: q(m, c), m = 0..7, holds the states
// at k-3 .. k+4; side 0 is left-biased over k-3..k+3 (reference Q_k), side 1
// right-biased over k+4..k-2 (reference Q_{k+1}).  The characteristic
// fields are projected and interpolated in two passes over the stencil,
// fields 0 and 3 (which share A and B) and then fields 1 and 2, each pass
// re-reading the states from LDS: twelve projected values are live at a time
// instead of twenty-four (compiler barriers keep the passes apart).
template <bool ZOK = false, class QF>
WIU_DEV void side_flux7(QF q, int side, double nx_, double ny_, double mx, double my, double lam, double gam,
                        double eps, int ppm, double F[4], int split = 0, double* Dacc = nullptr) {
  const double Qr[4] = {q(3 + side, 0), q(3 + side, 1), q(3 + side, 2), q(3 + side, 3)};
  const double gm1 = gam - 1.0;
  const double rr = rcp(Qr[0]);
  const double u = Qr[1] * rr, v = Qr[2] * rr;
  const double q2 = u * u + v * v;
  const double p = gm1 * (Qr[3] - 0.5 * Qr[0] * q2);
  const double c2 = gam * p * rr;
  const double rc = rsqrt_(c2);
  const double c = c2 * rc;
  const double H = (Qr[3] + p) * rr;
  const double qn = u * nx_ + v * ny_;
  const double qt = v * nx_ - u * ny_;
  const double b1 = gm1 * (rc * rc);
  const double b2 = 0.5 * b1 * q2;

  // stencil position s = 0..6 (s = 3 the reference node) -> window index
  auto mi = [&](int s) { return side == 0 ? s : 7 - s; };
  double W[4];
  {
    double w0[7], w3[7];
#pragma unroll
    for (int s = 0; s < 7; ++s) {
      if (s == 3) continue;
      const int m = mi(s);
      const double dr = q(m, 0) - Qr[0], dm = q(m, 1) - Qr[1], dn = q(m, 2) - Qr[2], de = q(m, 3) - Qr[3];
      const double A = b2 * dr - b1 * (u * dm + v * dn - de);
      const double B = rc * (qn * dr - nx_ * dm - ny_ * dn);
      w0[s] = 0.5 * (A + B);
      w3[s] = 0.5 * (A - B);
    }
    W[0] = weno7<ZOK>(w0[0], w0[1], w0[2], w0[4], w0[5], w0[6], eps, ppm);
    asm volatile("" ::: "memory");
    W[3] = weno7<ZOK>(w3[0], w3[1], w3[2], w3[4], w3[5], w3[6], eps, ppm);
  }
  asm volatile("" ::: "memory");
  {
    double w1[7], w2[7];
#pragma unroll
    for (int s = 0; s < 7; ++s) {
      if (s == 3) continue;
      const int m = mi(s);
      const double dr = q(m, 0) - Qr[0], dm = q(m, 1) - Qr[1], dn = q(m, 2) - Qr[2], de = q(m, 3) - Qr[3];
      const double A = b2 * dr - b1 * (u * dm + v * dn - de);
      w1[s] = dr - A;
      w2[s] = nx_ * dn - ny_ * dm - qt * dr;
    }
    W[1] = weno7<ZOK>(w1[0], w1[1], w1[2], w1[4], w1[5], w1[6], eps, ppm);
    asm volatile("" ::: "memory");
    W[2] = weno7<ZOK>(w2[0], w2[1], w2[2], w2[4], w2[5], w2[6], eps, ppm);
  }
  const double s03 = W[0] + W[3], d30 = W[3] - W[0];
  const double sum = s03 + W[1];
  const double r0 = Qr[0] + sum;
  const double r1 = Qr[1] + (u * sum + c * nx_ * d30 - ny_ * W[2]);
  const double r2 = Qr[2] + (v * sum + c * ny_ * d30 + nx_ * W[2]);
  const double r3 = Qr[3] + (H * s03 + c * qn * d30 + 0.5 * q2 * W[1] + qt * W[2]);
  const double ri = rcp(r0);
  const double ul = r1 * ri, vl = r2 * ri;
  const double pl = gm1 * (r3 - 0.5 * (r1 * ul + r2 * vl));
  const double Ul = mx * ul + my * vl;
  const double sl = side == 0 ? lam : -lam;
  F[0] = 0.5 * (r0 * Ul + sl * r0);
  F[1] = 0.5 * (r1 * Ul + mx * pl + sl * r1);
  F[2] = 0.5 * (r2 * Ul + my * pl + sl * r2);
  F[3] = 0.5 * ((r3 + pl) * Ul + sl * r3);
  if (split != 0) {
    // another split for the leading midpoint flux: accumulate its difference
    const double Qm[4] = {r0, r1, r2, r3};
    double G[4];
    mid_split_alt(split, Qm, mx, my, side, gam, G);
#pragma unroll
    for (int c = 0; c < 4; ++c) Dacc[c] += G[c] - F[c];
  }
}

// Midpoint flux with the midpoint state interpolated component by component
// (Sec. 2.4) in conservative (vars 1) or primitive (vars 2: rho, u, v, p)
// variables instead of characteristic ones.  Same window and sides as
// side_flux / side_flux7 (R = 2, 3: q(m), m = 0..5 at k-2..k+3; R = 4:
// m = 0..7 at k-3..k+4), same deviation form: each variable is interpolated
// as its deviation from the reference node's value, which is then added
// back.  Primitive values are formed from the staged conservative states
// with one reciprocal density per stencil point.
template <int R, bool ZOK = false, class QF>
WIU_DEV void side_flux_comp(QF q, int side, int vars, double mx, double my, double lam, double gam, double eps,
                            int ppm, double F[4], int split = 0, double* Dacc = nullptr) {
  constexpr int QL = R == 4 ? 3 : 2;        // reference position in the window (side 0)
  constexpr int NS = R == 2 ? 4 : 2 * R - 1;  // stencil positions s = 0..NS-1, reference at s = QL
  const double gm1 = gam - 1.0;
  auto mi = [&](int s) { return side == 0 ? s : 2 * QL + 1 - s; };
  double rinv[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) rinv[s] = vars == 2 ? rcp(q(mi(s), 0)) : 0.0;
  // variable c at stencil position s
  auto var = [&](int s, int c) -> double {
    const int m = mi(s);
    if (vars == 1 || c == 0) return q(m, c);
    if (c == 1) return q(m, 1) * rinv[s];
    if (c == 2) return q(m, 2) * rinv[s];
    const double a = q(m, 1), b = q(m, 2);
    return gm1 * (q(m, 3) - 0.5 * (a * a + b * b) * rinv[s]);
  };
  double V[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    asm volatile("" ::: "memory");  // one variable at a time (register pressure)
    const double vr = var(QL, c);
    double v[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) v[s] = s == QL ? 0.0 : var(s, c) - vr;
    double w;
    if constexpr (R == 4) w = weno7<ZOK>(v[0], v[1], v[2], v[4], v[5], v[6], eps, ppm);
    else if constexpr (R == 3) w = weno5<ZOK>(v[0], v[1], v[3], v[4], eps, ppm);
    else w = weno3<ZOK>(v[0], v[1], v[3], eps, ppm);
    V[c] = vr + w;
  }
  double r0, r1, r2, r3;
  if (vars == 1) {
    r0 = V[0]; r1 = V[1]; r2 = V[2]; r3 = V[3];
  } else {
    r0 = V[0]; r1 = V[0] * V[1]; r2 = V[0] * V[2];
    r3 = fma(V[3], rcp(gm1), 0.5 * V[0] * (V[1] * V[1] + V[2] * V[2]));
  }
  const double ri = rcp(r0);
  const double ul = r1 * ri, vl = r2 * ri;
  const double pl = gm1 * (r3 - 0.5 * (r1 * ul + r2 * vl));
  const double Ul = mx * ul + my * vl;
  const double sl = side == 0 ? lam : -lam;
  F[0] = 0.5 * (r0 * Ul + sl * r0);
  F[1] = 0.5 * (r1 * Ul + mx * pl + sl * r1);
  F[2] = 0.5 * (r2 * Ul + my * pl + sl * r2);
  F[3] = 0.5 * ((r3 + pl) * Ul + sl * r3);
  if (split != 0) {
    // another split for the leading midpoint flux: accumulate its difference
    const double Qm[4] = {r0, r1, r2, r3};
    double G[4];
    mid_split_alt(split, Qm, mx, my, side, gam, G);
#pragma unroll
    for (int c = 0; c < 4; ++c) Dacc[c] += G[c] - F[c];
  }
}

// Nodal contravariant flux E^ = (rho U, m U + kx p, n U + ky p, (e + p) U),
// U = kx u + ky v, with the nodal metric (Sec. 2.1).
WIU_DEV void nodal_flux(const double Q[4], double kx, double ky, double gam, double E[4]) {
  const double ri = rcp(Q[0]);
  const double u = Q[1] * ri, v = Q[2] * ri;
  const double p = (gam - 1.0) * (Q[3] - 0.5 * (Q[1] * u + Q[2] * v));
  const double U = kx * u + ky * v;
  E[0] = Q[0] * U;
  E[1] = Q[1] * U + kx * p;
  E[2] = Q[2] * U + ky * p;
  E[3] = (Q[3] + p) * U;
}

// Nodal split fluxes f^+- = (E^ +- lam Q)/2 with the nodal metric (Sec. 2.3).
WIU_DEV void nodal_split(const double Q[4], double kx, double ky, double lam, double gam, double fp[4],
                         double fm[4]) {
  const double ri = rcp(Q[0]);
  const double u = Q[1] * ri, v = Q[2] * ri;
  const double p = (gam - 1.0) * (Q[3] - 0.5 * (Q[1] * u + Q[2] * v));
  const double U = kx * u + ky * v;
  const double E0 = Q[0] * U, E1 = Q[1] * U + kx * p, E2 = Q[2] * U + ky * p, E3 = (Q[3] + p) * U;
  fp[0] = 0.5 * (E0 + lam * Q[0]); fm[0] = 0.5 * (E0 - lam * Q[0]);
  fp[1] = 0.5 * (E1 + lam * Q[1]); fm[1] = 0.5 * (E1 - lam * Q[1]);
  fp[2] = 0.5 * (E2 + lam * Q[2]); fm[2] = 0.5 * (E2 - lam * Q[2]);
  fp[3] = 0.5 * (E3 + lam * Q[3]); fm[3] = 0.5 * (E3 - lam * Q[3]);
}

// Wave speed |k . u| + c |k| (Sec. 2.3); returns a negative value for a
// non-physical or non-finite state so callers can flag it.
// Wave speed |k . u| + c |k| (Sec. 2.3), evaluated as |k . u| + sqrt(c^2 |k|^2)
// (one root per direction; c^2 shared by both directions of a node).
// No contraction here: the adjoint locates the node attaining a line maximum
// by recomputing this value in another kernel, which must round identically.
struct WaveState {
  double u, v, c2;
  bool bad;  // rho <= 0 or p <= 0 (or not finite)
};

WIU_DEV WaveState wave_state(const double Q[4], double gam) {
#pragma clang fp contract(off)
  const double ri = rcp(Q[0]);
  WaveState w;
  w.u = Q[1] * ri;
  w.v = Q[2] * ri;
  const double p = (gam - 1.0) * (Q[3] - 0.5 * (Q[1] * w.u + Q[2] * w.v));
  w.c2 = gam * p * ri;
  w.bad = !(Q[0] > 0.0) || !(p > 0.0);
  return w;
}

WIU_DEV double wave_speed_dir(const WaveState& w, double kx, double ky) {
#pragma clang fp contract(off)
  return fabs(kx * w.u + ky * w.v) + sqrt(w.c2 * (kx * kx + ky * ky));
}

WIU_DEV double wave_speed(const double Q[4], double kx, double ky, double gam, bool& bad) {
  const WaveState w = wave_state(Q, gam);
  const double s = wave_speed_dir(w, kx, ky);
  bad = w.bad || !(s < 1.0e300);
  return s;
}

// ---------------------------------------------------------------------------
// Upwind-biased numerical flux H_{i+1/2} = h^+ + h^- (Eqs. 3.4, 3.8, 3.16,
// 3.20 and the Appendix, alpha = 1; h^- is h^+ mirrored about i+1/2).
// fp(k), fm(k): nodal split fluxes at node k; Fp(k), Fm(k): midpoint split
// fluxes at k+1/2.
// ---------------------------------------------------------------------------

// h^+_{i+1/2} of the seventh-order schemes from f(m) = f_{i+m} and
// F(m) = f_{i+1/2+m}.  Two printed coefficients are read as corrected, as
// the central-scheme decomposition (Eq. 2.7) into the printed central
// operators requires: 7-2MP's f_i weight -93 (printed -92), 7-6MP's node term
// 3840 f_i (printed at f_{i-1}).
template <int SC, class NF, class MF>
WIU_DEV double h7_plus(NF f, MF F) {
  if constexpr (SC == 4) {
    return F(0) + (1.0 / 107520.0) * (-243.0 * f(-3) + 1990.0 * f(-2) - 7481.0 * f(-1) + 8164.0 * f(0) -
                                      341.0 * f(1) - 2378.0 * f(2) + 289.0 * f(3));
  } else if constexpr (SC == 5) {
    return F(0) + (1.0 / 1260.0) * (-128.0 * F(-1) + 404.0 * F(0) - 2.0 * f(-2) + 47.0 * f(-1) - 93.0 * f(0) -
                                    233.0 * f(1) + 5.0 * f(2));
  } else if constexpr (SC == 6) {
    return F(0) + (1.0 / 420.0) * (18.0 * f(-1) - 66.0 * f(0) - 108.0 * f(1) - 3.0 * F(-2) - 31.0 * F(-1) +
                                   179.0 * F(0) + 11.0 * F(1));
  } else {
    return F(0) + (1.0 / 26880.0) * (3840.0 * f(0) - 45.0 * F(-3) + 501.0 * F(-2) - 3874.0 * F(-1) +
                                     746.0 * F(0) - 1249.0 * F(1) + 81.0 * F(2));
  }
}

// h^+_{i+1/2} of the one-midpoint families with free parameter a (Eq. 3.5
// for SC 0, Eq. 3.17 for SC 2, Appendix (1) for SC 4); a = 1 is the printed
// scheme, which hflux evaluates in its printed form instead.
template <int SC, class NF, class MF>
WIU_DEV double h1mp_plus(double a, NF f, MF F) {
  if constexpr (SC == 0) {
    return a * F(0) + (a * 0.125 - 1.0 / 6.0) * f(-1) + (-0.75 * a + 5.0 / 6.0) * f(0) +
           (-0.375 * a + 1.0 / 3.0) * f(1);
  } else if constexpr (SC == 2) {
    return a * F(0) + (-3.0 / 128.0 * a + 1.0 / 30.0) * f(-2) + (5.0 / 32.0 * a - 13.0 / 60.0) * f(-1) +
           (-45.0 / 64.0 * a + 47.0 / 60.0) * f(0) + (-15.0 / 32.0 * a + 0.45) * f(1) +
           (5.0 / 128.0 * a - 0.05) * f(2);
  } else {
    return a * F(0) + (5.0 / 1024.0 * a - 1.0 / 140.0) * f(-3) + (-21.0 / 512.0 * a + 5.0 / 84.0) * f(-2) +
           (175.0 / 1024.0 * a - 101.0 / 420.0) * f(-1) + (-175.0 / 256.0 * a + 319.0 / 420.0) * f(0) +
           (-525.0 / 1024.0 * a + 107.0 / 210.0) * f(1) + (35.0 / 512.0 * a - 19.0 / 210.0) * f(2) +
           (-7.0 / 1024.0 * a + 1.0 / 105.0) * f(3);
  }
}

// H_{k+1/2} = h^+_{k+1/2} + h^-_{k+1/2} of WENOIU5-2MP (Eq. 3.20 and its
// mirror image) with the nodal split fluxes written as f^+- = (E +- lam Q)/2.
// Collecting the terms of both halves gives
//   H = 6/5 (F^+_k + F^-_k) - 2/15 (F^+_{k-1} + F^-_{k+1})
//     + 1/60 [E_{k-1} + E_{k+2} - 3 (E_k + E_{k+1})]
//     + lam/60 [Q_{k-1} - Q_{k+2} + 5 (Q_k - Q_{k+1})],
// the linear map of hflux<3> in eleven operations instead of about twenty;
// for a uniform state the lam Q terms vanish exactly.  E(m), Q(m): nodal
// flux and state at k + m; Fp(m), Fm(m): midpoint split fluxes at k + m + 1/2.
template <class EF, class QF, class GP, class GM>
WIU_DEV double hsum52(double lam, EF E, QF Q, GP Fp, GM Fm) {
  const double g0 = Fp(0) + Fm(0), g1 = Fp(-1) + Fm(1);
  const double ep = fma(-3.0, E(0) + E(1), E(-1) + E(2));
  const double qp = fma(5.0, Q(0) - Q(1), Q(-1) - Q(2));
  return fma(1.0 / 60.0, fma(lam, qp, ep), fma(-2.0 / 15.0, g1, 1.2 * g0));
}

template <int SC, class FP, class FM, class GP, class GM>
WIU_DEV double hflux(int i, double ah, FP fp, FM fm, GP Fp, GM Fm) {
  if constexpr (SC == 0 || SC == 2 || SC == 4) {
    if (ah != 1.0)
      return h1mp_plus<SC>(ah, [&](int m) { return fp(i + m); }, [&](int m) { return Fp(i + m); }) +
             h1mp_plus<SC>(ah, [&](int m) { return fm(i + 1 - m); }, [&](int m) { return Fm(i - m); });
  }
  if constexpr (SC == 0) {
    return Fp(i) + (1.0 / 24.0) * (2.0 * fp(i) - fp(i - 1) - fp(i + 1)) +
           Fm(i) + (1.0 / 24.0) * (2.0 * fm(i + 1) - fm(i + 2) - fm(i));
  } else if constexpr (SC == 1) {
    return Fp(i) + (1.0 / 6.0) * (2.0 * fp(i) - Fp(i - 1) - Fp(i)) +
           Fm(i) + (1.0 / 6.0) * (2.0 * fm(i + 1) - Fm(i + 1) - Fm(i));
  } else if constexpr (SC == 2) {
    return Fp(i) + (1.0 / 1920.0) * (19.0 * fp(i - 2) - 116.0 * fp(i - 1) + 154.0 * fp(i) - 36.0 * fp(i + 1) -
                                     21.0 * fp(i + 2)) +
           Fm(i) + (1.0 / 1920.0) * (19.0 * fm(i + 3) - 116.0 * fm(i + 2) + 154.0 * fm(i + 1) - 36.0 * fm(i) -
                                     21.0 * fm(i - 1));
  } else if constexpr (SC == 3) {
    return Fp(i) + (1.0 / 30.0) * (fp(i - 1) + fp(i) - 4.0 * fp(i + 1) + 6.0 * Fp(i) - 4.0 * Fp(i - 1)) +
           Fm(i) + (1.0 / 30.0) * (fm(i + 2) + fm(i + 1) - 4.0 * fm(i) + 6.0 * Fm(i) - 4.0 * Fm(i + 1));
  } else {
    return h7_plus<SC>([&](int m) { return fp(i + m); }, [&](int m) { return Fp(i + m); }) +
           h7_plus<SC>([&](int m) { return fm(i + 1 - m); }, [&](int m) { return Fm(i - m); });
  }
}

}  // namespace wiu
