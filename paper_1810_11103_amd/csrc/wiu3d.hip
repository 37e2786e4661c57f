// Three-dimensional Euler equations on curvilinear grids (gfx950, fp64): the
// paper's method in its general form (Sec. 2.1, Eq. 2.2) -- metrics in the
// symmetric conservative form (Eq. 2.4) with each scheme's central operator,
// Jacobian by Eq. 2.5, the characteristic projection of Sec. 3.4 with five
// eigenvectors, the WENOIU midpoint fluxes and upwind-biased difference of
// every scheme, TVD-RK3.  The paper's configuration only (characteristic
// variables, Lax-Friedrichs split, alpha = 1, Jiang-Shu weights).
//
// A direction pass is one LDS-tiled sweep (states staged once, one item per
// lane, item records in LDS, the flux difference and the stage update in the
// same kernel), with lanes along i wherever global memory is touched so
// loads and stores coalesce whatever the line direction.  The passes run
// zeta, eta, xi: the xi pass, whose lines are contiguous in memory, writes
// dU/dt or the RK stage (and, in stages 1 and 2, the next stage's maxima).
#include "wenoiu.h"

#include <utility>
#include "wiu_kernels.hpp"

namespace wiu {

constexpr double TAG_MAGIC3 = 1810.111033;
constexpr int NP3 = 19;   // metric planes (see wenoiu.h)

struct Dims3 {
  int n[3], bc[3];
  double L[3];
  long long np;        // nodes
  int mp[2];           // metric box pitches nx+2G, ny+2G
  long long mplane;    // metric plane size
};

WIU_DEV long long m3idx(const Dims3& d, int i, int j, int k) {
  return ((long long)(k + GHOST) * d.mp[1] + (j + GHOST)) * d.mp[0] + (i + GHOST);
}
WIU_DEV long long u3idx(const Dims3& d, int i, int j, int k) {
  return ((long long)k * d.n[1] + j) * d.n[0] + i;
}

// ===========================================================================
// Coordinates at any position: a node coordinate (base) plus an offset --
// shifts across periodic seams, and beyond transmissive ends the linear
// extension direction by direction (trilinear at edges and corners, as
// sum over the out-of-range set T of prod_{d in T} e_d times the mixed
// backward difference at the clamped node) -- so differences of nearby
// positions take the base difference error-free.
// ===========================================================================
WIU_DEV void c3_point(const Dims3& d, const double* __restrict__ X, int c, const int p_in[3], double& base,
                      double& off) {
  int p[3] = {p_in[0], p_in[1], p_in[2]};
  off = 0.0;
  int cc[3], in[3], e[3];
  for (int a = 0; a < 3; ++a) {
    if (d.bc[a] == WIU_BC_PERIODIC) {
      const int w = bc_index(p[a], d.n[a], 0);
      if (a == c) off += (double)((p[a] - w) / d.n[a]) * d.L[a];
      p[a] = w;
    }
    cc[a] = min(max(p[a], 0), d.n[a] - 1);
    e[a] = abs(p[a] - cc[a]);
    in[a] = e[a] ? (p[a] < 0 ? 1 : -1) : 0;
  }
  auto at = [&](int da, int db, int dc) {
    return X[((long long)(cc[2] + dc) * d.n[1] + (cc[1] + db)) * d.n[0] + (cc[0] + da)];
  };
  base = at(0, 0, 0);
  if (e[0] | e[1] | e[2]) {
    // mixed differences over the out-of-range directions
    double ext = 0.0;
    for (int t = 1; t < 8; ++t) {
      const int t0 = t & 1, t1 = (t >> 1) & 1, t2 = (t >> 2) & 1;
      if ((t0 && !e[0]) || (t1 && !e[1]) || (t2 && !e[2])) continue;
      double md = 0.0;
      for (int s = 0; s < 8; ++s) {
        if ((s & ~t) != 0) continue;  // s a subset of t
        const int s0 = s & 1, s1 = (s >> 1) & 1, s2 = (s >> 2) & 1;
        const double v = at(s0 * in[0], s1 * in[1], s2 * in[2]);
        md += ((s0 + s1 + s2) & 1) ? -v : v;
      }
      ext += (double)((t0 ? e[0] : 1) * (t1 ? e[1] : 1) * (t2 ? e[2] : 1)) * md;
    }
    off += ext;
  }
}

WIU_DEV double c3_diff(const Dims3& d, const double* X, int c, const int p1[3], const int p0[3]) {
  double b1, o1, b0, o0, s, e;
  c3_point(d, X, c, p1, b1, o1);
  c3_point(d, X, c, p0, b0, o0);
  two_sum(b1, -b0, s, e);
  return s + ((o1 - o0) + e);
}

struct Coord3 {
  const double* x[3];
};

// Inner derivatives D_a x_c (a, c = 0..2) on the box [-E, n+E)^3:
// Dx[3a + c][box index].
__global__ void m3_inner_kernel(Dims3 d, MetricStencil ms, int E, Coord3 X, double* __restrict__ Dx) {
  const long long W0 = d.n[0] + 2 * E, W1 = d.n[1] + 2 * E, W2 = d.n[2] + 2 * E;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long P = W0 * W1 * W2;
  if (t >= P) return;
  const int p[3] = {(int)(t % W0) - E, (int)((t / W0) % W1) - E, (int)(t / (W0 * W1)) - E};
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int m = 1; m <= METRIC_REACH; ++m) {
        const double cm = ms.d[m - 1];
        if (cm == 0.0) continue;
        int p1[3] = {p[0], p[1], p[2]}, p0[3] = {p[0], p[1], p[2]};
        p1[a] += m;
        p0[a] -= m;
        s += cm * c3_diff(d, X.x[c], c, p1, p0);
      }
      Dx[(3 * a + c) * P + t] = s;
    }
}

// Nodal metrics (Eq. 2.4) and J^{-1} (Eq. 2.5) on [-B, n+B)^3 into T[10]:
// for direction m with (a, b) the next two directions cyclically and
// component l with (p, q) the next two coordinates cyclically,
//   n^_{m,l} = 1/2 [D_b(q D_a p) - D_a(q D_b p) + D_a(p D_b q) - D_b(p D_a q)],
// with p, q taken relative to the node.  Periodic directions evaluate at the
// wrapped node.
__global__ void m3_nodal_kernel(Dims3 d, MetricStencil ms, int B, int E, Coord3 X, const double* __restrict__ Dx,
                                double* __restrict__ T) {
  const long long V0 = d.n[0] + 2 * B, V1 = d.n[1] + 2 * B, V2 = d.n[2] + 2 * B;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long P = V0 * V1 * V2;
  if (t >= P) return;
  int w[3] = {(int)(t % V0) - B, (int)((t / V0) % V1) - B, (int)(t / (V0 * V1)) - B};
  for (int a = 0; a < 3; ++a)
    if (d.bc[a] == WIU_BC_PERIODIC) w[a] = bc_index(w[a], d.n[a], 0);
  const long long W0 = d.n[0] + 2 * E, W1 = d.n[1] + 2 * E;
  const long long DP = W0 * W1 * (d.n[2] + 2 * E);
  auto dx = [&](int plane, const int p[3]) {
    return Dx[plane * DP + ((long long)(p[2] + E) * W1 + (p[1] + E)) * W0 + (p[0] + E)];
  };
  double J = 0.0;
  for (int m = 0; m < 3; ++m) {
    const int a = (m + 1) % 3, b = (m + 2) % 3;
    for (int l = 0; l < 3; ++l) {
      const int pc = (l + 1) % 3, qc = (l + 2) % 3;
      // D_outer((X_cv - X_cv(w)) D_inner X_cd)
      auto term = [&](int outer, int cv, int inner, int cd) {
        double s = 0.0;
        for (int k = 1; k <= METRIC_REACH; ++k) {
          const double ck = ms.d[k - 1];
          if (ck == 0.0) continue;
          int p1[3] = {w[0], w[1], w[2]}, p0[3] = {w[0], w[1], w[2]};
          p1[outer] += k;
          p0[outer] -= k;
          const double f1 = c3_diff(d, X.x[cv], cv, p1, w) * dx(3 * inner + cd, p1);
          const double f0 = c3_diff(d, X.x[cv], cv, p0, w) * dx(3 * inner + cd, p0);
          s += ck * (f1 - f0);
        }
        return s;
      };
      const double v = 0.5 * (term(b, qc, a, pc) - term(a, qc, b, pc) + term(a, pc, b, qc) - term(b, pc, a, qc));
      T[(3 * m + l) * P + t] = v;
      J += v * dx(3 * m + l, w);
    }
  }
  T[9 * P + t] = J * (1.0 / 3.0);
}

// Stored metrics: nodal planes and midpoint interpolation in each metric's
// own direction, ghost band included, plus the tag.  jform 6 replaces
// J^{-1} by Eq. 2.6, 1/3 sum_{m,l} D_m(n^_{m,l} x_l) with x_l relative to
// the (wrapped) node, which needs the nodal band B >= GHOST + METRIC_REACH.
__global__ void m3_band_kernel(Dims3 d, int scheme, int B, const double* __restrict__ T, double* __restrict__ M,
                               int* __restrict__ status, int jform, MetricStencil ms, Coord3 X, double ah) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    double* tag = M + NP3 * d.mplane;
    tag[0] = TAG_MAGIC3; tag[1] = (double)scheme; tag[2] = (double)d.n[0]; tag[3] = (double)d.n[1];
    tag[4] = (double)d.n[2]; tag[5] = (double)(d.bc[0] + 2 * d.bc[1] + 4 * d.bc[2]); tag[6] = ah;
    tag[7] = (double)jform;
  }
  if (t >= d.mplane) return;
  const int p[3] = {(int)(t % d.mp[0]) - GHOST, (int)((t / d.mp[0]) % d.mp[1]) - GHOST,
                    (int)(t / ((long long)d.mp[0] * d.mp[1])) - GHOST};
  const long long V0 = d.n[0] + 2 * B, V1 = d.n[1] + 2 * B;
  const long long TP = V0 * V1 * (d.n[2] + 2 * B);
  auto tv = [&](int plane, int i, int j, int k) {
    return T[plane * TP + ((long long)(k + B) * V1 + (j + B)) * V0 + (i + B)];
  };
  for (int q = 0; q < 10; ++q) M[q * d.mplane + t] = tv(q, p[0], p[1], p[2]);
  if (jform == 6) {
    int w[3] = {p[0], p[1], p[2]};
    for (int a = 0; a < 3; ++a)
      if (d.bc[a] == WIU_BC_PERIODIC) w[a] = bc_index(w[a], d.n[a], 0);
    double J = 0.0;
    for (int m = 0; m < 3; ++m)
      for (int l = 0; l < 3; ++l)
        for (int k = 1; k <= METRIC_REACH; ++k) {
          const double ck = ms.d[k - 1];
          if (ck == 0.0) continue;
          int p1[3] = {w[0], w[1], w[2]}, p0[3] = {w[0], w[1], w[2]};
          p1[m] += k;
          p0[m] -= k;
          J += ck * (tv(3 * m + l, p1[0], p1[1], p1[2]) * c3_diff(d, X.x[l], l, p1, w) -
                     tv(3 * m + l, p0[0], p0[1], p0[2]) * c3_diff(d, X.x[l], l, p0, w));
        }
    M[9 * d.mplane + t] = J * (1.0 / 3.0);
  }
  const bool eight = scheme >= 4;
  for (int m = 0; m < 3; ++m)
    for (int l = 0; l < 3; ++l) {
      auto v = [&](int s) {
        int r[3] = {p[0], p[1], p[2]};
        r[m] += s;
        return tv(3 * m + l, r[0], r[1], r[2]);
      };
      M[(10 + 3 * m + l) * d.mplane + t] =
          eight ? (-5.0 * (v(-3) + v(4)) + 49.0 * (v(-2) + v(3)) - 245.0 * (v(-1) + v(2)) +
                   1225.0 * (v(0) + v(1))) * (1.0 / 2048.0)
                : (3.0 * v(-2) - 25.0 * v(-1) + 150.0 * v(0) + 150.0 * v(1) - 25.0 * v(2) + 3.0 * v(3)) *
                      (1.0 / 256.0);
    }
  if (p[0] >= 0 && p[0] < d.n[0] && p[1] >= 0 && p[1] < d.n[1] && p[2] >= 0 && p[2] < d.n[2]) {
    const double j = M[9 * d.mplane + t];
    if (!(j > 0.0) || !(j < 1.0e300)) atomicOr(status, ST_JACOBIAN);
  }
}

// ===========================================================================
// Physics in three dimensions (Sec. 2.1; Sec. 3.4 eigenvectors).
// ===========================================================================
WIU_DEV void flux3(const double Q[5], const double k[3], double gam, double E[5]) {
  const double ri = rcp(Q[0]);
  const double u = Q[1] * ri, v = Q[2] * ri, w = Q[3] * ri;
  const double p = (gam - 1.0) * (Q[4] - 0.5 * (Q[1] * u + Q[2] * v + Q[3] * w));
  const double U = k[0] * u + k[1] * v + k[2] * w;
  E[0] = Q[0] * U;
  E[1] = Q[1] * U + k[0] * p;
  E[2] = Q[2] * U + k[1] * p;
  E[3] = Q[3] * U + k[2] * p;
  E[4] = (Q[4] + p) * U;
}

// |k . u| + c |k| without contraction (every kernel rounds it alike).
WIU_DEV double speed3(const double Q[5], const double k[3], double gam, bool& bad) {
#pragma clang fp contract(off)
  const double ri = rcp(Q[0]);
  const double u = Q[1] * ri, v = Q[2] * ri, w = Q[3] * ri;
  const double p = (gam - 1.0) * (Q[4] - 0.5 * (Q[1] * u + Q[2] * v + Q[3] * w));
  const double c2 = gam * p * ri;
  bad = !(Q[0] > 0.0) || !(p > 0.0);
  const double s = fabs(k[0] * u + k[1] * v + k[2] * w) + sqrt(c2 * (k[0] * k[0] + k[1] * k[1] + k[2] * k[2]));
  bad = bad || !(s < 1.0e300);
  return s;
}

// Tangent basis of the unit direction n: t1 the axis of the smallest
// component of n (ties to the later axis) made orthogonal to n, t2 = t1 x n.
WIU_DEV void tangents3(const double n[3], double t1[3], double t2[3]) {
  int e = 2;
  if (fabs(n[1]) < fabs(n[e])) e = 1;
  if (fabs(n[0]) < fabs(n[e])) e = 0;
  const double an = n[e];
  for (int c = 0; c < 3; ++c) t1[c] = (c == e ? 1.0 : 0.0) - an * n[c];
  const double r = rsqrt_(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
  for (int c = 0; c < 3; ++c) t1[c] *= r;
  t2[0] = t1[1] * n[2] - t1[2] * n[1];
  t2[1] = t1[2] * n[0] - t1[0] * n[2];
  t2[2] = t1[0] * n[1] - t1[1] * n[0];
}

// Another split of the midpoint flux at the interpolated state Q with the
// midpoint metric k (Sec. 7; the 3-D forms of the 2-D ones).
//   split 1, Steger-Warming: F+- = R diag(l+-) L Q along n = k/|k| at Q, with
//     l = |k| (q_n - c, q_n, q_n, q_n, q_n + c), l+- = (l +- |l|)/2; the
//     shear rows of L annihilate Q, so only the acoustic and entropy fields
//     contribute;
//   split 2, van Leer: the Mach-number split along n.
WIU_DEV void mid_split_alt3(int split, const double Q[5], const double k[3], int side, double gam, double G[5]) {
  const double kn = sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
  const double rkn = rcp(kn);
  const double n[3] = {k[0] * rkn, k[1] * rkn, k[2] * rkn};
  const double ri = rcp(Q[0]);
  const double V[3] = {Q[1] * ri, Q[2] * ri, Q[3] * ri};
  const double q2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
  const double p = (gam - 1.0) * (Q[4] - 0.5 * Q[0] * q2);
  const double c2 = gam * p * ri;
  const double rc = rsqrt_(c2);
  const double c = c2 * rc;
  const double qn = V[0] * n[0] + V[1] * n[1] + V[2] * n[2];
  if (split == 1) {
    const double H = (Q[4] + p) * ri;
    const double b1 = (gam - 1.0) * (rc * rc);
    const double b2 = 0.5 * b1 * q2;
    const double A = b2 * Q[0] - b1 * (V[0] * Q[1] + V[1] * Q[2] + V[2] * Q[3] - Q[4]);
    const double Bn = rc * (qn * Q[0] - (n[0] * Q[1] + n[1] * Q[2] + n[2] * Q[3]));
    const double l0 = kn * (qn - c), l1 = kn * qn, l4 = kn * (qn + c);
    auto part = [&](double l) { return side == 0 ? 0.5 * (l + fabs(l)) : 0.5 * (l - fabs(l)); };
    const double w0 = part(l0) * 0.5 * (A + Bn), w1 = part(l1) * (Q[0] - A), w4 = part(l4) * 0.5 * (A - Bn);
    G[0] = w0 + w1 + w4;
    for (int a = 0; a < 3; ++a) G[1 + a] = (w0 + w1 + w4) * V[a] + c * n[a] * (w4 - w0);
    G[4] = H * (w0 + w4) + c * qn * (w4 - w0) + 0.5 * q2 * w1;
    return;
  }
  const double M = qn * rc;
  if ((side == 0 && 1.0 <= M) || (side == 1 && M <= -1.0)) {
    flux3(Q, k, gam, G);
    return;
  }
  if ((side == 0 && M <= -1.0) || (side == 1 && 1.0 <= M)) {
    for (int a = 0; a < 5; ++a) G[a] = 0.0;
    return;
  }
  const double sg = side == 0 ? 1.0 : -1.0;
  const double fm = sg * kn * Q[0] * c * (M + sg) * (M + sg) * 0.25;
  const double vt = -qn + sg * 2.0 * c;
  const double e2 = (gam - 1.0) * qn + sg * 2.0 * c;
  G[0] = fm;
  for (int a = 0; a < 3; ++a) G[1 + a] = fm * (V[a] + n[a] * vt / gam);
  G[4] = fm * (e2 * e2 / (2.0 * (gam * gam - 1.0)) + 0.5 * (q2 - qn * qn));
}

// One side of the midpoint k+1/2 (side 0: F+, reference Q_k; side 1: F-,
// reference Q_{k+1}): project the stencil's deviations from the reference
// on the characteristic fields (rows of L for q_n - c, q_n, shear t2, shear
// t1, q_n + c), interpolate each with WENO, map back with R, add the
// reference, then the Lax-Friedrichs half flux with the midpoint metric.
// q(s, c): state at window slot s = 0..7 (nodes k-3 .. k+4).
// With split != 0, Dacc accumulates the other split's difference G - F.
template <int R, bool ZOK = false, class QF>
WIU_DEV void side_flux3(QF q, int side, const double n[3], const double mk[3], double lam, double gam, double eps,
                        int ppm, double F[5], int split = 0, double* Dacc = nullptr) {
  double Qr[5];
  for (int c = 0; c < 5; ++c) Qr[c] = q(3 + side, c);
  double t1[3], t2[3];
  tangents3(n, t1, t2);
  const double gm1 = gam - 1.0;
  const double rr = rcp(Qr[0]);
  const double V[3] = {Qr[1] * rr, Qr[2] * rr, Qr[3] * rr};
  const double q2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
  const double p = gm1 * (Qr[4] - 0.5 * Qr[0] * q2);
  const double c2 = gam * p * rr;
  const double rc = rsqrt_(c2);
  const double c = c2 * rc;
  const double H = (Qr[4] + p) * rr;
  const double qn = V[0] * n[0] + V[1] * n[1] + V[2] * n[2];
  const double qa = V[0] * t2[0] + V[1] * t2[1] + V[2] * t2[2];
  const double qb = V[0] * t1[0] + V[1] * t1[1] + V[2] * t1[2];
  const double b1 = gm1 * (rc * rc);
  const double b2 = 0.5 * b1 * q2;
  // window slots of the stencil in interpolation order (left-biased for side
  // 0, mirrored for side 1); the reference slot has zero deviation
  // r = 2: k-2 .. k+1, r = 3: k-2 .. k+2, r = 4: k-3 .. k+3 (for side 0)
  constexpr int NS = R == 2 ? 4 : (R == 3 ? 5 : 7);
  constexpr int C0 = R == 4 ? 3 : 2;     // index of the reference in that order
  double w[5][NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (s == C0) {
      for (int f = 0; f < 5; ++f) w[f][s] = 0.0;
      continue;
    }
    const int slot = side == 0 ? 3 - C0 + s : 4 + C0 - s;
    double dq[5];
    for (int cc = 0; cc < 5; ++cc) dq[cc] = q(slot, cc) - Qr[cc];
    const double dmV = V[0] * dq[1] + V[1] * dq[2] + V[2] * dq[3];
    const double A = b2 * dq[0] - b1 * (dmV - dq[4]);
    const double Bn = rc * (qn * dq[0] - (n[0] * dq[1] + n[1] * dq[2] + n[2] * dq[3]));
    w[0][s] = 0.5 * (A + Bn);
    w[1][s] = dq[0] - A;
    w[2][s] = t2[0] * dq[1] + t2[1] * dq[2] + t2[2] * dq[3] - qa * dq[0];
    w[3][s] = t1[0] * dq[1] + t1[1] * dq[2] + t1[2] * dq[3] - qb * dq[0];
    w[4][s] = 0.5 * (A - Bn);
  }
  double Wf[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    if constexpr (R == 2) Wf[f] = weno3<ZOK>(w[f][0], w[f][1], w[f][3], eps, ppm);
    else if constexpr (R == 3) Wf[f] = weno5<ZOK>(w[f][0], w[f][1], w[f][3], w[f][4], eps, ppm);
    else Wf[f] = weno7<ZOK>(w[f][0], w[f][1], w[f][2], w[f][4], w[f][5], w[f][6], eps, ppm);
  }
  // Q = Q_ref + R W
  const double s04 = Wf[0] + Wf[4], d40 = Wf[4] - Wf[0];
  const double sum = s04 + Wf[1];
  double r[5];
  r[0] = Qr[0] + sum;
  for (int a = 0; a < 3; ++a) r[1 + a] = Qr[1 + a] + (V[a] * sum + c * n[a] * d40 + t2[a] * Wf[2] + t1[a] * Wf[3]);
  r[4] = Qr[4] + (H * s04 + c * qn * d40 + 0.5 * q2 * Wf[1] + qa * Wf[2] + qb * Wf[3]);
  double E[5];
  flux3(r, mk, gam, E);
  const double sl = side == 0 ? lam : -lam;
  for (int a = 0; a < 5; ++a) F[a] = 0.5 * (E[a] + sl * r[a]);
  if (split != 0) {
    double G[5];
    mid_split_alt3(split, r, mk, side, gam, G);
    for (int a = 0; a < 5; ++a) Dacc[a] += G[a] - F[a];
  }
}

// The same side flux with the interpolation component by component
// (Sec. 2.4): vars 1 conservative, vars 2 primitive (rho, u, v, w, p), on
// deviations from the reference node's values.
template <int R, bool ZOK, class QF>
WIU_DEV void side_flux3_comp(QF q, int side, int vars, const double mk[3], double lam, double gam, double eps,
                             int ppm, double F[5], int split = 0, double* Dacc = nullptr) {
  constexpr int NS = R == 2 ? 4 : (R == 3 ? 5 : 7);
  constexpr int C0 = R == 4 ? 3 : 2;
  auto val = [&](int slot, double V[5]) {
    for (int c = 0; c < 5; ++c) V[c] = q(slot, c);
    if (vars == 2) {
      const double ri = rcp(V[0]);
      const double u = V[1] * ri, v = V[2] * ri, w = V[3] * ri;
      V[4] = (gam - 1.0) * (V[4] - 0.5 * (V[1] * u + V[2] * v + V[3] * w));
      V[1] = u; V[2] = v; V[3] = w;
    }
  };
  double Vr[5];
  val(3 + side, Vr);
  double w[5][NS];
#pragma unroll
  for (int s_ = 0; s_ < NS; ++s_) {
    if (s_ == C0) {
      for (int f = 0; f < 5; ++f) w[f][s_] = 0.0;
      continue;
    }
    const int slot = side == 0 ? 3 - C0 + s_ : 4 + C0 - s_;
    double V[5];
    val(slot, V);
    for (int f = 0; f < 5; ++f) w[f][s_] = V[f] - Vr[f];
  }
  double Vm[5];
#pragma unroll
  for (int f = 0; f < 5; ++f) {
    double W;
    if constexpr (R == 2) W = weno3<ZOK>(w[f][0], w[f][1], w[f][3], eps, ppm);
    else if constexpr (R == 3) W = weno5<ZOK>(w[f][0], w[f][1], w[f][3], w[f][4], eps, ppm);
    else W = weno7<ZOK>(w[f][0], w[f][1], w[f][2], w[f][4], w[f][5], w[f][6], eps, ppm);
    Vm[f] = Vr[f] + W;
  }
  double r[5];
  if (vars == 2) {
    r[0] = Vm[0];
    for (int a = 0; a < 3; ++a) r[1 + a] = Vm[0] * Vm[1 + a];
    r[4] = Vm[4] / (gam - 1.0) + 0.5 * Vm[0] * (Vm[1] * Vm[1] + Vm[2] * Vm[2] + Vm[3] * Vm[3]);
  } else {
    for (int a = 0; a < 5; ++a) r[a] = Vm[a];
  }
  double E[5];
  flux3(r, mk, gam, E);
  const double sl = side == 0 ? lam : -lam;
  for (int a = 0; a < 5; ++a) F[a] = 0.5 * (E[a] + sl * r[a]);
  if (split != 0) {
    double G[5];
    mid_split_alt3(split, r, mk, side, gam, G);
    for (int a = 0; a < 5; ++a) Dacc[a] += G[a] - F[a];
  }
}

// ===========================================================================
// Direction passes.
// ===========================================================================
struct S3Args {
  Dims3 d;
  const double* U;                 // state the fluxes are built from
  const double* M;
  const unsigned long long* lam;   // line maxima: xi lines [ny nz], eta [nx nz], zeta [nx ny]
  unsigned long long* nlam;        // xi pass of an RK stage: the next stage's maxima (or null)
  unsigned long long* ncfl;        // with nlam, when set: the next state's CFL maximum per j [ny]
  double gamma, alpha, eps;
  int ppm;
  int vars;                        // WIU_VARS_* (interpolation variables)
  double ah;                       // free parameter of the one-midpoint schemes
  int weights;                     // WIU_WEIGHTS_*
  int split;                       // WIU_SPLIT_* of the leading midpoint flux
  double* Racc;                    // accumulated flux differences [5][np]
  double* out;                     // dU/dt (mode 2) or the new stage state (mode 3)
  const double* U0;                // RK base state
  const double* dt;                // device time step
  double ca, cb;
  int* status;
  // rules beyond the sides of non-periodic directions (x lo .. z hi):
  // WIU_SIDE_TRANSMISSIVE, _WALL or _FIXED with the state `fixed`
  int side[6];
  double fixed[6][5];
};

WIU_DEV long long lam_off(const Dims3& d, int D) {
  return D == 0 ? 0 : (D == 1 ? (long long)d.n[1] * d.n[2] : (long long)d.n[1] * d.n[2] + (long long)d.n[0] * d.n[2]);
}
WIU_DEV long long line3(const Dims3& d, int D, const int p[3]) {
  return D == 0 ? (long long)p[2] * d.n[1] + p[1] : (D == 1 ? (long long)p[2] * d.n[0] + p[0]
                                                             : (long long)p[1] * d.n[0] + p[0]);
}

WIU_DEV bool tag3_ok(const Dims3& d, const double* M, int scheme, double ah) {
  const double* tag = M + NP3 * d.mplane;
  return tag[0] == TAG_MAGIC3 && tag[1] == (double)scheme && tag[2] == (double)d.n[0] &&
         tag[3] == (double)d.n[1] && tag[4] == (double)d.n[2] &&
         tag[5] == (double)(d.bc[0] + 2 * d.bc[1] + 4 * d.bc[2]) && tag[6] == ah;
}

// LDS of a 3-D sweep tile: NA items along the line by NB lines.  Per item
// the nodal flux E^ and both midpoint side fluxes (15 values; f+- are rebuilt
// from E^ and the staged state); the states of items k - QL .. k + QL + 1.
// Lanes of a wave touch consecutive words: line-major for xi tiles (lanes
// along the line), position-major otherwise (lanes across lines along i).
template <int SC, int DIR, int NA, int NB, bool OPT = false> struct Sweep3Lds {
  static constexpr int QL = Range<SC>::QL;
  static constexpr int NQ = NA + 2 * QL + 1;
  // with the options, 5 more per item: D, the difference another midpoint
  // split makes to H at the item's midpoint
  static constexpr int NREC = OPT ? 20 : 15;
  double sh[NREC][NA * NB];
  double sq[5][NB * NQ];
  double red[DIR == 0 ? NA * NB : 1];  // xi tiles: the next stage's eta speeds, reduced over the lines
  static WIU_DEV int si(int tb, int ta) { return DIR == 0 ? tb * NA + ta : ta * NB + tb; }
  static WIU_DEV int qi(int tb, int pos) { return DIR == 0 ? tb * NQ + pos : pos * NB + tb; }
};

// One direction pass.  A workgroup owns NB lines (consecutive j for xi,
// consecutive i otherwise, at one value of the remaining index) and a
// segment of OUT = NA - EXTRA output nodes along them: it stages the states
// of the segment (boundary rule applied) in LDS, computes one item per lane
// (nodal flux at k and both side fluxes at k + 1/2), then the first OUT
// lanes of each line form H_{i+1/2} - H_{i-1/2} and, by `mode`: 0 Racc = R;
// 1 Racc += R; 2 dU/dt = -(Racc + R)/J^{-1}; 3 the RK stage
// U_out = ca U0 + cb (U + dt dU/dt).  Four block-wide barriers on every path
// (five in an xi pass that accumulates the next stage's maxima).
// OPT: compiled with the scheme options (a.vars, a.ah, a.weights); without
// it the sweep runs the paper's configuration and carries no code for them.
template <int SC, int DIR, int NA, int NB, bool OPT>
__global__ void __launch_bounds__(NA * NB) s3_sweep_kernel(S3Args a, int mode) {
  __shared__ Sweep3Lds<SC, DIR, NA, NB, OPT> L;
  using R_ = Range<SC>;
  using LT = Sweep3Lds<SC, DIR, NA, NB, OPT>;
  constexpr int OUT = NA - R_::EXTRA, QL = R_::QL, NQ = LT::NQ, NT = NA * NB;
  const Dims3& d = a.d;
  const double ah = OPT ? a.ah : 1.0;
  const int ppm = OPT && a.weights != 0 ? 2 : a.ppm;  // 2: WENO-Z weights
  const int split = OPT ? a.split : 0;                 // another split of the leading midpoint flux
  if (!tag3_ok(d, a.M, SC, ah)) {  // block-uniform
    if (threadIdx.x == 0 && threadIdx.y == 0) atomicOr(a.status, ST_SCHEME);
    return;
  }
  const int n = d.n[DIR];
  const int nac = DIR == 0 ? d.n[1] : d.n[0];   // grouped index across the lines
  const int nseg = (n + OUT - 1) / OUT, ngrp = (nac + NB - 1) / NB;
  // XCD-aware order: consecutive logical tiles share an XCD's L2; for eta
  // and zeta the line group (along i) varies fastest, so neighbouring tiles
  // read the same rows and pages of the k-planes
  const long long tile = xcd_remap(blockIdx.x, gridDim.x);
  int seg, grp, cb;
  if (DIR == 0) {
    seg = (int)(tile % nseg);
    const long long rest = tile / nseg;
    grp = (int)(rest % ngrp); cb = (int)(rest / ngrp);
  } else {
    grp = (int)(tile % ngrp);
    const long long rest = tile / ngrp;
    seg = (int)(rest % nseg); cb = (int)(rest / nseg);
  }
  const int ta = DIR == 0 ? threadIdx.x : threadIdx.y;           // along
  const int tb = DIR == 0 ? threadIdx.y : threadIdx.x;           // across
  const int la = grp * NB + tb;
  const bool live = la < nac;
  const int o0 = seg * OUT;
  const int out = min(OUT, n - o0);
  const int k = o0 + R_::LO + ta;
  auto node = [&](int kk, int line, int p[3]) {
    if (DIR == 0) { p[0] = kk; p[1] = line; p[2] = cb; }
    else if (DIR == 1) { p[0] = line; p[1] = kk; p[2] = cb; }
    else { p[0] = line; p[1] = cb; p[2] = kk; }
  };
  // stage the states of the segment: each thread's elements (NIT at most)
  // are all loaded before any is stored, so their latencies overlap; a
  // segment whose window lies inside the line needs no index mapping
  {
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int k0 = o0 + R_::LO - QL;
    const bool inside = k0 >= 0 && k0 + NQ <= n;  // uniform over the block
    constexpr int NIT = (NQ * NB + NT - 1) / NT;
    double Qs[NIT][5];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = tid + it * NT;
      if (e >= NQ * NB) break;
      const int pos = DIR == 0 ? e % NQ : e / NB;
      const int lb = DIR == 0 ? e / NQ : e % NB;
      const int ln = grp * NB + lb;
      double* Qv = Qs[it];
      if (ln >= nac) continue;
      if (inside) {
        int p[3];
        node(k0 + pos, ln, p);
        const long long o = u3idx(d, p[0], p[1], p[2]);
#pragma unroll
        for (int c = 0; c < 5; ++c) Qv[c] = a.U[c * d.np + o];
      } else {
        // beyond a non-periodic end the side's rule: transmissive (boundary
        // node), reflecting wall (mirror node, momentum along the boundary
        // node's unit metric direction reversed) or a fixed state
        const int kr = k0 + pos;
        const bool out_of = d.bc[DIR] != WIU_BC_PERIODIC && (kr < 0 || kr >= n);
        const int sd = 2 * DIR + (kr < 0 ? 0 : 1);
        const int rule = out_of ? a.side[sd] : WIU_SIDE_TRANSMISSIVE;
        if (rule == WIU_SIDE_FIXED) {
#pragma unroll
          for (int c = 0; c < 5; ++c) Qv[c] = a.fixed[sd][c];
        } else {
          const int kb = kr < 0 ? 0 : n - 1;
          const int kk = rule == WIU_SIDE_WALL ? min(max(2 * kb - kr, 0), n - 1) : bc_index(kr, n, d.bc[DIR]);
          int p[3];
          node(kk, ln, p);
          const long long o = u3idx(d, p[0], p[1], p[2]);
#pragma unroll
          for (int c = 0; c < 5; ++c) Qv[c] = a.U[c * d.np + o];
          if (rule == WIU_SIDE_WALL) {
            node(kb, ln, p);
            const long long mo = m3idx(d, p[0], p[1], p[2]);
            double nv[3];
            for (int c = 0; c < 3; ++c) nv[c] = a.M[(3 * DIR + c) * d.mplane + mo];
            const double rn = rsqrt_(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
            const double mn = (Qv[1] * nv[0] + Qv[2] * nv[1] + Qv[3] * nv[2]) * rn;
            for (int c = 0; c < 3; ++c) Qv[1 + c] -= 2.0 * mn * (nv[c] * rn);
          }
        }
      }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int e = tid + it * NT;
      if (e >= NQ * NB) break;
      const int pos = DIR == 0 ? e % NQ : e / NB;
      const int lb = DIR == 0 ? e / NQ : e % NB;
      if (grp * NB + lb >= nac) continue;
#pragma unroll
      for (int c = 0; c < 5; ++c) L.sq[c][LT::qi(lb, pos)] = Qs[it][c];
    }
  }
  __syncthreads();
  double lam = 0.0;
  if (live) {
    int p[3];
    node(0, la, p);
    lam = a.alpha * __longlong_as_double((long long)a.lam[lam_off(d, DIR) + line3(d, DIR, p)]);
  }
  const double gam = a.gamma;
  const int slot = LT::si(tb, ta);
  const bool need_node = live && k >= o0 + Traits<SC>::NLO && k < o0 + out + Traits<SC>::NHI;
  const bool need_mid = live && k >= o0 + Traits<SC>::MLO && k < o0 + out + Traits<SC>::MHI;
  auto kn = [&](int kk, double v[3]) {
    int p[3];
    node(kk, la, p);
    const long long o = m3idx(d, p[0], p[1], p[2]);
    for (int c = 0; c < 3; ++c) v[c] = a.M[(3 * DIR + c) * d.mplane + o];
  };
  if (need_node) {
    double Q[5], k0v[3], E[5];
    for (int c = 0; c < 5; ++c) Q[c] = L.sq[c][LT::qi(tb, ta + QL)];
    kn(k, k0v);
    flux3(Q, k0v, gam, E);
    for (int c = 0; c < 5; ++c) L.sh[c][slot] = E[c];
  }
  if (need_mid) {
    double k0v[3], k1v[3], mk[3], nv[3];
    kn(k, k0v);
    kn(k + 1, k1v);
    int p[3];
    node(k, la, p);
    const long long o = m3idx(d, p[0], p[1], p[2]);
    for (int c = 0; c < 3; ++c) {
      mk[c] = a.M[(10 + 3 * DIR + c) * d.mplane + o];
      nv[c] = 0.5 * (k0v[c] + k1v[c]);
    }
    const double rn = rsqrt_(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    for (int c = 0; c < 3; ++c) nv[c] *= rn;
    // window slot s = 0..7 is node k - 3 + s
    auto q = [&](int s_, int c) { return L.sq[c][LT::qi(tb, ta + QL - 3 + s_)]; };
    double D[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      asm volatile("" ::: "memory");  // one side at a time (register pressure)
      double F[5];
      if (OPT && a.vars != 0)
        side_flux3_comp<Traits<SC>::R, OPT>(q, side, a.vars, mk, lam, gam, a.eps, ppm, F, split, D);
      else
        side_flux3<Traits<SC>::R, OPT>(q, side, nv, mk, lam, gam, a.eps, ppm, F, split, D);
      for (int c = 0; c < 5; ++c) L.sh[5 + 5 * side + c][slot] = F[c];
    }
    if constexpr (OPT) {
      for (int c = 0; c < 5; ++c) L.sh[LT::NREC - 5 + c][slot] = D[c];
    }
  }
  // epilogue operands of this lane's output node, issued before the
  // barriers so that their latency overlaps them and the flux difference
  const bool act = live && ta < out;
  const int i = o0 + ta;
  double xr[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, x0[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, jv = 1.0;
  long long t = 0;
  if (act) {
    int p[3];
    node(i, la, p);
    t = u3idx(d, p[0], p[1], p[2]);
    if (mode != 0) {
#pragma unroll
      for (int c = 0; c < 5; ++c) xr[c] = a.Racc[c * d.np + t];
    }
    if (mode >= 2) jv = a.M[9 * d.mplane + m3idx(d, p[0], p[1], p[2])];
    if (mode == 3 && a.ca != 0.0) {
#pragma unroll
      for (int c = 0; c < 5; ++c) x0[c] = a.U0[c * d.np + t];
    }
  }
  // nodal metrics of all three directions, for the next stage's maxima
  double km[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) km[c] = 0.0;
  const bool fused = DIR == 0 && mode == 3 && a.nlam != nullptr;  // uniform over the grid
  if (fused && act) {
    int p[3];
    node(i, la, p);
    const long long mo = m3idx(d, p[0], p[1], p[2]);
#pragma unroll
    for (int c = 0; c < 9; ++c) km[c] = a.M[c * d.mplane + mo];
  }
  __syncthreads();
  constexpr int S = DIR == 0 ? 1 : NB;
  // H_{k+1/2} once per item, for the midpoints k + 1/2 of k in [o0 - 1,
  // o0 + out), into the item's nodal-flux slots once every record is read;
  // each midpoint's H is then read by both of its nodes (exact telescoping)
  {
    const bool hact = live && k >= o0 - 1 && k < o0 + out;
    double Hk[5];
    if (hact) {
      const int qs = LT::qi(tb, ta + QL);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const double* e = &L.sh[c][slot];
        const double* qv = &L.sq[c][qs];
        const double* gp = &L.sh[5 + c][slot];
        const double* gm = &L.sh[10 + c][slot];
        if constexpr (SC == 3) {
          Hk[c] = hsum52(lam, [&](int m) { return e[m * S]; }, [&](int m) { return qv[m * S]; },
                         [&](int m) { return gp[m * S]; }, [&](int m) { return gm[m * S]; });
        } else {
          auto fp = [&](int kk) { return 0.5 * (e[(kk - k) * S] + lam * qv[(kk - k) * S]); };
          auto fm = [&](int kk) { return 0.5 * (e[(kk - k) * S] - lam * qv[(kk - k) * S]); };
          auto Fp = [&](int kk) { return gp[(kk - k) * S]; };
          auto Fm = [&](int kk) { return gm[(kk - k) * S]; };
          Hk[c] = hflux<SC>(k, ah, fp, fm, Fp, Fm);
        }
        if constexpr (OPT) {
          if (split != 0) Hk[c] += L.sh[LT::NREC - 5 + c][slot];
        }
      }
    }
    __syncthreads();
    if (hact) {
#pragma unroll
      for (int c = 0; c < 5; ++c) L.sh[c][slot] = Hk[c];
    }
    __syncthreads();
  }
  if constexpr (DIR == 0) {
    if (fused) {
      // RK stage with the next stage's line maxima (Sec. 2.3), every lane
      // taking part in the reductions: a wave is one line (j, k) along i, the
      // tile's NB lines are consecutive j at one k.  Wave speeds as in the
      // separate maxima pass (same routine, clamped at zero), so the maxima
      // are bit-identical to it.
      static_assert(NA == 64, "xi tile: one line per wave");
      double sx = 0.0, se = 0.0, sz = 0.0;
      bool bad = false;
      if (act) {
        const int hs = LT::si(tb, i - (o0 + R_::LO));
        const double rj = -rcp(jv);
        const double dt = a.dt[0];
        const int pq = LT::qi(tb, ta - R_::LO + QL);
        double Qn[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          const double Lv = (xr[c] + (L.sh[c][hs] - L.sh[c][hs - S])) * rj;
          const double us = L.sq[c][pq] + dt * Lv;
          Qn[c] = a.ca == 0.0 ? a.cb * us : a.ca * x0[c] + a.cb * us;
          a.out[c * d.np + t] = Qn[c];
        }
        double sp[3];
#pragma unroll
        for (int D = 0; D < 3; ++D) {
          const double kk[3] = {km[3 * D], km[3 * D + 1], km[3 * D + 2]};
          bool b;
          sp[D] = speed3(Qn, kk, a.gamma, b);
          bad |= b;
        }
        sx = fmax(0.0, sp[0]);
        se = fmax(0.0, sp[1]);
        sz = fmax(0.0, sp[2]);
      }
      if (bad) atomicOr(a.status, ST_NONPHYS);
      unsigned long long* lx = a.nlam;
      unsigned long long* le = lx + (long long)d.n[1] * d.n[2];
      unsigned long long* lz = le + (long long)d.n[0] * d.n[2];
      if (a.ncfl) {
        // CFL maximum, formed as the separate maxima pass forms it, in
        // partial maxima per j: the tiles of one k plane run together, so
        // their atomics spread over ny addresses
        double cf = act ? (sx + se + sz) / jv : 0.0;
        for (int off = 32; off > 0; off >>= 1) cf = fmax(cf, __shfl_xor(cf, off, 64));
        if (ta == 0 && live) atomicMax(&a.ncfl[la], (unsigned long long)__double_as_longlong(cf));
      }
      // xi lines (j, k): reduce over the wave (along i)
      for (int off = 32; off > 0; off >>= 1) sx = fmax(sx, __shfl_xor(sx, off, 64));
      if (ta == 0 && live) atomicMax(&lx[(long long)cb * d.n[1] + la], (unsigned long long)__double_as_longlong(sx));
      // zeta lines (i, j): one node of the tile each
      if (act) atomicMax(&lz[(long long)la * d.n[0] + i], (unsigned long long)__double_as_longlong(sz));
      // eta lines (i, k): reduce over the tile's lines
      L.red[LT::si(tb, ta)] = se;
      __syncthreads();
      if (tb == 0 && ta < out) {
        double m = L.red[LT::si(0, ta)];
#pragma unroll
        for (int l = 1; l < NB; ++l) m = fmax(m, L.red[LT::si(l, ta)]);
        atomicMax(&le[(long long)cb * d.n[0] + i], (unsigned long long)__double_as_longlong(m));
      }
      return;
    }
  }
  if (!act) return;
  const int hs = LT::si(tb, i - (o0 + R_::LO));
  double Rv[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) Rv[c] = L.sh[c][hs] - L.sh[c][hs - S];
  if (mode == 0) {
    for (int c = 0; c < 5; ++c) a.Racc[c * d.np + t] = Rv[c];
    return;
  }
  if (mode == 1) {
    for (int c = 0; c < 5; ++c) a.Racc[c * d.np + t] = xr[c] + Rv[c];
    return;
  }
  const double rj = -rcp(jv);
  if (mode == 2) {
    for (int c = 0; c < 5; ++c) a.out[c * d.np + t] = (xr[c] + Rv[c]) * rj;
    return;
  }
  // the stage state at the output node is the staged tile entry (an interior
  // node, untouched by the side rules); U0 is not read when its coefficient
  // is zero (first stage)
  const double dt = a.dt[0];
  const int pq = LT::qi(tb, ta - R_::LO + QL);
  for (int c = 0; c < 5; ++c) {
    const double Lv = (xr[c] + Rv[c]) * rj;
    const double us = L.sq[c][pq] + dt * Lv;
    a.out[c * d.np + t] = a.ca == 0.0 ? a.cb * us : a.ca * x0[c] + a.cb * us;
  }
}

// Line maxima of the wave speeds in all three directions and the CFL
// maximum.  One thread per (i, j) column walks a chunk of KC3 nodes along k
// (the third grid dimension covers the chunks): zeta lines reduce in
// registers over the chunk, xi lines across the wave (threads along i), eta
// lines by atomics.
constexpr int KC3 = 16;
__global__ void __launch_bounds__(256) w3_max_kernel(Dims3 d, const double* __restrict__ U,
                                                     const double* __restrict__ M, double gam,
                                                     unsigned long long* __restrict__ lam, int* __restrict__ status) {
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
  const bool act = i < d.n[0] && j < d.n[1];
  unsigned long long* lx = lam;
  unsigned long long* le = lam + (long long)d.n[1] * d.n[2];
  unsigned long long* lz = le + (long long)d.n[0] * d.n[2];
  unsigned long long* cflm = lz + (long long)d.n[0] * d.n[1];
  double smz = 0.0, cm = 0.0;
  bool bad = false;
  const int k0 = blockIdx.z * KC3, k1 = min(k0 + KC3, d.n[2]);  // uniform over the block
  for (int k = k0; k < k1; ++k) {
    double sx = 0.0;
    if (act) {
      const long long o = u3idx(d, i, j, k), mo = m3idx(d, i, j, k);
      double Q[5];
      for (int c = 0; c < 5; ++c) Q[c] = U[c * d.np + o];
      double s[3];
      for (int D = 0; D < 3; ++D) {
        const double kk[3] = {M[(3 * D) * d.mplane + mo], M[(3 * D + 1) * d.mplane + mo],
                              M[(3 * D + 2) * d.mplane + mo]};
        bool b;
        s[D] = speed3(Q, kk, gam, b);
        bad |= b;
      }
      sx = fmax(0.0, s[0]);
      atomicMax(&le[(long long)k * d.n[0] + i], (unsigned long long)__double_as_longlong(fmax(0.0, s[1])));
      smz = fmax(smz, s[2]);
      cm = fmax(cm, (sx + fmax(0.0, s[1]) + fmax(0.0, s[2])) / M[9 * d.mplane + mo]);
    }
    double v = sx;
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0 && j < d.n[1])
      atomicMax(&lx[(long long)k * d.n[1] + j], (unsigned long long)__double_as_longlong(v));
  }
  if (act) atomicMax(&lz[(long long)j * d.n[0] + i], (unsigned long long)__double_as_longlong(smz));
  for (int off = 32; off > 0; off >>= 1) cm = fmax(cm, __shfl_xor(cm, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(cflm, (unsigned long long)__double_as_longlong(cm));
  if (bad) atomicOr(status, ST_NONPHYS);
}

}  // namespace wiu

using namespace wiu;

namespace {

constexpr size_t A3 = 256;
size_t al3(size_t v) { return (v + A3 - 1) / A3 * A3; }

bool grid3_ok(const wiu_grid3* g) {
  if (!g) return false;
  const int n[3] = {g->nx, g->ny, g->nz};
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1 || g->bc[a] < 0 || g->bc[a] > 1) return false;
    if (g->bc[a] == WIU_BC_TRANSMISSIVE && n[a] < 2) return false;
    if (g->bc[a] == WIU_BC_PERIODIC && !(g->period[a] > 0.0 && g->period[a] < 1.0e300)) return false;
    if (n[a] > 4096) return false;
    if (g->bc[a] == WIU_BC_PERIODIC) continue;
    for (int e = 2 * a; e < 2 * a + 2; ++e) {
      if (g->side[e] < WIU_SIDE_TRANSMISSIVE || g->side[e] > WIU_SIDE_FIXED) return false;
      if (g->side[e] == WIU_SIDE_FIXED) {
        const double* q = g->fixed[e];
        if (!(q[0] > 0.0) || !(q[0] < 1.0e300)) return false;
        const double p = q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];  // (gamma - 1) p
        if (!(p > 0.0) || !(p < 1.0e300)) return false;
      }
    }
  }
  return (long long)n[0] * n[1] * n[2] <= (1LL << 31);
}

Dims3 dims3(const wiu_grid3* g) {
  Dims3 d;
  d.n[0] = g->nx; d.n[1] = g->ny; d.n[2] = g->nz;
  for (int a = 0; a < 3; ++a) { d.bc[a] = g->bc[a]; d.L[a] = g->period[a]; }
  d.np = (long long)g->nx * g->ny * g->nz;
  d.mp[0] = g->nx + 2 * GHOST; d.mp[1] = g->ny + 2 * GHOST;
  d.mplane = (long long)d.mp[0] * d.mp[1] * (g->nz + 2 * GHOST);
  return d;
}

// Workspace: [status | line maxima, two buffers (this and the next RK
// stage) | dt | big area], the big area holding either the metric scratch
// (inner derivatives, nodal band) or the stepping buffers (Racc, U1, U2).
struct Ws3 {
  size_t lam, lam2, dt, big, metric_dx, metric_t, racc, u1, u2, total;
  long long nlam;
};

Ws3 ws3(const wiu_grid3* g) {
  const Dims3 d = dims3(g);
  Ws3 w;
  w.nlam = (long long)g->ny * g->nz + (long long)g->nx * g->nz + (long long)g->nx * g->ny + 1;
  w.lam = A3;
  // a maxima set: the line maxima and the CFL maximum (nlam entries), then
  // the partial CFL maxima per j [ny] that several steps per call carry
  const size_t set = al3((w.nlam + g->ny) * 8);
  w.lam2 = w.lam + set;  // the next RK stage's maxima
  w.dt = w.lam2 + set;
  w.big = w.dt + A3;
  const int B = GHOST + METRIC_REACH, E = B + 8;  // the widest band (Eq. 2.6)
  const size_t dxb = al3(9 * (size_t)(g->nx + 2 * E) * (g->ny + 2 * E) * (g->nz + 2 * E) * 8);
  const size_t tb = al3(10 * (size_t)(g->nx + 2 * B) * (g->ny + 2 * B) * (g->nz + 2 * B) * 8);
  w.metric_dx = w.big;
  w.metric_t = w.big + dxb;
  w.racc = w.big;
  w.u1 = w.racc + al3(5 * (size_t)d.np * 8);
  w.u2 = w.u1 + al3(5 * (size_t)d.np * 8);
  const size_t step_end = w.u2 + al3(5 * (size_t)d.np * 8);
  const size_t met_end = w.metric_t + tb;
  w.total = step_end > met_end ? step_end : met_end;
  return w;
}

bool alpha3_ok(int scheme, double a) {
  return a > 0.0 && a < 1.0e300 && (a == 1.0 || scheme == WIU_3_1MP || scheme == WIU_5_1MP || scheme == WIU_7_1MP);
}

bool params3_ok(const wiu_params* p, int scheme) {
  return p && p->gamma > 1.0 && p->alpha_lf > 0.0 && p->eps >= 0.0 && (p->ppm == 0 || p->ppm == 1) &&
         p->vars >= WIU_VARS_CHARACTERISTIC && p->vars <= WIU_VARS_PRIMITIVE && alpha3_ok(scheme, p->alpha_h) &&
         (p->weights == WIU_WEIGHTS_JS || p->weights == WIU_WEIGHTS_Z) && p->split >= WIU_SPLIT_LF &&
         p->split <= WIU_SPLIT_VL;
}

void options3(const wiu_params* p, S3Args& a) {
  a.vars = p->vars; a.ah = p->alpha_h; a.weights = p->weights; a.split = p->split;
}

void sides3(const wiu_grid3* g, S3Args& a) {
  for (int e = 0; e < 6; ++e) {
    a.side[e] = g->bc[e / 2] == WIU_BC_PERIODIC ? WIU_SIDE_TRANSMISSIVE : g->side[e];
    for (int c = 0; c < 5; ++c) a.fixed[e][c] = g->fixed[e][c];
  }
}

dim3 lin_grid(long long n) { return dim3((unsigned)((n + 255) / 256)); }

// Tile shapes: xi 64 items x 4 lines (lanes along the line, one line per
// wave), eta and zeta 32 items x 8 lines (lanes across the lines, along i).
template <int SC, int DIR, int NA, int NB, bool OPT>
hipError_t launch_sweep3_t(const S3Args& a, int mode, hipStream_t st) {
  constexpr int OUT = NA - Range<SC>::EXTRA;
  const int n = a.d.n[DIR];
  const int nac = DIR == 0 ? a.d.n[1] : a.d.n[0];
  const int nb = DIR == 2 ? a.d.n[1] : a.d.n[2];
  const long long tiles = (long long)((n + OUT - 1) / OUT) * ((nac + NB - 1) / NB) * nb;
  const dim3 block = DIR == 0 ? dim3(NA, NB) : dim3(NB, NA);
  void* h = prof_open(WIU_K_SWEEP3, st);
  hipLaunchKernelGGL((s3_sweep_kernel<SC, DIR, NA, NB, OPT>), dim3((unsigned)tiles), block, 0, st, a, mode);
  prof_close(h);
  return hipGetLastError();
}

template <int SC, bool OPT>
hipError_t launch_pass3_o(const S3Args& a, int D, int mode, hipStream_t st) {
  if (D == 0) return launch_sweep3_t<SC, 0, 64, 4, OPT>(a, mode, st);
  if (D == 1) return launch_sweep3_t<SC, 1, 32, 8, OPT>(a, mode, st);
  return launch_sweep3_t<SC, 2, 32, 8, OPT>(a, mode, st);
}

// the options kernels only when an option is in use
template <int SC>
hipError_t launch_pass3(const S3Args& a, int D, int mode, hipStream_t st) {
  if (a.vars != 0 || a.ah != 1.0 || a.weights != 0 || a.split != 0) return launch_pass3_o<SC, true>(a, D, mode, st);
  return launch_pass3_o<SC, false>(a, D, mode, st);
}

hipError_t pass3(int scheme, const S3Args& a, int D, int mode, hipStream_t st) {
  switch (scheme) {
    case 0: return launch_pass3<0>(a, D, mode, st);
    case 1: return launch_pass3<1>(a, D, mode, st);
    case 2: return launch_pass3<2>(a, D, mode, st);
    case 3: return launch_pass3<3>(a, D, mode, st);
    case 4: return launch_pass3<4>(a, D, mode, st);
    case 5: return launch_pass3<5>(a, D, mode, st);
    case 6: return launch_pass3<6>(a, D, mode, st);
    case 7: return launch_pass3<7>(a, D, mode, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t maxima3(const Dims3& d, const double* U, const double* M, double gam, unsigned long long* lam,
                   long long nlam, int* status, hipStream_t st) {
  if (launch_fill_u64(lam, nlam, st) != hipSuccess) return hipErrorUnknown;
  hipLaunchKernelGGL(w3_max_kernel, dim3((d.n[0] + 63) / 64, (d.n[1] + 3) / 4, (d.n[2] + KC3 - 1) / KC3), dim3(256),
                     0, st, d, U, M, gam, lam, status);
  return hipGetLastError();
}

int rc3(hipError_t e) { return e == hipSuccess ? WIU_OK : WIU_EHIP; }

}  // namespace

// nsteps TVD-RK3 steps; with cfl > 0 each at the CFL time step of its state,
// written to dt[step] before the stages read it, otherwise all at the device
// scalar *dt, only read.  Only the first step has a separate maxima pass: the
// xi pass of each stage accumulates the next stage's maxima (that of the last
// stage, for the next step, also the partial CFL maxima per j).
static int rk3_3d(const wiu_grid3* g, int scheme, const wiu_params* p, double* U, const double* M, double cfl, double* dt,
           void* ws, wiu_stream_t stream, int nsteps = 1) {
  if (!grid3_ok(g) || scheme < 0 || scheme > 7 || !params3_ok(p, scheme) || !U || !M || !dt || !ws || nsteps < 1)
    return WIU_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const Dims3 d = dims3(g);
  const Ws3 w = ws3(g);
  char* base = (char*)ws;
  double* U1 = (double*)(base + w.u1);
  double* U2 = (double*)(base + w.u2);
  S3Args a;
  a.nlam = nullptr;
  a.ncfl = nullptr;
  a.d = d; a.M = M; a.lam = (unsigned long long*)(base + w.lam);
  a.gamma = p->gamma; a.alpha = p->alpha_lf; a.eps = p->eps; a.ppm = p->ppm;
  a.Racc = (double*)(base + w.racc);
  a.U0 = U; a.status = (int*)base;
  sides3(g, a);
  options3(p, a);
  // U1 = U + dt L(U); U2 = 3/4 U + 1/4 (U1 + dt L(U1)); U = 1/3 U + 2/3 (U2 + dt L(U2))
  const double* src[3] = {U, U1, U2};
  double* dst[3] = {U1, U2, U};
  const double ca[3] = {0.0, 0.75, 1.0 / 3.0}, cb[3] = {1.0, 0.25, 2.0 / 3.0};
  // two maxima sets: sa holds the current state's, sb receives the next
  // stage's; the first step's come from a separate pass
  unsigned long long* sa = (unsigned long long*)(base + w.lam);
  unsigned long long* sb = (unsigned long long*)(base + w.lam2);
  if (maxima3(d, U, M, p->gamma, sa, w.nlam, a.status, st) != hipSuccess) return WIU_EHIP;
  for (int step = 0; step < nsteps; ++step) {
    double* dts = cfl > 0.0 ? dt + step : dt;
    if (cfl > 0.0) {
      const hipError_t e = step == 0 ? launch_cfl_dt(sa + w.nlam - 1, cfl, dts, st)
                                     : launch_cfl_dt_lines(sa + w.nlam, d.n[1], cfl, dts, st);
      if (e != hipSuccess) return WIU_EHIP;
    }
    a.dt = dts;
    for (int s = 0; s < 3; ++s) {
      a.U = src[s]; a.out = dst[s]; a.ca = ca[s]; a.cb = cb[s];
      a.lam = s == 1 ? sb : sa;  // the maxima of U, U1, U2
      unsigned long long* next = s == 0 ? sb : (s == 1 ? sa : (step + 1 < nsteps ? sb : nullptr));
      const bool with_cfl = s == 2 && next;
      if (next && launch_fill_u64(next, w.nlam + (with_cfl ? d.n[1] : 0), st) != hipSuccess) return WIU_EHIP;
      for (int q = 0; q < 3; ++q) {  // zeta, eta, then xi, which writes the stage state
        const int D = 2 - q;
        a.nlam = D == 0 ? next : nullptr;
        a.ncfl = D == 0 && with_cfl ? next + w.nlam : nullptr;
        if (pass3(scheme, a, D, q == 0 ? 0 : (q == 1 ? 1 : 3), st) != hipSuccess) return WIU_EHIP;
      }
    }
    std::swap(sa, sb);
  }
  return WIU_OK;
}

extern "C" {

size_t wiu3_metrics_size(const wiu_grid3* g) {
  if (!grid3_ok(g)) return 0;
  return ((size_t)NP3 * dims3(g).mplane + 8) * sizeof(double);
}

size_t wiu3_workspace_bytes(const wiu_grid3* g) { return grid3_ok(g) ? ws3(g).total : 0; }

int wiu3_metrics(const wiu_grid3* g, int scheme, int jform, const wiu_params* p, const double* x, const double* y,
                 const double* z, double* M, void* ws, wiu_stream_t stream) {
  const double ah = p ? p->alpha_h : 1.0;
  if (!grid3_ok(g) || scheme < 0 || scheme > 7 || (jform != 5 && jform != 6) || !alpha3_ok(scheme, ah) || !x ||
      !y || !z || !M || !ws)
    return WIU_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const Dims3 d = dims3(g);
  const Ws3 w = ws3(g);
  char* base = (char*)ws;
  double* Dx = (double*)(base + w.metric_dx);
  double* T = (double*)(base + w.metric_t);
  int* status = (int*)base;
  const MetricStencil ms = metric_stencil(scheme, ah);
  const int B = jform == 6 ? GHOST + METRIC_REACH : metric_band(scheme), E = B + 8;
  Coord3 X{{x, y, z}};
  const long long ND = (long long)(d.n[0] + 2 * E) * (d.n[1] + 2 * E) * (d.n[2] + 2 * E);
  const long long NT = (long long)(d.n[0] + 2 * B) * (d.n[1] + 2 * B) * (d.n[2] + 2 * B);
  hipLaunchKernelGGL(m3_inner_kernel, lin_grid(ND), dim3(256), 0, st, d, ms, E, X, Dx);
  hipLaunchKernelGGL(m3_nodal_kernel, lin_grid(NT), dim3(256), 0, st, d, ms, B, E, X, Dx, T);
  hipLaunchKernelGGL(m3_band_kernel, lin_grid(d.mplane), dim3(256), 0, st, d, scheme, B, T, M, status, jform, ms, X, ah);
  return rc3(hipGetLastError());
}

int wiu3_rhs(const wiu_grid3* g, int scheme, const wiu_params* p, const double* U, const double* M, double* dUdt,
             void* ws, wiu_stream_t stream) {
  if (!grid3_ok(g) || scheme < 0 || scheme > 7 || !params3_ok(p, scheme) || !U || !M || !dUdt || !ws) return WIU_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const Dims3 d = dims3(g);
  const Ws3 w = ws3(g);
  char* base = (char*)ws;
  S3Args a;
  a.nlam = nullptr;
  a.ncfl = nullptr;
  a.d = d; a.U = U; a.M = M; a.lam = (unsigned long long*)(base + w.lam);
  a.gamma = p->gamma; a.alpha = p->alpha_lf; a.eps = p->eps; a.ppm = p->ppm;
  a.Racc = (double*)(base + w.racc); a.out = dUdt;
  sides3(g, a);
  options3(p, a);
  a.U0 = nullptr; a.dt = nullptr; a.ca = 0.0; a.cb = 1.0; a.status = (int*)base;
  if (maxima3(d, U, M, p->gamma, (unsigned long long*)a.lam, w.nlam, a.status, st) != hipSuccess) return WIU_EHIP;
  for (int q = 0; q < 3; ++q)  // zeta, eta, then xi, which writes dU/dt
    if (pass3(scheme, a, 2 - q, q == 0 ? 0 : (q == 1 ? 1 : 2), st) != hipSuccess) return WIU_EHIP;
  return WIU_OK;
}

int wiu3_cfl_dt(const wiu_grid3* g, const wiu_params* p, const double* U, const double* M, double cfl, double* dt,
                void* ws, wiu_stream_t stream) {
  if (!grid3_ok(g) || !p || !(p->gamma > 1.0) || !U || !M || !dt || !ws || !(cfl > 0.0)) return WIU_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const Dims3 d = dims3(g);
  const Ws3 w = ws3(g);
  char* base = (char*)ws;
  unsigned long long* lam = (unsigned long long*)(base + w.lam);
  if (maxima3(d, U, M, p->gamma, lam, w.nlam, (int*)base, st) != hipSuccess) return WIU_EHIP;
  return rc3(launch_cfl_dt(lam + w.nlam - 1, cfl, dt, st));
}

int wiu3_rk3_step(const wiu_grid3* g, int scheme, const wiu_params* p, double* U, const double* M, const double* dt,
                  void* ws, wiu_stream_t stream) {
  return rk3_3d(g, scheme, p, U, M, 0.0, const_cast<double*>(dt), ws, stream);
}

int wiu3_rk3_step_cfl(const wiu_grid3* g, int scheme, const wiu_params* p, double* U, const double* M, double cfl,
                      double* dt, void* ws, wiu_stream_t stream) {
  if (!(cfl > 0.0)) return WIU_EINVAL;
  return rk3_3d(g, scheme, p, U, M, cfl, dt, ws, stream);
}

int wiu3_rk3_steps_cfl(const wiu_grid3* g, int scheme, const wiu_params* p, double* U, const double* M, double cfl,
                       int nsteps, double* dt, void* ws, wiu_stream_t stream) {
  if (!(cfl > 0.0) || nsteps < 1) return WIU_EINVAL;
  return rk3_3d(g, scheme, p, U, M, cfl, dt, ws, stream, nsteps);
}

}  // extern "C"
