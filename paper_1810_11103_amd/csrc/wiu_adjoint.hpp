// Hand-written reverse mode (vector-Jacobian products) of the device building
// blocks in wiu_device.hpp, metrics held fixed.  Each routine recomputes the
// forward quantities it needs in registers and then applies the chain rule
// backwards; "bar" variables are adjoints.  Non-smooth points: the mappings
// are C^1 at w = C (both pieces have zero slope there); |x| uses sign(0) = 0.
#pragma once

#include "wiu_device.hpp"

namespace wiu {

// ---------------------------------------------------------------------------
// WENO r = 3 (inputs a, b, d, e around the zero centre) -- see weno5.
// Accumulates the adjoints of the inputs.
// ---------------------------------------------------------------------------
WIU_DEV void weno5_vjp(double a, double b, double d, double e, double eps, int ppm, double ob, double& ab,
                       double& bb, double& db, double& eb) {
  const double C[3] = {0.0625, 0.625, 0.3125};
  const double KL[3] = {WIU_M3L0, WIU_M3L1, WIU_M3L2};
  const double KH[3] = {WIU_M3H0, WIU_M3H1, WIU_M3H2};
  const double p[3] = {0.375 * a - 1.25 * b, 0.375 * d - 0.125 * b, 0.75 * d - 0.125 * e};
  const double d1 = b - a, d2 = -b, d3 = d, d4 = e - d;
  const double t[3] = {d2 - d1, d3 - d2, d4 - d3};
  const double s[3] = {fma(3.0, d2, -d1), -(d2 + d3), fma(-3.0, d3, d4)};
  // IS_k = 13/12 t^2 + 1/4 s^2 (Eq. 3.22), E = eps + IS, D = E^2
  double E[3], D[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double u = 0.5 * s[k];
    E[k] = fma(13.0 / 12.0, t[k] * t[k], fma(u, u, eps));
    D[k] = E[k] * E[k];
  }
  // alpha_k = C_k prod_{l != k} D_l (the common factor of the products cancels)
  const double P[3] = {D[1] * D[2], D[0] * D[2], D[0] * D[1]};
  const double al[3] = {C[0] * P[0], C[1] * P[1], C[2] * P[2]};
  const double r = rcp_w(al[0] + al[1] + al[2]);
  double w[3], g[3], h[3], dw[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    w[k] = al[k] * r;
    dw[k] = w[k] - C[k];
    h[k] = kd(dw[k], KL[k], KH[k]);  // K d, as the forward sweep forms it
    g[k] = ppm ? fma(dw[k], fma(dw[k], h[k], -1.0), w[k]) : w[k];  // C + K d^3
  }
  const double rs = rcp_w(g[0] + g[1] + g[2]);
  const double N = g[0] * p[0] + g[1] * p[1] + g[2] * p[2];
  // out = N / sum g
  const double Nb = ob * rs;
  const double sgb = -(Nb * N) * rs;
  double pb[3], cb[3];
  double rb = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    pb[k] = Nb * g[k];
    const double gb = fma(Nb, p[k], sgb);
    const double wb = ppm ? gb * (3.0 * (dw[k] * h[k])) : gb;  // dg/dw = 3 K d^2
    cb[k] = wb * r;
    rb = fma(wb, al[k], rb);
  }
  const double Sb = -(rb * r) * r;
  // adjoints of alpha_k times C_k, then of D_l
#pragma unroll
  for (int k = 0; k < 3; ++k) cb[k] = (cb[k] + Sb) * C[k];
  const double Db[3] = {fma(cb[1], D[2], cb[2] * D[1]), fma(cb[0], D[2], cb[2] * D[0]),
                        fma(cb[0], D[1], cb[1] * D[0])};
  double tb[3], sb[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double q = E[k] * Db[k];  // dIS = 2 E dD
    tb[k] = (13.0 / 3.0) * q * t[k];
    sb[k] = q * s[k];
  }
  const double d1b = -tb[0] - sb[0];
  const double d2b = tb[0] - tb[1] + 3.0 * sb[0] - sb[1];
  const double d3b = tb[1] - tb[2] - sb[1] - 3.0 * sb[2];
  const double d4b = tb[2] + sb[2];
  ab += -d1b + 0.375 * pb[0];
  bb += d1b - d2b - 1.25 * pb[0] - 0.125 * pb[1];
  db += d3b - d4b + 0.375 * pb[1] + 0.75 * pb[2];
  eb += d4b - 0.125 * pb[2];
}

// WENO r = 2 (inputs a, b, d around the zero centre) -- see weno3.
WIU_DEV void weno3_vjp(double a, double b, double d, double eps, int ppm, double ob, double& ab, double& bb,
                       double& db) {
  const double C[2] = {0.25, 0.75};
  const double KL[2] = {WIU_M2L0, WIU_M2L1};
  const double KH[2] = {WIU_M2H0, WIU_M2H1};
  const double p[2] = {-0.5 * b, 0.5 * d};
  const double d1 = b - a, d2 = -b, d3 = d;
  const double t[2] = {d2 - d1, d3 - d2};
  const double s[2] = {fma(3.0, d2, -d1), -(d2 + d3)};
  double E[2], D[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double u = 0.5 * s[k];
    E[k] = fma(13.0 / 12.0, t[k] * t[k], fma(u, u, eps));
    D[k] = E[k] * E[k];
  }
  const double al[2] = {C[0] * D[1], C[1] * D[0]};
  const double r = rcp_w(al[0] + al[1]);
  double w[2], g[2], h[2], dw[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    w[k] = al[k] * r;
    dw[k] = w[k] - C[k];
    h[k] = kd(dw[k], KL[k], KH[k]);  // K d, as the forward sweep forms it
    g[k] = ppm ? fma(dw[k], h[k] - 1.0, w[k]) : w[k];  // C + K d^2
  }
  const double rs = rcp_w(g[0] + g[1]);
  const double N = g[0] * p[0] + g[1] * p[1];
  // out = N / sum g
  const double Nb = ob * rs;
  const double sgb = -(Nb * N) * rs;
  double pb[2], cb[2], rb = 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    pb[k] = Nb * g[k];
    const double gb = fma(Nb, p[k], sgb);
    const double wb = ppm ? gb * (2.0 * h[k]) : gb;  // dg/dw = 2 K d
    cb[k] = wb * r;
    rb = fma(wb, al[k], rb);
  }
  const double Sb = -(rb * r) * r;
  // alpha_0 = C_0 D_1, alpha_1 = C_1 D_0; dIS = 2 E dD
  const double q0 = E[0] * ((cb[1] + Sb) * C[1]), q1 = E[1] * ((cb[0] + Sb) * C[0]);
  double tb[2], sb[2];
  tb[0] = (13.0 / 3.0) * q0 * t[0]; sb[0] = q0 * s[0];
  tb[1] = (13.0 / 3.0) * q1 * t[1]; sb[1] = q1 * s[1];
  const double d1b = -tb[0] - sb[0];
  const double d2b = tb[0] - tb[1] + 3.0 * sb[0] - sb[1];
  const double d3b = tb[1] - sb[1];
  ab += -d1b;
  bb += d1b - d2b - 0.5 * pb[0];
  db += d3b + 0.5 * pb[1];
}

// ---------------------------------------------------------------------------
// Reverse of side_flux for one side: given Fb = adjoint of F^{+-}_{k+1/2},
// accumulate the adjoints of the states k-2 .. k+3 and of the line
// eigenvalue.  The states are read through q(m, c) and the adjoints added
// through qb(m, c, value), so both can live in LDS.  Per stencil node only
// the five forward values A, B, drho, dm, dn of the projection are kept; the
// characteristic values are rebuilt from them where needed.
// ---------------------------------------------------------------------------
template <bool FIFTH, class QF, class QBF>
WIU_DEV void side_flux_vjp(QF q, int side, double nx_, double ny_, double mx, double my, double lam, double gam,
                           double eps, int ppm, const double Fb[4], QBF qb, double& lamb) {
  const int mr = 2 + side;
  const double Qr[4] = {q(mr, 0), q(mr, 1), q(mr, 2), q(mr, 3)};
  const double gm1 = gam - 1.0;
  // ---- forward recompute
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
  constexpr int NS = FIFTH ? 5 : 4;
  // stencil slot s <-> state m (left-biased order for side 0, mirrored for 1);
  // slot 2 is the reference node, whose deviation is zero
  auto mof = [&](int s_) { return side == 0 ? s_ : 5 - s_; };
  // characteristic value k of slot s_, recomputed from the staged states
  // wherever it is needed (keeps the register working set small)
  auto wv = [&](int k, int s_) {
    const int m = mof(s_);
    const double dr = q(m, 0) - Qr[0], dm = q(m, 1) - Qr[1], dn = q(m, 2) - Qr[2];
    if (k == 2) return nx_ * dn - ny_ * dm - qt * dr;
    const double de = q(m, 3) - Qr[3];
    const double A = b2 * dr - b1 * (u * dm + v * dn - de);
    if (k == 1) return dr - A;
    const double B = rc * (qn * dr - nx_ * dm - ny_ * dn);
    return k == 0 ? 0.5 * (A + B) : 0.5 * (A - B);
  };
  double W[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if constexpr (FIFTH) W[k] = weno5(wv(k, 0), wv(k, 1), wv(k, 3), wv(k, 4), eps, ppm);
    else W[k] = weno3(wv(k, 0), wv(k, 1), wv(k, 3), eps, ppm);
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
  // ---- reverse: F = (r Ul + (0, mx pl, my pl, pl Ul) + sl r) / 2
  double r0b = 0.5 * Fb[0] * (Ul + sl);
  double r1b = 0.5 * Fb[1] * (Ul + sl);
  double r2b = 0.5 * Fb[2] * (Ul + sl);
  double r3b = 0.5 * Fb[3] * (Ul + sl);
  const double Ulb = 0.5 * (Fb[0] * r0 + Fb[1] * r1 + Fb[2] * r2 + Fb[3] * (r3 + pl));
  const double plb = 0.5 * (Fb[1] * mx + Fb[2] * my + Fb[3] * Ul);
  const double slb = 0.5 * (Fb[0] * r0 + Fb[1] * r1 + Fb[2] * r2 + Fb[3] * r3);
  lamb += side == 0 ? slb : -slb;
  double ulb = Ulb * mx, vlb = Ulb * my;
  r3b += gm1 * plb;
  r1b -= 0.5 * gm1 * plb * ul;
  ulb -= 0.5 * gm1 * plb * r1;
  r2b -= 0.5 * gm1 * plb * vl;
  vlb -= 0.5 * gm1 * plb * r2;
  r1b += ulb * ri;
  r2b += vlb * ri;
  r0b -= (ulb * r1 + vlb * r2) * ri * ri;
  // r = Qr + R W
  double Qrb[4] = {r0b, r1b, r2b, r3b};
  const double sumb = r0b + u * r1b + v * r2b;
  double ub = r1b * sum, vb = r2b * sum;
  const double d30b = c * (nx_ * r1b + ny_ * r2b + qn * r3b);
  const double cb = d30 * (nx_ * r1b + ny_ * r2b + qn * r3b);
  const double Wb2 = -ny_ * r1b + nx_ * r2b + qt * r3b;
  const double s03b = H * r3b + sumb;
  const double Hb = s03 * r3b;
  double qnb = c * d30 * r3b;
  double q2b = 0.5 * W[1] * r3b;
  const double Wb1 = 0.5 * q2 * r3b + sumb;
  double qtb = W[2] * r3b;
  const double Wb[4] = {s03b - d30b, Wb1, Wb2, s03b + d30b};
  // WENO per characteristic component: wb[k][s] = adjoint of value k at slot s.
  // The compiler barrier makes the reverse re-read the staged states instead
  // of keeping every forward intermediate of the four components live.
  double wb[4][NS];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    asm volatile("" ::: "memory");
#pragma unroll
    for (int s_ = 0; s_ < NS; ++s_) wb[k][s_] = 0.0;
    if constexpr (FIFTH)
      weno5_vjp(wv(k, 0), wv(k, 1), wv(k, 3), wv(k, 4), eps, ppm, Wb[k], wb[k][0], wb[k][1], wb[k][3], wb[k][4]);
    else
      weno3_vjp(wv(k, 0), wv(k, 1), wv(k, 3), eps, ppm, Wb[k], wb[k][0], wb[k][1], wb[k][3]);
  }
  // projection of the deviations: per slot, adjoints of A, B and of the
  // deviation itself, then onto the slot's state and the reference state
  double b1b = 0.0, b2b = 0.0, rcb = 0.0;
#pragma unroll
  for (int s_ = 0; s_ < NS; ++s_) {
    if (s_ == 2) continue;
    const int m = mof(s_);
    const double dr = q(m, 0) - Qr[0], dm = q(m, 1) - Qr[1], dn = q(m, 2) - Qr[2], de = q(m, 3) - Qr[3];
    const double Ab = 0.5 * (wb[0][s_] + wb[3][s_]) - wb[1][s_];
    const double Bb = 0.5 * (wb[0][s_] - wb[3][s_]);
    double drb = wb[1][s_] - qt * wb[2][s_], dmb = -ny_ * wb[2][s_], dnb = nx_ * wb[2][s_], deb = 0.0;
    qtb -= dr * wb[2][s_];
    // A = b2 dr - b1 (u dm + v dn - de)
    b2b += Ab * dr;
    drb += Ab * b2;
    b1b -= Ab * (u * dm + v * dn - de);
    ub -= Ab * b1 * dm;
    vb -= Ab * b1 * dn;
    dmb -= Ab * b1 * u;
    dnb -= Ab * b1 * v;
    deb += Ab * b1;
    // B = rc (qn dr - nx dm - ny dn)
    rcb += Bb * (qn * dr - nx_ * dm - ny_ * dn);
    qnb += Bb * rc * dr;
    drb += Bb * rc * qn;
    dmb -= Bb * rc * nx_;
    dnb -= Bb * rc * ny_;
    // deviation = q[m] - Qr
    qb(m, 0, drb); qb(m, 1, dmb); qb(m, 2, dnb); qb(m, 3, deb);
    Qrb[0] -= drb; Qrb[1] -= dmb; Qrb[2] -= dnb; Qrb[3] -= deb;
  }
  // reference state
  b1b += 0.5 * q2 * b2b;
  q2b += 0.5 * b1 * b2b;
  rcb += 2.0 * gm1 * rc * b1b;
  vb += nx_ * qtb;
  ub -= ny_ * qtb;
  ub += nx_ * qnb;
  vb += ny_ * qnb;
  Qrb[3] += Hb * rr;
  double pb = Hb * rr;
  double rrb = Hb * (Qr[3] + p);
  double c2b = cb * rc;
  rcb += cb * c2;
  c2b -= 0.5 * rcb * rc * rc * rc;
  pb += c2b * gam * rr;
  rrb += c2b * gam * p;
  Qrb[3] += gm1 * pb;
  Qrb[0] -= 0.5 * gm1 * q2 * pb;
  q2b -= 0.5 * gm1 * Qr[0] * pb;
  ub += 2.0 * u * q2b;
  vb += 2.0 * v * q2b;
  Qrb[1] += ub * rr;
  rrb += ub * Qr[1];
  Qrb[2] += vb * rr;
  rrb += vb * Qr[2];
  Qrb[0] -= rrb * rr * rr;
#pragma unroll
  for (int cc = 0; cc < 4; ++cc) qb(mr, cc, Qrb[cc]);
}

// Reverse of nodal_split: fpb, fmb = adjoints of f^+-; accumulates Qb, lamb.
WIU_DEV void nodal_split_vjp(const double Q[4], double kx, double ky, double lam, double gam, const double fpb[4],
                             const double fmb[4], double Qb[4], double& lamb) {
  const double gm1 = gam - 1.0;
  const double ri = rcp(Q[0]);
  const double u = Q[1] * ri, v = Q[2] * ri;
  const double p = gm1 * (Q[3] - 0.5 * (Q[1] * u + Q[2] * v));
  const double U = kx * u + ky * v;
  double Eb[4], db[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    Eb[c] = 0.5 * (fpb[c] + fmb[c]);
    db[c] = 0.5 * (fpb[c] - fmb[c]);
    Qb[c] += lam * db[c];
    lamb += Q[c] * db[c];
  }
  // E = (rho U, m U + kx p, n U + ky p, (e + p) U)
  const double Ub = Eb[0] * Q[0] + Eb[1] * Q[1] + Eb[2] * Q[2] + Eb[3] * (Q[3] + p);
  const double pb = Eb[1] * kx + Eb[2] * ky + Eb[3] * U;
  Qb[0] += Eb[0] * U;
  Qb[1] += Eb[1] * U;
  Qb[2] += Eb[2] * U;
  Qb[3] += Eb[3] * U;
  double ub = Ub * kx, vb = Ub * ky;
  // p = gm1 (e - (m u + n v)/2)
  Qb[3] += gm1 * pb;
  Qb[1] -= 0.5 * gm1 * pb * u;
  ub -= 0.5 * gm1 * pb * Q[1];
  Qb[2] -= 0.5 * gm1 * pb * v;
  vb -= 0.5 * gm1 * pb * Q[2];
  Qb[1] += ub * ri;
  Qb[2] += vb * ri;
  const double rib = ub * Q[1] + vb * Q[2];
  Qb[0] -= rib * ri * ri;
}

// Reverse of the wave speed |k . u| + sqrt(c^2 |k|^2) (c^2 = gam p / rho).
WIU_DEV void wave_speed_vjp(const double Q[4], double kx, double ky, double gam, double sb, double Qb[4]) {
  const double gm1 = gam - 1.0;
  const double ri = 1.0 / Q[0];
  const double u = Q[1] * ri, v = Q[2] * ri;
  const double p = gm1 * (Q[3] - 0.5 * (Q[1] * u + Q[2] * v));
  const double U = kx * u + ky * v;
  const double K2 = kx * kx + ky * ky;
  const double sc = sqrt(gam * p * ri * K2);
  const double sgn = U > 0.0 ? 1.0 : (U < 0.0 ? -1.0 : 0.0);
  const double Ub = sb * sgn;
  // c^2 = gam p ri, d sqrt(c^2 K2) / d c^2 = K2 / (2 sqrt(c^2 K2))
  const double c2b = sb * K2 / (2.0 * sc);
  const double pb = c2b * gam * ri;
  double rib = c2b * gam * p;
  double ub = Ub * kx, vb = Ub * ky;
  Qb[3] += gm1 * pb;
  Qb[1] -= 0.5 * gm1 * pb * u;
  ub -= 0.5 * gm1 * pb * Q[1];
  Qb[2] -= 0.5 * gm1 * pb * v;
  vb -= 0.5 * gm1 * pb * Q[2];
  Qb[1] += ub * ri;
  Qb[2] += vb * ri;
  rib += ub * Q[1] + vb * Q[2];
  Qb[0] -= rib * ri * ri;
}

// Adjoint of the flux combination: coefficients of H_{i+1/2} on the split
// fluxes (Eqs. 3.4, 3.8, 3.16, 3.20 and their mirror images).  H(i) =
//   sum_m NP[m] f+(i+m) + MP[m] F+(i+m) + NM[m] f-(i+m) + MM[m] F-(i+m),
// m = -2 .. 3 (index m + 2); F(k) is the value at k + 1/2.
template <int SC> struct HCoef;
template <> struct HCoef<0> {
  static constexpr double NP[6] = {0, -1.0 / 24, 2.0 / 24, -1.0 / 24, 0, 0};
  static constexpr double MP[6] = {0, 0, 1.0, 0, 0, 0};
  static constexpr double NM[6] = {0, 0, -1.0 / 24, 2.0 / 24, -1.0 / 24, 0};
  static constexpr double MM[6] = {0, 0, 1.0, 0, 0, 0};
};
template <> struct HCoef<1> {
  static constexpr double NP[6] = {0, 0, 2.0 / 6, 0, 0, 0};
  static constexpr double MP[6] = {0, -1.0 / 6, 5.0 / 6, 0, 0, 0};
  static constexpr double NM[6] = {0, 0, 0, 2.0 / 6, 0, 0};
  static constexpr double MM[6] = {0, 0, 5.0 / 6, -1.0 / 6, 0, 0};
};
template <> struct HCoef<2> {
  static constexpr double NP[6] = {19.0 / 1920, -116.0 / 1920, 154.0 / 1920, -36.0 / 1920, -21.0 / 1920, 0};
  static constexpr double MP[6] = {0, 0, 1.0, 0, 0, 0};
  static constexpr double NM[6] = {0, -21.0 / 1920, -36.0 / 1920, 154.0 / 1920, -116.0 / 1920, 19.0 / 1920};
  static constexpr double MM[6] = {0, 0, 1.0, 0, 0, 0};
};
template <> struct HCoef<3> {
  static constexpr double NP[6] = {0, 1.0 / 30, 1.0 / 30, -4.0 / 30, 0, 0};
  static constexpr double MP[6] = {0, -4.0 / 30, 36.0 / 30, 0, 0, 0};
  static constexpr double NM[6] = {0, 0, -4.0 / 30, 1.0 / 30, 1.0 / 30, 0};
  static constexpr double MM[6] = {0, 0, 36.0 / 30, -4.0 / 30, 0, 0};
};

}  // namespace wiu
