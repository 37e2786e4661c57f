// Adjoint (vector-Jacobian product) kernels of the residual, metrics held
// fixed: given Gbar = adjoint of dU/dt, form Ubar = (d rhs / dU)^T Gbar, scaled
// and added to a linear combination of other arrays (AdjArgs), which is how the
// RK3 step adjoint combines its stages without separate passes.
//
// Per direction a tile of items recomputes the forward quantities, reverses
// the midpoint and nodal split fluxes (wiu_adjoint.hpp) and stores every
// item's contributions to the six states of its stencil in LDS; each output
// node then gathers its contributions in a fixed order (no atomics, so the
// result is deterministic).  Contributions to positions outside the line
// (wrapped or clamped by the boundary rule) and the adjoint of the line
// eigenvalue (a maximum over the line, Sec. 2.3, propagated to its first
// maximal node) are added by a per-line fix-up kernel.
#include "wiu_adjoint.hpp"
#include "wiu_kernels.hpp"

namespace wiu {

constexpr int NGHOST_ADJ = 6;  // positions beyond each end of a line that items touch

// Line-major (xi) or position-major (eta) so that the lanes of a wave touch
// consecutive words, as for the forward sweep tile.
template <int DIR, int NA, int NB> struct AdjLds {
  static constexpr int NQ = NA + 5, NR = NA + 6;
  double sq[4][NB * NQ];      // states k-2 .. k+3 of the items
  double rb[4][NB * NR];      // Rbar at positions k-3 .. k+3
  double cq[24][NA * NB];     // contributions [m*4 + c][item], m: position k-2+m
  double lb[NA * NB];         // line-eigenvalue adjoint per item
  int ka[NA * NB];            // k if node k attains the line maximum, else INT_MAX
  double xlb[NA];             // eta tiles folding the xi fix-up: per output row, the
  int xks[NA];                //   row's eigenvalue adjoint and first maximal node
  static WIU_DEV int si(int tb, int ta) { return DIR == 0 ? tb * NA + ta : ta * NB + tb; }
  static WIU_DEV int qi(int tb, int pos) { return DIR == 0 ? tb * NQ + pos : pos * NB + tb; }
  static WIU_DEV int ri(int tb, int pos) { return DIR == 0 ? tb * NR + pos : pos * NB + tb; }
};

template <int SC, int DIR, int NA, int NB>
__global__ void __launch_bounds__(NA * NB, 2) adj_sweep_kernel(AdjArgs s) {
  constexpr int LO = -3;                 // first item relative to the output segment
  constexpr int OUT = NA - 6;
  constexpr int NT = NA * NB;
  constexpr int NQ = NA + 5;
  using LT = AdjLds<DIR, NA, NB>;
  __shared__ LT L;
  const Dims& d = s.d;
  const int ta = DIR == 0 ? threadIdx.x : threadIdx.y;
  const int tb = DIR == 0 ? threadIdx.y : threadIdx.x;
  const int n_al = DIR == 0 ? d.nx : d.ny;
  const int n_ac = DIR == 0 ? d.ny : d.nx;
  const int bc_al = DIR == 0 ? d.bcx : d.bcy;
  const int total = gridDim.x * gridDim.y;
  const int lid = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, total);
  const int bxl = lid % gridDim.x, byl = lid / gridDim.x;
  const int seg = DIR == 0 ? bxl : byl;
  const int nseg = DIR == 0 ? gridDim.x : gridDim.y;
  const int lgrp = DIR == 0 ? byl : bxl;
  const int line = lgrp * NB + tb;
  const int o0 = seg * OUT;
  const int out = min(OUT, n_al - o0);
  const int k = o0 + LO + ta;
  const int slot = LT::si(tb, ta);
  const bool live = line < n_ac;
  const int tid = threadIdx.x + blockDim.x * threadIdx.y;

  // stage states (boundary rule applied) and Rbar = -Gbar / J^{-1} (zero off
  // the line); every load of the thread's elements is issued before any is
  // stored, so their latencies overlap
  {
    const int k0 = o0 + LO - 2;
    const int r0 = o0 + LO - 3;
    constexpr int NR = NA + 6;
    constexpr int IQ = (NQ * NB + NT - 1) / NT, IR = (NR * NB + NT - 1) / NT;
    double qv[IQ][4], gv[IR][4], jv[IR];
#pragma unroll
    for (int it = 0; it < IQ; ++it) {
      const int e = tid + it * NT;
      const int pos = DIR == 0 ? e % NQ : e / NB;
      const int lb_ = DIR == 0 ? e / NQ : e % NB;
      const int ln = lgrp * NB + lb_;
      if (e < NQ * NB && ln < n_ac) {
        const int kk = bc_index(k0 + pos, n_al, bc_al);
        const long long o = DIR == 0 ? (long long)ln * d.nx + kk : (long long)kk * d.nx + ln;
#pragma unroll
        for (int c = 0; c < 4; ++c) qv[it][c] = s.U[c * d.np + o];
      }
    }
#pragma unroll
    for (int it = 0; it < IR; ++it) {
      const int e = tid + it * NT;
      const int pos = DIR == 0 ? e % NR : e / NB;
      const int lb_ = DIR == 0 ? e / NR : e % NB;
      const int ln = lgrp * NB + lb_;
      const int p = r0 + pos;
#pragma unroll
      for (int c = 0; c < 4; ++c) gv[it][c] = 0.0;
      jv[it] = -1.0;
      if (e < NR * NB && ln < n_ac && p >= 0 && p < n_al) {
        const int ii = DIR == 0 ? p : ln, jj = DIR == 0 ? ln : p;
        const long long o = (long long)jj * d.nx + ii;
        jv[it] = s.M[4 * d.mplane + (long long)(jj + GHOST) * d.mpitch + (ii + GHOST)];
#pragma unroll
        for (int c = 0; c < 4; ++c) gv[it][c] = s.Gbar[c * d.np + o];
      }
    }
#pragma unroll
    for (int it = 0; it < IQ; ++it) {
      const int e = tid + it * NT;
      const int pos = DIR == 0 ? e % NQ : e / NB;
      const int lb_ = DIR == 0 ? e / NQ : e % NB;
      if (e < NQ * NB && lgrp * NB + lb_ < n_ac) {
#pragma unroll
        for (int c = 0; c < 4; ++c) L.sq[c][LT::qi(lb_, pos)] = qv[it][c];
      }
    }
#pragma unroll
    for (int it = 0; it < IR; ++it) {
      const int e = tid + it * NT;
      const int pos = DIR == 0 ? e % NR : e / NB;
      const int lb_ = DIR == 0 ? e / NR : e % NB;
      if (e < NR * NB) {
        const double rj = -1.0 / jv[it];
#pragma unroll
        for (int c = 0; c < 4; ++c) L.rb[c][LT::ri(lb_, pos)] = gv[it][c] * rj;
      }
    }
  }
  __syncthreads();

  // each item accumulates its contributions straight into its own LDS slot
#pragma unroll
  for (int e = 0; e < 24; ++e) L.cq[e][slot] = 0.0;
  double lamb = 0.0;
  int kmax = INT_MAX;
  // Neighbouring tiles recompute their overlapping items; an item's
  // eigenvalue adjoint and maximal-node flag are counted only by the tile
  // that owns the item's position (the end tiles own the items beyond the
  // line's ends).
  const bool owner = (k >= o0 || o0 == 0) && (k < o0 + out || o0 + out == n_al);
  const bool item = live && k >= o0 + LO && k <= o0 + out + 2;
  if (item) {
    // Hbar(i) = Rbar(i) - Rbar(i+1); Rbar(p) sits at rb[.][tb][p - (k - 3) + ta]
    auto Hb = [&](int c, int i) {
      const int a = i - (o0 + LO - 3);
      return L.rb[c][LT::ri(tb, a)] - L.rb[c][LT::ri(tb, a + 1)];
    };
    double fpb[4], fmb[4], Fpb[4], Fmb[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      fpb[c] = fmb[c] = Fpb[c] = Fmb[c] = 0.0;
#pragma unroll
      for (int mm = 0; mm < 6; ++mm) {
        const int m = mm - 2;  // H(i) uses node / midpoint i + m, so item k feeds H(k - m)
        if (HCoef<SC>::NP[mm] != 0.0) fpb[c] += HCoef<SC>::NP[mm] * Hb(c, k - m);
        if (HCoef<SC>::NM[mm] != 0.0) fmb[c] += HCoef<SC>::NM[mm] * Hb(c, k - m);
        if (HCoef<SC>::MP[mm] != 0.0) Fpb[c] += HCoef<SC>::MP[mm] * Hb(c, k - m);
        if (HCoef<SC>::MM[mm] != 0.0) Fmb[c] += HCoef<SC>::MM[mm] * Hb(c, k - m);
      }
    }
    auto q = [&](int m, int c) { return L.sq[c][LT::qi(tb, ta + m)]; };
    auto qb = [&](int m, int c, double v) { L.cq[m * 4 + c][slot] += v; };
    const double qk[4] = {q(2, 0), q(2, 1), q(2, 2), q(2, 3)};
    const long long mstride = DIR == 0 ? 1 : d.mpitch;
    const long long mline = DIR == 0 ? (long long)(line + GHOST) * d.mpitch + GHOST
                                     : (long long)GHOST * d.mpitch + (line + GHOST);
    const double* Mk = s.M + (DIR == 0 ? 0 : 2) * d.mplane;
    const double* Mm = s.M + (DIR == 0 ? 5 : 7) * d.mplane;
    const long long mo = mline + mstride * k;
    const unsigned long long* lp = DIR == 0 ? s.lam_xi : s.lam_eta;
    const double smax = __longlong_as_double((long long)lp[line]);
    const double lam = s.alpha * smax;
    const double kx0 = Mk[mo], ky0 = Mk[d.mplane + mo];
    if (owner && k >= 0 && k < n_al) {
      bool bad;
      if (wave_speed(qk, kx0, ky0, s.gamma, bad) == smax) kmax = k;
    }
    {
      double nb[4] = {0.0, 0.0, 0.0, 0.0};
      nodal_split_vjp(qk, kx0, ky0, lam, s.gamma, fpb, fmb, nb, lamb);
#pragma unroll
      for (int c = 0; c < 4; ++c) qb(2, c, nb[c]);
    }
    bool midnz = false;
#pragma unroll
    for (int c = 0; c < 4; ++c) midnz |= (Fpb[c] != 0.0) || (Fmb[c] != 0.0);
    if (midnz && k <= o0 + out + 1) {
      const double kx1 = Mk[mo + mstride], ky1 = Mk[d.mplane + mo + mstride];
      const double mx = Mm[mo], my = Mm[d.mplane + mo];
      const double nbx = 0.5 * (kx0 + kx1), nby = 0.5 * (ky0 + ky1);
      const double rn = rsqrt_(nbx * nbx + nby * nby);
      const double nx_ = nbx * rn, ny_ = nby * rn;
      // the two sides one after the other (not interleaved) to bound the
      // register working set
#pragma nounroll
      for (int side = 0; side < 2; ++side) {
        double Fb[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) Fb[c] = side == 0 ? Fpb[c] : Fmb[c];
        side_flux_vjp<Traits<SC>::fifth>(q, side, nx_, ny_, mx, my, lam, s.gamma, s.eps, s.ppm, Fb, qb, lamb);
      }
    }
  }
  L.lb[slot] = owner ? lamb : 0.0;
  L.ka[slot] = kmax;
  // eta tiles folding the xi fix-up: reduce each output row's xi partials
  // (fixed order over the row's segments)
  const bool xfold = DIR == 1 && s.x_lam_part != nullptr;
  if (xfold && tb == 0 && ta < out) {
    const int row = o0 + ta;
    const double* lp = s.x_lam_part + (long long)row * s.x_nseg;
    const int* ap = s.x_arg_part + (long long)row * s.x_nseg;
    double sum = 0.0;
    int kf = INT_MAX;
    // eight segments' loads in flight at a time, then their sum in order
    for (int t0 = 0; t0 < s.x_nseg; t0 += 8) {
      double v[8];
      int a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool in = t0 + u < s.x_nseg;
        v[u] = in ? lp[t0 + u] : 0.0;
        a[u] = in ? ap[t0 + u] : INT_MAX;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (t0 + u < s.x_nseg) sum += v[u];
        kf = min(kf, a[u]);
      }
    }
    L.xlb[ta] = sum;
    L.xks[ta] = kf;
    if (kf >= d.nx && sum != 0.0) atomicOr(s.status, ST_ARGMAX);
  }
  __syncthreads();

  if (!live) return;
  // line-eigenvalue adjoint of this tile (fixed-order sum over its items) and
  // its first node attaining the line maximum
  if (ta == 0) {
    // four interleaved partial sums (fixed association, shorter dependence chain)
    double sum4[4] = {0.0, 0.0, 0.0, 0.0};
    int kf = INT_MAX;
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      sum4[t & 3] += L.lb[LT::si(tb, t)];
      kf = min(kf, L.ka[LT::si(tb, t)]);
    }
    const double sum = (sum4[0] + sum4[1]) + (sum4[2] + sum4[3]);
    s.lam_part[(long long)line * nseg + seg] = sum;
    s.arg_part[(long long)line * nseg + seg] = kf;
  }
  // gather at output positions (and ghost positions at the two line ends)
  auto gather = [&](int p, double g[4]) {
    const int t0 = p - (o0 + LO);  // slot offset of item k = p
#pragma unroll
    for (int c = 0; c < 4; ++c) g[c] = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const int t = t0 + 2 - m;  // item k = p + 2 - m
      if (t >= 0 && t < NA) {
#pragma unroll
        for (int c = 0; c < 4; ++c) g[c] += L.cq[m * 4 + c][LT::si(tb, t)];
      }
    }
  };
  if (ta < out) {
    const int p = o0 + ta;
    double g[4];
    gather(p, g);
    const long long o = DIR == 0 ? (long long)line * d.nx + p : (long long)p * d.nx + line;
    const double coef = s.coef_c * (s.coef_dt ? s.coef_dt[0] : 1.0);
    if (xfold) {
      // xi fix-up of node (line, p) of row p: off-line contributions that the
      // boundary rule maps here (only the six columns at each end), then the
      // row eigenvalue's adjoint if this is the row's first maximal node
      constexpr int NG = 2 * NGHOST_ADJ;
      if (line < NGHOST_ADJ || line >= d.nx - NGHOST_ADJ) {
        for (int gi = 0; gi < NG; ++gi) {
          const int pg = gi < NGHOST_ADJ ? -1 - gi : d.nx + (gi - NGHOST_ADJ);
          if (bc_index(pg, d.nx, d.bcx) != line) continue;
          const double* gb =
              s.x_ghost + (((long long)p * 2 + (gi < NGHOST_ADJ ? 0 : 1)) * NGHOST_ADJ + gi % NGHOST_ADJ) * 4;
#pragma unroll
          for (int c = 0; c < 4; ++c) g[c] += gb[c];
        }
      }
      const double xl = L.xlb[ta];
      if (L.xks[ta] == line && xl != 0.0) {
        const int pq = LT::qi(tb, p - (o0 + LO - 2));
        const double Q[4] = {L.sq[0][pq], L.sq[1][pq], L.sq[2][pq], L.sq[3][pq]};
        const long long mo = (long long)(p + GHOST) * d.mpitch + (line + GHOST);
        wave_speed_vjp(Q, s.M[mo], s.M[d.mplane + mo], s.gamma, s.alpha * xl, g);
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const long long e = c * d.np + o;
      double v = coef * g[c];
      if (s.accumulate) {
        v += s.Ubar[e];
      } else {
#pragma unroll
        for (int k = 0; k < 3; ++k)
          if (s.base_x[k]) v += s.base_a[k] * s.base_x[k][e];
      }
      s.Ubar[e] = v;
    }
  }
  if (ta < 2 * NGHOST_ADJ) {
    const bool low = ta < NGHOST_ADJ;
    const int j = low ? ta : ta - NGHOST_ADJ;
    const int p = low ? -1 - j : n_al + j;
    const bool mine = low ? (o0 == 0) : (o0 + out == n_al);
    if (mine) {
      double g[4];
      gather(p, g);
      double* gb = s.ghost + (((long long)line * 2 + (low ? 0 : 1)) * NGHOST_ADJ + j) * 4;
#pragma unroll
      for (int c = 0; c < 4; ++c) gb[c] = g[c];
    }
  }
}

// Per-line fix-up, one wave per line: the off-line (ghost) contributions
// onto the nodes the boundary rule maps them to, and the line eigenvalue's
// adjoint (lam = alpha max_k s_k, Sec. 2.3) onto the first node attaining the
// maximum.  Each target node is owned by one lane, which adds its terms in a
// fixed order, so the result is deterministic.
__global__ void __launch_bounds__(256) adj_fixup_kernel(AdjArgs s, int dir, int nseg) {
  const Dims& d = s.d;
  const int lane = threadIdx.x & 63;
  const int line = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int n_al = dir == 0 ? d.nx : d.ny;
  const int n_ac = dir == 0 ? d.ny : d.nx;
  const int bc_al = dir == 0 ? d.bcx : d.bcy;
  if (line >= n_ac) return;
  constexpr int NG = 2 * NGHOST_ADJ;
  auto target = [&](int g) {
    const int p = g < NGHOST_ADJ ? -1 - g : n_al + (g - NGHOST_ADJ);
    return bc_index(p, n_al, bc_al);
  };
  // Lane g < NG holds ghost position g: its target node tg and contribution
  // gv (all loaded at once).  The first lane of each distinct target owns
  // it and sums the contributions of every lane with that target in lane
  // order, read across the wave; the owners' current Ubar is loaded at once
  // too, so these loads overlap the reduction below.
  int tg = -1;
  double gv[4] = {0.0, 0.0, 0.0, 0.0};
  if (lane < NG) {
    tg = target(lane);
    const double* gb =
        s.ghost + (((long long)line * 2 + (lane < NGHOST_ADJ ? 0 : 1)) * NGHOST_ADJ + lane % NGHOST_ADJ) * 4;
#pragma unroll
    for (int c = 0; c < 4; ++c) gv[c] = gb[c];
  }
  int t = lane < NG ? tg : -1;
  bool own = lane < NG;
  double acc[4] = {0.0, 0.0, 0.0, 0.0}, ub[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int g = 0; g < NG; ++g) {  // lane g's values, read into scalar registers
    const int tgg = __builtin_amdgcn_readlane(tg, g);
    double gg[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const long long bits = __double_as_longlong(gv[c]);
      const unsigned lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffLL), g);
      const unsigned hi = __builtin_amdgcn_readlane((int)(bits >> 32), g);
      gg[c] = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    }
    if (lane < NG && tgg == t) {
      if (g < lane) own = false;
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] += gg[c];
    }
  }
  if (own) {
    const long long o = dir == 0 ? (long long)line * d.nx + t : (long long)t * d.nx + line;
#pragma unroll
    for (int c = 0; c < 4; ++c) ub[c] = s.Ubar[c * d.np + o];
  }
  // eigenvalue adjoint and first maximal node over the line's segments
  double lb = 0.0;
  int ks = INT_MAX;
  for (int q = lane; q < nseg; q += 64) {
    lb += s.lam_part[(long long)line * nseg + q];
    ks = min(ks, s.arg_part[(long long)line * nseg + q]);
  }
  for (int off = 32; off > 0; off >>= 1) {  // symmetric butterfly: every lane gets the same bits
    lb += __shfl_xor(lb, off, 64);
    ks = min(ks, __shfl_xor(ks, off, 64));
  }
  // lane NG: the maximal node if no ghost maps there
  if (lane == NG && ks < n_al) {
    t = ks;
    own = true;
    for (int g = 0; g < NG; ++g) own = own && target(g) != t;
    if (own) {
      const long long o = dir == 0 ? (long long)line * d.nx + t : (long long)t * d.nx + line;
#pragma unroll
      for (int c = 0; c < 4; ++c) ub[c] = s.Ubar[c * d.np + o];
    }
  }
  if (own) {
    const long long o = dir == 0 ? (long long)line * d.nx + t : (long long)t * d.nx + line;
    if (t == ks && lb != 0.0) {
      const double Q[4] = {s.U[o], s.U[d.np + o], s.U[2 * d.np + o], s.U[3 * d.np + o]};
      const int ii = dir == 0 ? t : line, jj = dir == 0 ? line : t;
      const long long mo = (long long)(jj + GHOST) * d.mpitch + (ii + GHOST);
      const double* Mk = s.M + (dir == 0 ? 0 : 2) * d.mplane;
      wave_speed_vjp(Q, Mk[mo], Mk[d.mplane + mo], s.gamma, s.alpha * lb, acc);
    }
    const double coef = s.coef_c * (s.coef_dt ? s.coef_dt[0] : 1.0);
#pragma unroll
    for (int c = 0; c < 4; ++c) s.Ubar[c * d.np + o] = ub[c] + coef * acc[c];
  }
  if (lane == 0 && ks >= n_al && lb != 0.0) atomicOr(s.status, ST_ARGMAX);
}

// Adjoint tile length along the line: of two compiled shapes per direction,
// the one that recomputes the fewest items for this line length (each tile
// yields NA - 6 outputs).  Results depend on the choice only in the
// association of the eigenvalue-adjoint sums.
//   xi : 128 x 1 or 64 x 2;  eta: 128 x 2 or 64 x 4 (lines x items per workgroup)
int adj_tile_na(int dir, int n_al) {
  (void)dir;
  const long long i128 = (long long)((n_al + 121) / 122) * 128, i64 = (long long)((n_al + 57) / 58) * 64;
  return i64 < i128 ? 64 : 128;
}

template <int SC, int DIR, int NA>
hipError_t launch_adj_t(const AdjArgs& a, hipStream_t st) {
  constexpr int NB = DIR == 0 ? 128 / NA : 256 / NA;
  constexpr int OUT = NA - 6;
  const int n_al = DIR == 0 ? a.d.nx : a.d.ny;
  const int n_ac = DIR == 0 ? a.d.ny : a.d.nx;
  const int nseg = (n_al + OUT - 1) / OUT;
  const int nlin = (n_ac + NB - 1) / NB;
  dim3 grid = DIR == 0 ? dim3(nseg, nlin) : dim3(nlin, nseg);
  dim3 block = DIR == 0 ? dim3(NA, NB) : dim3(NB, NA);
  hipLaunchKernelGGL((adj_sweep_kernel<SC, DIR, NA, NB>), grid, block, 0, st, a);
  return hipGetLastError();
}

int adj_nseg(int dir, int n_al) {
  const int OUT = adj_tile_na(dir, n_al) - 6;
  return (n_al + OUT - 1) / OUT;
}

template <int SC, int DIR>
hipError_t launch_adj_d(const AdjArgs& a, hipStream_t st) {
  const int n_al = DIR == 0 ? a.d.nx : a.d.ny;
  return adj_tile_na(DIR, n_al) == 64 ? launch_adj_t<SC, DIR, 64>(a, st) : launch_adj_t<SC, DIR, 128>(a, st);
}

hipError_t launch_adj_sweep(int scheme, int dir, const AdjArgs& a, hipStream_t st, bool fixup) {
  hipError_t e;
  switch (scheme * 2 + dir) {
    case 0: e = launch_adj_d<0, 0>(a, st); break;
    case 1: e = launch_adj_d<0, 1>(a, st); break;
    case 2: e = launch_adj_d<1, 0>(a, st); break;
    case 3: e = launch_adj_d<1, 1>(a, st); break;
    case 4: e = launch_adj_d<2, 0>(a, st); break;
    case 5: e = launch_adj_d<2, 1>(a, st); break;
    case 6: e = launch_adj_d<3, 0>(a, st); break;
    default: e = launch_adj_d<3, 1>(a, st); break;
  }
  if (e != hipSuccess || !fixup) return e;
  const int nlines = dir == 0 ? a.d.ny : a.d.nx;
  const int nseg = adj_nseg(dir, dir == 0 ? a.d.nx : a.d.ny);
  hipLaunchKernelGGL(adj_fixup_kernel, dim3((nlines + 3) / 4), dim3(256), 0, st, a, dir, nseg);
  return hipGetLastError();
}

}  // namespace wiu
