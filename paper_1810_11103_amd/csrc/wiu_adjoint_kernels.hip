// Adjoint (vector-Jacobian product) kernels of the residual, metrics held
// fixed: given Gbar = adjoint of dU/dt, accumulate Ubar = (d rhs / dU)^T Gbar.
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

template <int NA, int NB> struct AdjLds {
  double sq[4][NB][NA + 5];   // states k-2 .. k+3 of the items
  double rb[4][NB][NA + 6];   // Rbar at positions k-3 .. k+3
  double cq[24][NA * NB];     // contributions [m*4 + c][item], m: position k-2+m
  double lb[NA * NB];         // line-eigenvalue adjoint per item
};

template <int SC, int DIR, int NA, int NB>
__global__ void __launch_bounds__(NA * NB) adj_sweep_kernel(AdjArgs s) {
  constexpr int LO = -3;                 // first item relative to the output segment
  constexpr int OUT = NA - 6;
  constexpr int NT = NA * NB;
  constexpr int NQ = NA + 5;
  __shared__ AdjLds<NA, NB> L;
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
  const int slot = tb * NA + ta;
  const bool live = line < n_ac;
  const int tid = threadIdx.x + blockDim.x * threadIdx.y;

  // stage states (boundary rule applied) and Rbar = -Gbar / J^{-1} (zero off the line)
  {
    const int k0 = o0 + LO - 2;
    for (int e = tid; e < NQ * NB; e += NT) {
      const int pos = DIR == 0 ? e % NQ : e / NB;
      const int lb_ = DIR == 0 ? e / NQ : e % NB;
      const int ln = lgrp * NB + lb_;
      if (ln < n_ac) {
        const int kk = bc_index(k0 + pos, n_al, bc_al);
        const long long o = DIR == 0 ? (long long)ln * d.nx + kk : (long long)kk * d.nx + ln;
#pragma unroll
        for (int c = 0; c < 4; ++c) L.sq[c][lb_][pos] = s.U[c * d.np + o];
      }
    }
    const int r0 = o0 + LO - 3;
    constexpr int NR = NA + 6;
    for (int e = tid; e < NR * NB; e += NT) {
      const int pos = DIR == 0 ? e % NR : e / NB;
      const int lb_ = DIR == 0 ? e / NR : e % NB;
      const int ln = lgrp * NB + lb_;
      const int p = r0 + pos;
      double v[4] = {0.0, 0.0, 0.0, 0.0};
      if (ln < n_ac && p >= 0 && p < n_al) {
        const int ii = DIR == 0 ? p : ln, jj = DIR == 0 ? ln : p;
        const long long o = (long long)jj * d.nx + ii;
        const double rj = -1.0 / s.M[4 * d.mplane + (long long)(jj + GHOST) * d.mpitch + (ii + GHOST)];
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = s.Gbar[c * d.np + o] * rj;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) L.rb[c][lb_][pos] = v[c];
    }
  }
  __syncthreads();

  double cq[6][4];
#pragma unroll
  for (int m = 0; m < 6; ++m)
#pragma unroll
    for (int c = 0; c < 4; ++c) cq[m][c] = 0.0;
  double lamb = 0.0;
  const bool item = live && k >= o0 + LO && k <= o0 + out + 2;
  if (item) {
    // Hbar(i) = Rbar(i) - Rbar(i+1); Rbar(p) sits at rb[.][tb][p - (k - 3) + ta]
    auto Hb = [&](int c, int i) {
      const int a = i - (o0 + LO - 3);
      return L.rb[c][tb][a] - L.rb[c][tb][a + 1];
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
    double q[6][4];
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
      for (int c = 0; c < 4; ++c) q[m][c] = L.sq[c][tb][ta + m];
    const long long mstride = DIR == 0 ? 1 : d.mpitch;
    const long long mline = DIR == 0 ? (long long)(line + GHOST) * d.mpitch + GHOST
                                     : (long long)GHOST * d.mpitch + (line + GHOST);
    const double* Mk = s.M + (DIR == 0 ? 0 : 2) * d.mplane;
    const double* Mm = s.M + (DIR == 0 ? 5 : 7) * d.mplane;
    const long long mo = mline + mstride * k;
    const unsigned long long* lp = DIR == 0 ? s.lam_xi : s.lam_eta;
    const double lam = s.alpha * __longlong_as_double((long long)lp[line]);
    const double kx0 = Mk[mo], ky0 = Mk[d.mplane + mo];
    nodal_split_vjp(q[2], kx0, ky0, lam, s.gamma, fpb, fmb, cq[2], lamb);
    bool midnz = false;
#pragma unroll
    for (int c = 0; c < 4; ++c) midnz |= (Fpb[c] != 0.0) || (Fmb[c] != 0.0);
    if (midnz && k <= o0 + out + 1) {
      const double kx1 = Mk[mo + mstride], ky1 = Mk[d.mplane + mo + mstride];
      const double mx = Mm[mo], my = Mm[d.mplane + mo];
      const double nbx = 0.5 * (kx0 + kx1), nby = 0.5 * (ky0 + ky1);
      const double rn = rsqrt_(nbx * nbx + nby * nby);
      const double nx_ = nbx * rn, ny_ = nby * rn;
      side_flux_vjp<Traits<SC>::fifth>(q, 0, nx_, ny_, mx, my, lam, s.gamma, s.eps, s.ppm, Fpb, cq, lamb);
      side_flux_vjp<Traits<SC>::fifth>(q, 1, nx_, ny_, mx, my, lam, s.gamma, s.eps, s.ppm, Fmb, cq, lamb);
    }
  }
#pragma unroll
  for (int m = 0; m < 6; ++m)
#pragma unroll
    for (int c = 0; c < 4; ++c) L.cq[m * 4 + c][slot] = cq[m][c];
  // Neighbouring tiles recompute their overlapping items; an item's
  // eigenvalue adjoint is counted only by the tile that owns the item's
  // position (the end tiles own the items beyond the line's ends).
  const bool owner = (k >= o0 || o0 == 0) && (k < o0 + out || o0 + out == n_al);
  L.lb[slot] = owner ? lamb : 0.0;
  __syncthreads();

  if (!live) return;
  // line-eigenvalue adjoint of this tile: fixed-order sum over its items
  if (ta == 0) {
    double sum = 0.0;
    for (int t = 0; t < NA; ++t) sum += L.lb[tb * NA + t];
    s.lam_part[(long long)line * nseg + seg] = sum;
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
        for (int c = 0; c < 4; ++c) g[c] += L.cq[m * 4 + c][tb * NA + t];
      }
    }
  };
  if (ta < out) {
    const int p = o0 + ta;
    double g[4];
    gather(p, g);
    const long long o = DIR == 0 ? (long long)line * d.nx + p : (long long)p * d.nx + line;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const long long e = c * d.np + o;
      s.Ubar[e] = s.accumulate ? s.Ubar[e] + g[c] : g[c];
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

// Per-line fix-up: ghost contributions onto the nodes the boundary rule maps
// them to, then the line eigenvalue's adjoint onto its first maximal node.
// One block of 256 threads per line.
__global__ void __launch_bounds__(256) adj_fixup_kernel(AdjArgs s, int dir, int nseg) {
  const Dims& d = s.d;
  const int line = blockIdx.x;
  const int n_al = dir == 0 ? d.nx : d.ny;
  const int bc_al = dir == 0 ? d.bcx : d.bcy;
  auto node_off = [&](int p) {
    return dir == 0 ? (long long)line * d.nx + p : (long long)p * d.nx + line;
  };
  __shared__ double red[256];
  __shared__ int ired[256];
  // first maximal node of the line's wave speed (the same expression and
  // rounding as the forward maximum)
  const double smax = __longlong_as_double((long long)(dir == 0 ? s.lam_xi : s.lam_eta)[line]);
  const double* Mk = s.M + (dir == 0 ? 0 : 2) * d.mplane;
  int best = n_al;
  for (int p = threadIdx.x; p < n_al; p += 256) {
    const long long o = node_off(p);
    const double Q[4] = {s.U[o], s.U[d.np + o], s.U[2 * d.np + o], s.U[3 * d.np + o]};
    const int ii = dir == 0 ? p : line, jj = dir == 0 ? line : p;
    const long long mo = (long long)(jj + GHOST) * d.mpitch + (ii + GHOST);
    bool bad;
    const double sp = wave_speed(Q, Mk[mo], Mk[d.mplane + mo], s.gamma, bad);
    if (sp == smax && p < best) best = p;
  }
  ired[threadIdx.x] = best;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) ired[threadIdx.x] = min(ired[threadIdx.x], ired[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  // ghost contributions, fixed order
  for (int side = 0; side < 2; ++side)
    for (int j = 0; j < NGHOST_ADJ; ++j) {
      const int p = side == 0 ? -1 - j : n_al + j;
      const double* gb = s.ghost + (((long long)line * 2 + side) * NGHOST_ADJ + j) * 4;
      const long long o = node_off(bc_index(p, n_al, bc_al));
      for (int c = 0; c < 4; ++c) s.Ubar[c * d.np + o] += gb[c];
    }
  // line eigenvalue: lam = alpha max_k s_k
  double lb = 0.0;
  for (int t = 0; t < nseg; ++t) lb += s.lam_part[(long long)line * nseg + t];
  const int ks = ired[0];
  if (ks < n_al && lb != 0.0) {
    const long long o = node_off(ks);
    const double Q[4] = {s.U[o], s.U[d.np + o], s.U[2 * d.np + o], s.U[3 * d.np + o]};
    const int ii = dir == 0 ? ks : line, jj = dir == 0 ? line : ks;
    const long long mo = (long long)(jj + GHOST) * d.mpitch + (ii + GHOST);
    double Qb[4] = {0.0, 0.0, 0.0, 0.0};
    wave_speed_vjp(Q, Mk[mo], Mk[d.mplane + mo], s.gamma, s.alpha * lb, Qb);
    for (int c = 0; c < 4; ++c) s.Ubar[c * d.np + o] += Qb[c];
  }
  (void)red;
}

// out = a x + b (y + dt z), elementwise over n values (RK3 adjoint stages).
__global__ void axpy_kernel(long long n, double a, const double* x, double b, const double* y, const double* dt,
                            const double* z, double* out) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) {
    const double xv = x ? x[t] : 0.0;
    const double yv = y ? y[t] : 0.0;
    const double zv = z ? dt[0] * z[t] : 0.0;
    out[t] = a * xv + b * (yv + zv);
  }
}

template <int SC, int DIR>
hipError_t launch_adj_t(const AdjArgs& a, hipStream_t st, int& nseg) {
  constexpr int NA = DIR == 0 ? 128 : 64;
  constexpr int NB = DIR == 0 ? 1 : 2;
  constexpr int OUT = NA - 6;
  const int n_al = DIR == 0 ? a.d.nx : a.d.ny;
  const int n_ac = DIR == 0 ? a.d.ny : a.d.nx;
  nseg = (n_al + OUT - 1) / OUT;
  const int nlin = (n_ac + NB - 1) / NB;
  dim3 grid = DIR == 0 ? dim3(nseg, nlin) : dim3(nlin, nseg);
  dim3 block = DIR == 0 ? dim3(NA, NB) : dim3(NB, NA);
  hipLaunchKernelGGL((adj_sweep_kernel<SC, DIR, NA, NB>), grid, block, 0, st, a);
  return hipGetLastError();
}

int adj_nseg(int dir, int n_al) {
  const int OUT = (dir == 0 ? 128 : 64) - 6;
  return (n_al + OUT - 1) / OUT;
}

hipError_t launch_adj_sweep(int scheme, int dir, const AdjArgs& a, hipStream_t st) {
  int nseg = 0;
  hipError_t e;
  switch (scheme * 2 + dir) {
    case 0: e = launch_adj_t<0, 0>(a, st, nseg); break;
    case 1: e = launch_adj_t<0, 1>(a, st, nseg); break;
    case 2: e = launch_adj_t<1, 0>(a, st, nseg); break;
    case 3: e = launch_adj_t<1, 1>(a, st, nseg); break;
    case 4: e = launch_adj_t<2, 0>(a, st, nseg); break;
    case 5: e = launch_adj_t<2, 1>(a, st, nseg); break;
    case 6: e = launch_adj_t<3, 0>(a, st, nseg); break;
    default: e = launch_adj_t<3, 1>(a, st, nseg); break;
  }
  if (e != hipSuccess) return e;
  const int nlines = dir == 0 ? a.d.ny : a.d.nx;
  hipLaunchKernelGGL(adj_fixup_kernel, dim3(nlines), dim3(256), 0, st, a, dir, nseg);
  return hipGetLastError();
}

hipError_t launch_axpy(long long n, double a, const double* x, double b, const double* y, const double* dt,
                       const double* z, double* out, hipStream_t st) {
  hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, a, x, b, y, dt, z, out);
  return hipGetLastError();
}

}  // namespace wiu
