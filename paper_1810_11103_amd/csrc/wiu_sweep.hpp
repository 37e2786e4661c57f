// Tile-level device code shared by the single-grid and batched kernels:
// the wave-speed maxima of one tile and one tile of a direction sweep.
#pragma once

#include "wiu_kernels.hpp"

namespace wiu {

struct WaveLds {
  double scol[4][64];
  double scfl[4];
};

// One 64 x 16 tile (tx, ty) of the wave-speed maxima; block of 64 x 4 threads.
WIU_DEV void wave_max_tile(const Dims& d, const double* __restrict__ U, const double* __restrict__ M, double gam,
                           unsigned long long* __restrict__ lam_xi, unsigned long long* __restrict__ lam_eta,
                           unsigned long long* __restrict__ cfl_max, int* __restrict__ status, int tx, int ty,
                           WaveLds& L) {
  // each thread row covers ROWS rows
  constexpr int ROWS = 4;
  auto& scol = L.scol;
  auto& scfl = L.scfl;
  __syncthreads();  // LDS of the previous tile is free
  const int i = tx * 64 + threadIdx.x;
  const int j0 = (ty * 4 + threadIdx.y) * ROWS;
  double colmax = 0.0, cflm = 0.0;
  bool bad_any = false;
  for (int r = 0; r < ROWS; ++r) {
    const int j = j0 + r;
    double sx = 0.0;
    if (i < d.nx && j < d.ny) {
      const long long o = (long long)j * d.nx + i;
      const double Q[4] = {U[o], U[d.np + o], U[2 * d.np + o], U[3 * d.np + o]};
      const long long mo = (long long)(j + GHOST) * d.mpitch + (i + GHOST);
      const WaveState w = wave_state(Q, gam);
      const double sxr = wave_speed_dir(w, M[mo], M[d.mplane + mo]);
      const double se = wave_speed_dir(w, M[2 * d.mplane + mo], M[3 * d.mplane + mo]);
      bad_any |= w.bad || !(sxr < 1.0e300) || !(se < 1.0e300);
      sx = fmax(0.0, sxr);  // NaN dropped, as below
      colmax = fmax(colmax, se);  // non-finite speeds are flagged through `status`
      cflm = fmax(cflm, (sx + se) / M[4 * d.mplane + mo]);
    }
    // row max across the 64 lanes of this wave (one wave = one row segment)
    double v = sx;
    for (int off = 32; off > 0; off >>= 1) {
      v = fmax(v, __shfl_xor(v, off, 64));
    }
    if (threadIdx.x == 0 && j < d.ny)
      atomicMax(&lam_xi[j], (unsigned long long)__double_as_longlong(v));
  }
  scol[threadIdx.y][threadIdx.x] = colmax;
  double c = cflm;
  for (int off = 32; off > 0; off >>= 1) {
    c = fmax(c, __shfl_xor(c, off, 64));
  }
  if (threadIdx.x == 0) scfl[threadIdx.y] = c;
  if (bad_any) atomicOr(status, ST_NONPHYS);
  __syncthreads();
  if (threadIdx.y == 0) {
    double m = scol[0][threadIdx.x];
    for (int t = 1; t < 4; ++t) m = fmax(m, scol[t][threadIdx.x]);
    if (i < d.nx) atomicMax(&lam_eta[i], (unsigned long long)__double_as_longlong(m));
    if (threadIdx.x == 0 && cfl_max) {
      double mm = scfl[0];
      for (int t = 1; t < 4; ++t) mm = fmax(mm, scfl[t]);
      atomicMax(cfl_max, (unsigned long long)__double_as_longlong(mm));
    }
  }
}


// Waves per SIMD a sweep kernel is compiled for: 4 (at most 128 VGPRs) for
// the third- and fifth-order schemes in the paper's configuration; the
// seventh-order interpolation, and the kernels that carry the scheme options,
// need more registers than that without spilling, so 3 (at most 168).
template <int SC, bool OPT> constexpr int sweep_waves() { return Traits<SC>::R == 4 || OPT ? 3 : 4; }

// LDS of a sweep tile.  Lanes of a wave run along the line for xi tiles and
// across lines (then along) for eta tiles; both arrays are laid out so that
// the lanes of a wave touch consecutive words (no bank conflicts): line-major
// for xi, position-major for eta.  Per item the nodal flux E^ is kept rather
// than f^+- = (E^ +- lam Q)/2, which the output phase rebuilds from E^ and the
// staged state (12 instead of 16 values per item, so larger tiles fit).
template <int SC, int DIR, int NA, int NB, bool OPT = false> struct SweepLds {
  static constexpr int NQ = NA + 2 * Range<SC>::QL + 1;  // states of items k - QL .. k + QL + 1
  // [kind*4 + comp][item]: kinds E^, F^+, F^- and, with the options, D (the
  // difference another midpoint split makes to H at the item's midpoint)
  static constexpr int NREC = OPT ? 16 : 12;
  double sh[NREC][NA * NB];
  double sq[4][NB * NQ];
  // item slot of (line tb, position ta) and state slot of (line tb, position pos)
  static WIU_DEV int si(int tb, int ta) { return DIR == 0 ? tb * NA + ta : ta * NB + tb; }
  static WIU_DEV int qi(int tb, int pos) { return DIR == 0 ? tb * NQ + pos : pos * NB + tb; }
};

// H_{k+1/2} of component c at the midpoint of item k (slot hs, its state at
// slot qs) from the records in LDS; with another split of the leading
// midpoint flux, plus that split's difference D at the same midpoint.
template <int SC, int DIR, int NA, int NB, bool OPT>
WIU_DEV double tile_hsum(const SweepLds<SC, DIR, NA, NB, OPT>& L, int c, int hs, int qs, int k, double lam,
                         double ah, bool alt) {
  // stencil nodes at constant offsets from the item (stride 1 along a xi
  // line, NB across eta lines)
  constexpr int S = DIR == 0 ? 1 : NB;
  const double* e = &L.sh[c][hs];
  const double* q = &L.sq[c][qs];
  const double* gp = &L.sh[4 + c][hs];
  const double* gm = &L.sh[8 + c][hs];
  double H;
  if constexpr (SC == 3) {
    H = hsum52(lam, [&](int m) { return e[m * S]; }, [&](int m) { return q[m * S]; },
               [&](int m) { return gp[m * S]; }, [&](int m) { return gm[m * S]; });
  } else {
    auto fp = [&](int kk) { return 0.5 * (e[(kk - k) * S] + lam * q[(kk - k) * S]); };
    auto fm = [&](int kk) { return 0.5 * (e[(kk - k) * S] - lam * q[(kk - k) * S]); };
    auto Fp = [&](int kk) { return gp[(kk - k) * S]; };
    auto Fm = [&](int kk) { return gm[(kk - k) * S]; };
    H = hflux<SC>(k, ah, fp, fm, Fp, Fm);
  }
  if constexpr (OPT) {
    if (alt) H += L.sh[12 + c][hs];
  }
  return H;
}

// H_{i+1/2} - H_{i-1/2} at output node i of line tb, once the items' H have
// replaced their nodal fluxes in LDS (sweep_tile): each midpoint's H is formed
// once and read by both of its nodes, so the differences telescope exactly.
template <int SC, int DIR, int NA, int NB, bool OPT>
WIU_DEV void tile_residual(const SweepLds<SC, DIR, NA, NB, OPT>& L, int tb, int o0, int i, double R[4]) {
  constexpr int S = DIR == 0 ? 1 : NB;
  const int hs = SweepLds<SC, DIR, NA, NB, OPT>::si(tb, i - (o0 + Range<SC>::LO));
#pragma unroll
  for (int c = 0; c < 4; ++c) R[c] = L.sh[c][hs] - L.sh[c][hs - S];
}

// Epilogue operands of one output node, loaded before the tile's last
// barrier so that their latency overlaps the barrier and the flux
// difference (at that point the compute phase's registers are free).
struct OutOperands {
  double x[4];   // R^xi (rhs), P (eta stage) or U0 (xi stage, when its coefficient is non-zero)
  double jinv;   // J^{-1} at the node
  double km[4];  // nodal metrics xi_x, xi_y, eta_x, eta_y (eta stage with next maxima)
};

// Output phase of an eta tile in RK-stage mode that also accumulates the line
// maxima of the new stage state (the next stage's eigenvalues, Sec. 2.3), so
// that stage needs no separate pass over the state.  Every lane of the block
// calls it (inactive lanes with act = false).  Lanes of a wave are NB lines
// (fast) by 64/NB positions: the eta maxima reduce over the positions, the
// xi maxima over the lines; wave speeds are clamped at zero as in the
// separate pass, so the maxima are bit-identical to it.
template <int SC, int NA, int NB, bool OPT>
WIU_DEV void fused_stage_out(const SweepArgs& s, SweepLds<SC, 1, NA, NB, OPT>& L, bool act, int line, int i, int o0,
                             int tb, const OutOperands& op) {
  static_assert(64 % NB == 0 && (NA * NB) % 64 == 0, "eta tile must pack whole waves");
  const Dims& d = s.d;
  double sx = 0.0, se = 0.0, cf = 0.0;
  bool bad = false;
  if (act) {
    double R[4];
    tile_residual<SC, 1, NA, NB, OPT>(L, tb, o0, i, R);
    const long long o = (long long)i * d.nx + line;
    const double rj = -rcp(op.jinv);
    const double dt = s.dt[0];
    double Qn[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      Qn[c] = op.x[c] + s.cb * (dt * (R[c] * rj));
      s.out[c * d.np + o] = Qn[c];
    }
    const WaveState w = wave_state(Qn, s.gamma);
    const double sxr = wave_speed_dir(w, op.km[0], op.km[1]);
    const double ser = wave_speed_dir(w, op.km[2], op.km[3]);
    bad = w.bad || !(sxr < 1.0e300) || !(ser < 1.0e300);
    sx = fmax(0.0, sxr);
    se = fmax(0.0, ser);
    if (s.ncfl) cf = fmax(0.0, (sx + ser) / op.jinv);
  }
  if (bad) atomicOr(s.status, ST_NONPHYS);
  // eta line (column) maxima: reduce over the positions of the wave
  for (int off = NB; off < 64; off <<= 1) se = fmax(se, __shfl_xor(se, off, 64));
  // xi line (row) maxima: reduce over the lines of the wave
  for (int off = 1; off < NB; off <<= 1) sx = fmax(sx, __shfl_xor(sx, off, 64));
  const int lane = (threadIdx.x + NB * threadIdx.y) & 63;
  if (lane < NB && line < d.nx) atomicMax(&s.nlam_eta[line], (unsigned long long)__double_as_longlong(se));
  if (tb == 0 && act) atomicMax(&s.nlam_xi[i], (unsigned long long)__double_as_longlong(sx));
  if (s.ncfl) {  // CFL maximum per eta line, reduced as the eta maxima
    for (int off = NB; off < 64; off <<= 1) cf = fmax(cf, __shfl_xor(cf, off, 64));
    if (lane < NB && line < d.nx) atomicMax(&s.ncfl[line], (unsigned long long)__double_as_longlong(cf));
  }
}

// One tile of a sweep: logical tile (bxl, byl) = (segment along the line,
// group of lines) for xi, (group of lines, segment) for eta.  Every thread of
// the block calls it with the same tile; it contains five block-wide
// barriers on every path that reaches the output phase, and none after.
// OPT: compiled with the scheme options (interpolation variables s.vars and
// the free parameter s.ah); without it the tile runs the paper's
// configuration (characteristic variables, alpha = 1) and carries no code
// for the options, which keeps its register count down.
template <int SC, int DIR, int NA, int NB, bool OPT>
WIU_DEV void sweep_tile(const SweepArgs& s, int bxl, int byl, SweepLds<SC, DIR, NA, NB, OPT>& L) {
  const double ah = OPT ? s.ah : 1.0;
  const bool alt = OPT && s.split != 0;                 // another midpoint split
  const int ppm = OPT && s.weights != 0 ? 2 : s.ppm;    // 2: WENO-Z weights
  using R_ = Range<SC>;
  constexpr int OUT = NA - R_::EXTRA;
  constexpr int NT = NA * NB;
  constexpr int QL = R_::QL;
  constexpr int NQ = SweepLds<SC, DIR, NA, NB, OPT>::NQ;
  auto& sh = L.sh;
  auto& sq = L.sq;

  const Dims& d = s.d;
  // metrics built for another scheme or grid: flag and do nothing (uniform
  // over the block, so no barrier is skipped by part of it)
  {
    const double* tag = s.M + 9 * d.mplane;
    if (tag[0] != TAG_MAGIC || tag[1] != (double)SC || tag[2] != (double)d.nx || tag[3] != (double)d.ny ||
        tag[6] != ah) {
      if (threadIdx.x == 0 && threadIdx.y == 0) atomicOr(s.status, ST_SCHEME);
      return;
    }
  }
  __syncthreads();  // LDS of the previous tile is free
  const int ta = DIR == 0 ? threadIdx.x : threadIdx.y;  // along
  const int tb = DIR == 0 ? threadIdx.y : threadIdx.x;  // across
  const int n_al = DIR == 0 ? d.nx : d.ny;
  const int n_ac = DIR == 0 ? d.ny : d.nx;
  const int bc_al = DIR == 0 ? d.bcx : d.bcy;
  const int line = (DIR == 0 ? byl : bxl) * NB + tb;
  const int o0 = (DIR == 0 ? bxl : byl) * OUT;
  const int out = min(OUT, n_al - o0);
  const int k = o0 + R_::LO + ta;
  using LT = SweepLds<SC, DIR, NA, NB, OPT>;
  const int slot = LT::si(tb, ta);
  const bool live = line < n_ac;

  // element offsets
  const long long mstride = DIR == 0 ? 1 : d.mpitch;
  const long long mline = DIR == 0 ? (long long)(line + GHOST) * d.mpitch + GHOST
                                   : (long long)GHOST * d.mpitch + (line + GHOST);
  const double* Mk = s.M + (DIR == 0 ? 0 : 2) * d.mplane;   // nodal k_x^ plane
  const double* Mm = s.M + (DIR == 0 ? 5 : 7) * d.mplane;   // midpoint plane
  const double gam = s.gamma;

  double lam = 0.0;
  if (live) {
    const unsigned long long* lp = DIR == 0 ? s.lam_xi : s.lam_eta;
    lam = s.alpha * __longlong_as_double((long long)lp[line]);
  }

  const bool need_node = live && k >= o0 + Traits<SC>::NLO && k < o0 + out + Traits<SC>::NHI;
  const bool need_mid = live && k >= o0 + Traits<SC>::MLO && k < o0 + out + Traits<SC>::MHI;

  // metrics of this thread's item, issued before the staging so that their
  // latency overlaps it
  const long long mo_k = mline + mstride * k;
  double kx0 = 0.0, ky0 = 0.0, kx1 = 0.0, ky1 = 0.0, mmx = 0.0, mmy = 0.0;
  if (need_node || need_mid) { kx0 = Mk[mo_k]; ky0 = Mk[d.mplane + mo_k]; }
  if (need_mid) {
    kx1 = Mk[mo_k + mstride]; ky1 = Mk[d.mplane + mo_k + mstride];
    mmx = Mm[mo_k]; mmy = Mm[d.mplane + mo_k];
  }

  // Stage the states of the tile (with the boundary rule applied) in LDS,
  // consecutive threads reading consecutive addresses.  Beyond the ends of a
  // non-periodic line the side's rule applies: transmissive (copy of the
  // boundary node), reflecting wall (mirror image about the boundary node,
  // momentum along the boundary node's metric direction reversed), a fixed
  // state, or an interface (the neighbouring block's nodes).
  {
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int k0 = o0 + R_::LO - QL;
    constexpr int S0 = DIR == 0 ? 0 : 2;  // this direction's low side
    // tiles whose window stays inside the line, or with no wall or fixed
    // side at the ends it reaches, load plainly (block-uniform test)
    const bool edge = bc_al != 0 && ((k0 < 0 && s.side[S0] != 0) || (k0 + NQ > n_al && s.side[S0 + 1] != 0));
    // tiles whose window lies inside the line need no index mapping at all
    const bool inside = k0 >= 0 && k0 + NQ <= n_al;
    // the thread's elements, NIT at most; in the paper's configuration every
    // load is issued before any is stored, so their latencies overlap (the
    // option kernels, short of registers, load and store one at a time)
    constexpr int NIT = (NQ * NB + NT - 1) / NT;
    constexpr int GRP = OPT ? 1 : NIT;
#pragma unroll
    for (int g0 = 0; g0 < NIT; g0 += GRP) {
      double Qs_[GRP][4];
#pragma unroll
      for (int it = 0; it < GRP; ++it) {
        const int e = tid + (g0 + it) * NT;
        if (e >= NQ * NB) break;
        const int pos = DIR == 0 ? e % NQ : e / NB;
        const int lb = DIR == 0 ? e / NQ : e % NB;
        const int ln = (DIR == 0 ? byl : bxl) * NB + lb;
        double* Qv = Qs_[it];
        if (inside) {
          if (ln < n_ac) {
            const int kr = k0 + pos;
            const long long o = DIR == 0 ? (long long)ln * d.nx + kr : (long long)kr * d.nx + ln;
#pragma unroll
            for (int c = 0; c < 4; ++c) Qv[c] = s.U[c * d.np + o];
          }
        } else if (ln < n_ac) {
          const int kr = k0 + pos;
          const bool lo = kr < 0;
          const int rule = (edge && (lo || kr >= n_al)) ? (lo ? s.side[S0] : s.side[S0 + 1]) : 0;
          if (rule == 2) {
#pragma unroll
            for (int c = 0; c < 4; ++c) Qv[c] = lo ? s.fixed[S0][c] : s.fixed[S0 + 1][c];
          } else if (rule == 3) {
            // interface: the neighbour's node; layers deeper than any stencil
            // reaches are clamped (staged but never used)
            const int sd = lo ? S0 : S0 + 1;
            const int m = min(lo ? -kr : kr - n_al + 1, WIU_MB_REACH - 1);
            const long long o = s.g0[sd] + m * s.gm[sd] + ln * s.gl[sd];
#pragma unroll
            for (int c = 0; c < 4; ++c) Qv[c] = s.nbU[sd][c * s.nbnp[sd] + o];
          } else {
            const int kb = lo ? 0 : n_al - 1;
            const int kk = rule == 1 ? min(max(2 * kb - kr, 0), n_al - 1) : bc_index(kr, n_al, bc_al);
            const long long o = DIR == 0 ? (long long)ln * d.nx + kk : (long long)kk * d.nx + ln;
#pragma unroll
            for (int c = 0; c < 4; ++c) Qv[c] = s.U[c * d.np + o];
            if (rule == 1) {
              const long long mb = DIR == 0 ? (long long)(ln + GHOST) * d.mpitch + (kb + GHOST)
                                            : (long long)(kb + GHOST) * d.mpitch + (ln + GHOST);
              const double bx = Mk[mb], by = Mk[d.mplane + mb];
              const double rn = rsqrt_(bx * bx + by * by);
              const double nbx = bx * rn, nby = by * rn;
              const double mn = Qv[1] * nbx + Qv[2] * nby;
              Qv[1] -= 2.0 * mn * nbx;
              Qv[2] -= 2.0 * mn * nby;
            }
          }
        }
      }
#pragma unroll
      for (int it = 0; it < GRP; ++it) {
        const int e = tid + (g0 + it) * NT;
        if (e >= NQ * NB) break;
        const int pos = DIR == 0 ? e % NQ : e / NB;
        const int lb = DIR == 0 ? e / NQ : e % NB;
        const int ln = (DIR == 0 ? byl : bxl) * NB + lb;
        if (ln < n_ac) {
#pragma unroll
          for (int c = 0; c < 4; ++c) sq[c][LT::qi(lb, pos)] = Qs_[it][c];
        }
      }
    }
  }
  __syncthreads();

  if (need_node || need_mid) {
    // stencil states Q_{k-QL..k+QL+1}, read from LDS where they are used
    auto q = [&](int m, int c) { return sq[c][LT::qi(tb, ta + m)]; };
    if (need_node) {
      const double qk[4] = {q(QL, 0), q(QL, 1), q(QL, 2), q(QL, 3)};
      double E[4];
      nodal_flux(qk, kx0, ky0, gam, E);
#pragma unroll
      for (int c = 0; c < 4; ++c) sh[c][slot] = E[c];
    }
    if (need_mid) {
      const double mx = mmx, my = mmy;
      const double nbx = 0.5 * (kx0 + kx1), nby = 0.5 * (ky0 + ky1);
      const double rn = rsqrt_(nbx * nbx + nby * nby);
      const double nx_ = nbx * rn, ny_ = nby * rn;
      // the two sides one after the other: the compiler barrier keeps their
      // working sets from being interleaved (register pressure)
      double D[4] = {0.0, 0.0, 0.0, 0.0};
      const int split = alt ? s.split : 0;
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        asm volatile("" ::: "memory");
        double F[4];
        if (OPT && s.vars != 0)
          side_flux_comp<Traits<SC>::R, OPT>(q, side, s.vars, mx, my, lam, gam, s.eps, ppm, F, split, D);
        else if constexpr (Traits<SC>::R == 4)
          side_flux7<OPT>(q, side, nx_, ny_, mx, my, lam, gam, s.eps, ppm, F, split, D);
        else
          side_flux<Traits<SC>::fifth, OPT>(q, side, nx_, ny_, mx, my, lam, gam, s.eps, ppm, F, split, D);
#pragma unroll
        for (int c = 0; c < 4; ++c) sh[4 + 4 * side + c][slot] = F[c];
      }
      if constexpr (OPT) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sh[12 + c][slot] = D[c];
      }
    }
  }

  // epilogue operands of this thread's output node, issued before the barrier
  const bool act = live && ta < out;
  const int i = o0 + ta;                  // output node along the line
  const int ii = DIR == 0 ? i : line, jj = DIR == 0 ? line : i;
  const long long o = (long long)jj * d.nx + ii;
  const long long mo = (long long)(jj + GHOST) * d.mpitch + (ii + GHOST);
  const bool fused = DIR == 1 && s.mode == 2 && s.nlam_xi;
  OutOperands op;
#pragma unroll
  for (int c = 0; c < 4; ++c) op.x[c] = op.km[c] = 0.0;
  op.jinv = 1.0;
  if (act && s.mode != 0) {
    op.jinv = s.M[4 * d.mplane + mo];
    const double* src = s.mode == 3 ? (s.ca != 0.0 ? s.U0 : nullptr) : s.Rxi;
    if (src) {
#pragma unroll
      for (int c = 0; c < 4; ++c) op.x[c] = src[c * d.np + o];
    }
    if (fused) {
#pragma unroll
      for (int c = 0; c < 4; ++c) op.km[c] = s.M[c * d.mplane + mo];
    }
  }
  __syncthreads();

  // H_{k+1/2} once per item, for the midpoints k + 1/2 of k in [o0 - 1,
  // o0 + out), into the item's nodal-flux slots once every record is read
  {
    const bool hact = live && k >= o0 - 1 && k < o0 + out;
    double Hk[4];
    if (hact) {
      const int qs = LT::qi(tb, ta + QL);
#pragma unroll
      for (int c = 0; c < 4; ++c) Hk[c] = tile_hsum<SC, DIR, NA, NB, OPT>(L, c, slot, qs, k, lam, ah, alt);
    }
    __syncthreads();
    if (hact) {
#pragma unroll
      for (int c = 0; c < 4; ++c) sh[c][slot] = Hk[c];
    }
    __syncthreads();
  }

  if constexpr (DIR == 1) {
    if (fused) {  // whole waves take part in the reductions
      fused_stage_out<SC, NA, NB, OPT>(s, L, act, line, i, o0, tb, op);
      return;
    }
  }
  if (!act) return;  // no barrier follows
  double R[4];
  tile_residual<SC, DIR, NA, NB, OPT>(L, tb, o0, i, R);
  if (s.mode == 0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) s.Rxi[c * d.np + o] = R[c];
    return;
  }
  const double rj = -rcp(op.jinv);
  if (s.mode == 1) {
#pragma unroll
    for (int c = 0; c < 4; ++c) s.out[c * d.np + o] = (op.x[c] + R[c]) * rj;
    return;
  }
  const double dt = s.dt[0];
  if (s.mode == 3) {
    // xi part of the stage update, P = ca U0 + cb (Us + dt R^xi / -J^{-1}),
    // into the R^xi buffer; the stage state at the output node is the staged
    // tile entry (an interior node, untouched by the boundary rule), and U0
    // is not read when its coefficient is zero (first stage)
    const int pq = LT::qi(tb, i - (o0 + R_::LO - QL));
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double un = s.cb * (sq[c][pq] + dt * (R[c] * rj));
      s.Rxi[c * d.np + o] = s.ca == 0.0 ? un : s.ca * op.x[c] + un;
    }
    return;
  }
  // mode 2: U_out = P + cb dt R^eta / -J^{-1}
#pragma unroll
  for (int c = 0; c < 4; ++c) s.out[c * d.np + o] = op.x[c] + s.cb * (dt * (R[c] * rj));
}


}  // namespace wiu
