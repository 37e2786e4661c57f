// ---------------------------------------------------------------------------
// Multi-block grids in the reference oracle -- TEST INFRASTRUCTURE ONLY.
//
// The paper motivates its schemes with multi-block grids (Sec. 1) but gives
// no rule for coupling blocks; this is the library's.  Blocks are
// right-handed structured grids.  A side of a non-periodic direction may be
// an interface to a side of another block (or of the same block) with the
// same number of nodes; the lines of the block then continue into the
// neighbour:
//   * states beyond the side are the neighbour's nodes (no overlap: the first
//     ghost layer is the neighbour's boundary layer);
//   * coordinates beyond the side are the neighbour's, plus a constant shift
//     (non-zero only across a periodic seam), so the metrics of both blocks
//     are evaluated on one coordinate field (free-stream preservation and
//     conservation across the interface, Secs. 2.2-2.4);
//   * the Lax-Friedrichs eigenvalue of a line (Sec. 2.3) is the maximum over
//     the whole line through all the blocks it crosses, so both blocks split
//     the flux at the interface identically;
//   * blocks joined by interfaces advance with one time step.
// Sides are numbered x lo (0), x hi (1), y lo (2), y hi (3).  Along side s a
// node has a position t, counted counterclockwise around the block, and a
// depth d inward (0 on the side).  Two right-handed blocks meet with their
// counterclockwise orders opposed, so position t of one side is position
// n - 1 - t of the other, and ghost depth m >= 1 is the neighbour's depth
// m - 1: the index map of an interface is fixed by the pair of sides.
// ---------------------------------------------------------------------------
#pragma once

#include "wenoiu_oracle.hpp"

#include <numeric>
#include <stdexcept>

namespace orc {

struct Block {
  Grid g;  // g.side[s] == SIDE_INTERFACE marks an interface side
  const double* x = nullptr;
  const double* y = nullptr;
  int nbr[4] = {-1, -1, -1, -1};  // neighbour block across an interface side
  int nbr_side[4] = {0, 0, 0, 0};  // the neighbour's side that abuts it
  double shift[4][2] = {};         // added to the neighbour's coordinates
};

inline int side_len(int s, int nx, int ny) { return s < 2 ? ny : nx; }

// Node (a, c) of an nx x ny block from (position t, depth d) along side s.
inline void side_node(int s, int nx, int ny, int t, int d, int& a, int& c) {
  switch (s) {
    case 0: a = d; c = ny - 1 - t; break;
    case 1: a = nx - 1 - d; c = t; break;
    case 2: a = t; c = d; break;
    default: a = nx - 1 - t; c = ny - 1 - d; break;
  }
}

// (position, depth) along side s of node (a, c).
inline void side_frame(int s, int nx, int ny, int a, int c, int& t, int& d) {
  switch (s) {
    case 0: t = ny - 1 - c; d = a; break;
    case 1: t = c; d = nx - 1 - a; break;
    case 2: t = a; d = c; break;
    default: t = nx - 1 - a; d = ny - 1 - c; break;
  }
}

// Position (a, c) beyond interface side s of block b, as a position (a2, c2)
// of the neighbour b2.
inline void through(const std::vector<Block>& B, int b, int s, int a, int c, int& b2, int& a2, int& c2) {
  const Grid& g = B[b].g;
  int t, d;
  side_frame(s, g.nx, g.ny, a, c, t, d);
  b2 = B[b].nbr[s];
  const Grid& g2 = B[b2].g;
  side_node(B[b].nbr_side[s], g2.nx, g2.ny, side_len(s, g.nx, g.ny) - 1 - t, -d - 1, a2, c2);
}

// Coordinates of block b at any position within the reach of the metrics.
// Periodic directions wrap; beyond an interface side the neighbour's
// coordinates (shifted) are read, the side of the xi direction taking
// precedence at a corner; positions beyond no interface extend the block's
// own nodes linearly (as for a single grid).  A corner reached through an
// interface lies beyond a side of the neighbour, so at most two interfaces
// are crossed.
inline void mb_coord(const std::vector<Block>& B, int b, int a, int c, long double& X, long double& Y) {
  long double sx = 0.0L, sy = 0.0L;
  for (int hop = 0; hop < 4; ++hop) {
    const Block& k = B[b];
    const Grid& g = k.g;
    if (g.bcx == PERIODIC) { sx += (long double)floordiv(a, g.nx) * (long double)g.Lx; a = wrap(a, g.nx); }
    if (g.bcy == PERIODIC) { sy += (long double)floordiv(c, g.ny) * (long double)g.Ly; c = wrap(c, g.ny); }
    int s = -1;
    if ((a < 0 || a >= g.nx) && g.side[a < 0 ? 0 : 1] == SIDE_INTERFACE) s = a < 0 ? 0 : 1;
    else if ((c < 0 || c >= g.ny) && g.side[c < 0 ? 2 : 3] == SIDE_INTERFACE) s = c < 0 ? 2 : 3;
    if (s < 0) {
      Coords{g, k.x, k.y}.at(a, c, X, Y);
      X += sx; Y += sy;
      return;
    }
    sx += (long double)k.shift[s][0];
    sy += (long double)k.shift[s][1];
    int b2, a2, c2;
    through(B, b, s, a, c, b2, a2, c2);
    b = b2; a = a2; c = c2;
  }
  throw std::runtime_error("mb_coord: position beyond the reach of the interfaces");
}

struct BlockCoords {
  const std::vector<Block>& B;
  int b;
  void at(int a, int c, long double& X, long double& Y) const { mb_coord(B, b, a, c, X, Y); }
};

// Reach of the metric evaluation beyond a side: the stored ghost band plus
// the midpoint interpolation (nodal band, at most G + 4) plus the widest
// central operator (7).
constexpr int MB_REACH = G + 4 + 7;

// Interfaces must pair up, match in length, join non-periodic directions and
// lead into blocks deep enough for that reach.
inline bool mb_valid(const std::vector<Block>& B) {
  const int n = (int)B.size();
  for (int b = 0; b < n; ++b) {
    const Grid& g = B[b].g;
    if (g.nx < 2 || g.ny < 2) return false;
    for (int s = 0; s < 4; ++s) {
      if (g.side[s] < SIDE_TRANSMISSIVE || g.side[s] > SIDE_INTERFACE) return false;
      if (g.side[s] != SIDE_INTERFACE) continue;
      if ((s < 2 ? g.bcx : g.bcy) == PERIODIC) return false;
      const int b2 = B[b].nbr[s], s2 = B[b].nbr_side[s];
      if (b2 < 0 || b2 >= n || s2 < 0 || s2 > 3) return false;
      const Grid& h = B[b2].g;
      if (h.side[s2] != SIDE_INTERFACE || B[b2].nbr[s2] != b || B[b2].nbr_side[s2] != s) return false;
      if (b2 == b && s2 == s) return false;
      if (side_len(s, g.nx, g.ny) != side_len(s2, h.nx, h.ny)) return false;
      if ((s2 < 2 ? h.nx : h.ny) < MB_REACH) return false;
      if (B[b2].shift[s2][0] != -B[b].shift[s][0] || B[b2].shift[s2][1] != -B[b].shift[s][1]) return false;
    }
  }
  return true;
}

// Metrics of block b, ghost band included, on the coupled coordinates.
inline void mb_metrics(Scheme sc, double alpha_h, const std::vector<Block>& B, int b, double* M) {
  compute_metrics_from(sc, alpha_h, B[b].g, BlockCoords{B, b}, M);
}

// Lines across blocks.  Line ids: block b's xi line j is base[b] + j, its
// eta line i is base[b] + ny + i.  Lines joined through interfaces form one
// group (union-find); blocks joined through interfaces form one component.
struct MbLines {
  std::vector<int> base, group, comp;
};

inline int uf_find(std::vector<int>& p, int v) {
  while (p[v] != v) { p[v] = p[p[v]]; v = p[v]; }
  return v;
}

inline MbLines mb_lines(const std::vector<Block>& B) {
  const int n = (int)B.size();
  MbLines L;
  L.base.resize(n + 1, 0);
  for (int b = 0; b < n; ++b) L.base[b + 1] = L.base[b] + B[b].g.nx + B[b].g.ny;
  L.group.resize(L.base[n]);
  std::iota(L.group.begin(), L.group.end(), 0);
  L.comp.resize(n);
  std::iota(L.comp.begin(), L.comp.end(), 0);
  auto line_of = [&](int b, int s, int a, int c) {  // line through node (a, c) normal to side s
    return L.base[b] + (s < 2 ? c : B[b].g.ny + a);
  };
  for (int b = 0; b < n; ++b)
    for (int s = 0; s < 4; ++s) {
      if (B[b].g.side[s] != SIDE_INTERFACE) continue;
      const Grid& g = B[b].g;
      const int b2 = B[b].nbr[s], s2 = B[b].nbr_side[s];
      const int len = side_len(s, g.nx, g.ny);
      for (int t = 0; t < len; ++t) {
        int a, c, a2, c2;
        side_node(s, g.nx, g.ny, t, 0, a, c);
        side_node(s2, B[b2].g.nx, B[b2].g.ny, len - 1 - t, 0, a2, c2);
        const int r1 = uf_find(L.group, line_of(b, s, a, c)), r2 = uf_find(L.group, line_of(b2, s2, a2, c2));
        if (r1 != r2) L.group[r1] = r2;
      }
      const int q1 = uf_find(L.comp, b), q2 = uf_find(L.comp, b2);
      if (q1 != q2) L.comp[q1] = q2;
    }
  for (auto& v : L.group) v = uf_find(L.group, v);
  for (auto& v : L.comp) v = uf_find(L.comp, v);
  return L;
}

// dU/dt of every block (Eq. 2.2 with the coupling above).
template <class T>
void mb_rhs(Scheme sc, const Params& pr, const std::vector<Block>& B, const std::vector<const T*>& U,
            const std::vector<const double*>& M, const std::vector<T*>& dUdt) {
  const int n = (int)B.size();
  const MbLines L = mb_lines(B);
  // Sec. 2.3: maximum wave speed over each line, then over each group of lines
  std::vector<T> smax(L.base[n], T(0.0));
  std::vector<char> seen(L.base[n], 0);
  for (int b = 0; b < n; ++b) {
    const Grid& g = B[b].g;
    const size_t NP = (size_t)g.nx * g.ny;
    MetricView mv{g.nx, g.ny, M[b]};
    for (int j = 0; j < g.ny; ++j)
      for (int i = 0; i < g.nx; ++i) {
        const size_t o = (size_t)j * g.nx + i;
        T Q[4] = {U[b][o], U[b][NP + o], U[b][2 * NP + o], U[b][3 * NP + o]};
        const int lx = L.group[L.base[b] + j], le = L.group[L.base[b] + g.ny + i];
        T sx = wave_speed(Q, pr.gamma, mv(0, i, j), mv(1, i, j));
        T se = wave_speed(Q, pr.gamma, mv(2, i, j), mv(3, i, j));
        if (!seen[lx] || sx > smax[lx]) { smax[lx] = sx; seen[lx] = 1; }
        if (!seen[le] || se > smax[le]) { smax[le] = se; seen[le] = 1; }
      }
  }
  for (int b = 0; b < n; ++b) {
    const Grid& g = B[b].g;
    std::vector<T> sxi(g.ny), seta(g.nx);
    for (int j = 0; j < g.ny; ++j) sxi[j] = smax[L.group[L.base[b] + j]];
    for (int i = 0; i < g.nx; ++i) seta[i] = smax[L.group[L.base[b] + g.ny + i]];
    Coupling<T> cp;
    cp.smax_xi = sxi.data();
    cp.smax_eta = seta.data();
    cp.ghost = [&](int s, int m, int line, int q) -> T {
      int a, c;  // position of the ghost node in block b
      switch (s) {
        case 0: a = -m; c = line; break;
        case 1: a = g.nx - 1 + m; c = line; break;
        case 2: a = line; c = -m; break;
        default: a = line; c = g.ny - 1 + m; break;
      }
      int b2, a2, c2;
      through(B, b, s, a, c, b2, a2, c2);
      const Grid& h = B[b2].g;
      return U[b2][(size_t)q * h.nx * h.ny + (size_t)c2 * h.nx + a2];
    };
    rhs<T>(sc, pr, g, U[b], M[b], dUdt[b], nullptr, nullptr, nullptr, &cp);
  }
}

// One TVD-RK3 step (Sec. 6) of all blocks; dt[b] per block (equal within a
// component for conservation across its interfaces).
inline void mb_rk3_step(Scheme sc, const Params& pr, const std::vector<Block>& B, const std::vector<double*>& U,
                        const std::vector<const double*>& M, const double* dt) {
  const int n = (int)B.size();
  std::vector<std::vector<double>> L(n), U1(n), U2(n);
  std::vector<const double*> src(n);
  std::vector<double*> out(n);
  for (int b = 0; b < n; ++b) {
    const size_t N = 4 * (size_t)B[b].g.nx * B[b].g.ny;
    L[b].resize(N); U1[b].resize(N); U2[b].resize(N);
    src[b] = U[b]; out[b] = L[b].data();
  }
  mb_rhs<double>(sc, pr, B, src, M, out);
  for (int b = 0; b < n; ++b) {
    for (size_t e = 0; e < L[b].size(); ++e) U1[b][e] = U[b][e] + dt[b] * L[b][e];
    src[b] = U1[b].data();
  }
  mb_rhs<double>(sc, pr, B, src, M, out);
  for (int b = 0; b < n; ++b) {
    for (size_t e = 0; e < L[b].size(); ++e) U2[b][e] = 0.75 * U[b][e] + 0.25 * (U1[b][e] + dt[b] * L[b][e]);
    src[b] = U2[b].data();
  }
  mb_rhs<double>(sc, pr, B, src, M, out);
  for (int b = 0; b < n; ++b)
    for (size_t e = 0; e < L[b].size(); ++e)
      U[b][e] = (1.0 / 3.0) * U[b][e] + (2.0 / 3.0) * (U2[b][e] + dt[b] * L[b][e]);
}

// CFL time step of each block: the single-grid rule over its component.
inline void mb_cfl_dt(const Params& pr, const std::vector<Block>& B, const std::vector<const double*>& U,
                      const std::vector<const double*>& M, double cfl, double* dt) {
  const int n = (int)B.size();
  const MbLines L = mb_lines(B);
  std::vector<double> cmin(n, 0.0);
  std::vector<char> seen(n, 0);
  for (int b = 0; b < n; ++b) {
    const double d = cfl_dt(pr, B[b].g, U[b], M[b], cfl);
    const int r = L.comp[b];
    if (!seen[r] || d < cmin[r]) { cmin[r] = d; seen[r] = 1; }
  }
  for (int b = 0; b < n; ++b) dt[b] = cmin[L.comp[b]];
}

}  // namespace orc
