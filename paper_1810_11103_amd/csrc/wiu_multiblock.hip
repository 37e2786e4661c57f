// Multi-block grids of libwenoiu (gfx950, fp64): validation of a block set,
// metrics on the coordinates of blocks coupled through interfaces, and the
// maxima of grid lines that cross blocks.  The coupling rule is the
// library's (the paper motivates multi-block grids, Sec. 1, but defines no
// coupling); it is stated with wiu_block in wenoiu.h.
#include "wenoiu.h"
#include "wiu_kernels.hpp"
#include "wiu_mb.hpp"

#include <vector>

namespace wiu {

namespace {

bool fixed_ok(const double* q) {
  const double rho = q[0];
  if (!(rho > 0.0) || !(rho < 1.0e300)) return false;
  const double p = q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / rho;  // (gamma - 1) p
  return p > 0.0 && p < 1.0e300;
}

bool periodic_dir(const wiu_block& b, int s) { return (s < 2 ? b.bc_x : b.bc_y) == WIU_BC_PERIODIC; }

}  // namespace

bool mb_blocks_ok(const wiu_block* blocks, int n) {
  if (!blocks || n < 1) return false;
  for (int i = 0; i < n; ++i) {
    const wiu_block& b = blocks[i];
    if (b.nx < 1 || b.ny < 1) return false;
    if (b.bc_x < 0 || b.bc_x > 1 || b.bc_y < 0 || b.bc_y > 1) return false;
    if (b.bc_x == WIU_BC_TRANSMISSIVE && b.nx < 2) return false;
    if (b.bc_y == WIU_BC_TRANSMISSIVE && b.ny < 2) return false;
    if (b.bc_x == WIU_BC_PERIODIC && !(b.period_x > 0.0 && b.period_x < 1.0e300)) return false;
    if (b.bc_y == WIU_BC_PERIODIC && !(b.period_y > 0.0 && b.period_y < 1.0e300)) return false;
    if (b.off_U < 0 || b.off_M < 0 || b.off_X < 0) return false;
    if (b.ny > 65535 * 4 || b.nx > (1 << 28)) return false;
    for (int s = 0; s < 4; ++s) {
      if (periodic_dir(b, s)) continue;
      const int k = b.side[s];
      if (k < WIU_SIDE_TRANSMISSIVE || k > WIU_SIDE_INTERFACE) return false;
      if (k == WIU_SIDE_FIXED && !fixed_ok(b.fixed[s])) return false;
      if (k != WIU_SIDE_INTERFACE) continue;
      const int j = b.nbr[s], s2 = b.nbr_side[s];
      if (j < 0 || j >= n || s2 < 0 || s2 > 3 || (j == i && s2 == s)) return false;
      const wiu_block& h = blocks[j];
      if (periodic_dir(h, s2) || h.side[s2] != WIU_SIDE_INTERFACE || h.nbr[s2] != i || h.nbr_side[s2] != s)
        return false;
      if (mb_side_len(s, b.nx, b.ny) != mb_side_len(s2, h.nx, h.ny)) return false;
      if ((s2 < 2 ? h.nx : h.ny) < WIU_MB_REACH) return false;
      for (int c = 0; c < 2; ++c)
        if (!(b.shift[s][c] > -1.0e300 && b.shift[s][c] < 1.0e300) || h.shift[s2][c] != -b.shift[s][c])
          return false;
    }
  }
  return true;
}

// ===========================================================================
// Coupled coordinates.  A position of block b is resolved to a node
// coordinate (the base) plus an offset: the linear extension beyond sides
// without an interface (rows, then columns: bilinear at corners, as for a
// single grid) and the shifts of the seams crossed.  Differences of nearby
// positions then take the base difference error-free and keep their digits
// across seams.  At most two interfaces are crossed (a corner reached through
// one lies beyond a side of the neighbour, which is at least WIU_MB_REACH
// nodes deep); the third pass extends the block's own nodes, with clamped
// indices, whatever the table holds.
// ===========================================================================
struct MbPoint {
  double bx, by, ox, oy;
};

WIU_DEV MbPoint mb_point(const MbCoord* __restrict__ tbl, const double* __restrict__ X, int b, int a, int c) {
  double ox = 0.0, oy = 0.0;
  for (int hop = 0;; ++hop) {
    const MbCoord& k = tbl[b];
    if (k.bcx == WIU_BC_PERIODIC) {
      const int w = bc_index(a, k.nx, 0);
      ox += (double)((a - w) / k.nx) * k.Lx;
      a = w;
    }
    if (k.bcy == WIU_BC_PERIODIC) {
      const int w = bc_index(c, k.ny, 0);
      oy += (double)((c - w) / k.ny) * k.Ly;
      c = w;
    }
    int s = -1;
    if (hop < 2) {
      if ((a < 0 || a >= k.nx) && k.side[a < 0 ? 0 : 1] == WIU_SIDE_INTERFACE) s = a < 0 ? 0 : 1;
      else if ((c < 0 || c >= k.ny) && k.side[c < 0 ? 2 : 3] == WIU_SIDE_INTERFACE) s = c < 0 ? 2 : 3;
    }
    if (s < 0) {
      const double* x = X + k.offX;
      const double* y = x + (long long)k.nx * k.ny;
      const int ca = min(max(a, 0), k.nx - 1), cc = min(max(c, 0), k.ny - 1);
      const double ea = (double)abs(a - ca), ec = (double)abs(c - cc);
      const int ia = a == ca ? ca : (a < 0 ? 1 : k.nx - 2);  // inward neighbour of the clamped node
      const int ic = c == cc ? cc : (c < 0 ? 1 : k.ny - 2);
      auto at = [&](const double* p, int aa, int cy) { return p[(long long)cy * k.nx + aa]; };
      MbPoint r;
      r.bx = at(x, ca, cc);
      r.by = at(y, ca, cc);
      const double xa = r.bx - at(x, ia, cc), ya = r.by - at(y, ia, cc);
      const double xc = r.bx - at(x, ca, ic), yc = r.by - at(y, ca, ic);
      const double xx = xa - (at(x, ca, ic) - at(x, ia, ic)), yx = ya - (at(y, ca, ic) - at(y, ia, ic));
      r.ox = ox + (ea * xa + ec * xc + ea * ec * xx);
      r.oy = oy + (ea * ya + ec * yc + ea * ec * yx);
      return r;
    }
    ox += k.shift[s][0];
    oy += k.shift[s][1];
    const int b2 = k.nbr[s];
    int a2, c2;
    mb_through(s, k.nx, k.ny, k.nbr_side[s], tbl[b2].nx, tbl[b2].ny, a, c, a2, c2);
    b = b2; a = a2; c = c2;
  }
}

WIU_DEV void mb_diff(const MbPoint& p1, const MbPoint& p0, double& dx, double& dy) {
  double s, e;
  two_sum(p1.bx, -p0.bx, s, e);
  dx = s + ((p1.ox - p0.ox) + e);
  two_sum(p1.by, -p0.by, s, e);
  dy = s + ((p1.oy - p0.oy) + e);
}

// Nodal metrics of block b on the band of width B (Sec. 2.2 in two
// dimensions with the scheme's central operator), T[5][(ny+2B)(nx+2B)].
// Periodic directions evaluate at the wrapped node, as for a single grid.
__global__ void mb_metrics_nodal_kernel(const MbCoord* __restrict__ tbl, int b, MetricStencil ms, int B,
                                        const double* __restrict__ X, double* __restrict__ T) {
  const int nx = tbl[b].nx, ny = tbl[b].ny;
  const int W = nx + 2 * B, Hh = ny + 2 * B;
  const int ta = blockIdx.x * blockDim.x + threadIdx.x;
  const int tb = blockIdx.y * blockDim.y + threadIdx.y;
  if (ta >= W || tb >= Hh) return;
  int a = ta - B, c = tb - B;
  if (tbl[b].bcx == WIU_BC_PERIODIC) a = bc_index(a, nx, 0);
  if (tbl[b].bcy == WIU_BC_PERIODIC) c = bc_index(c, ny, 0);
  double x_xi = 0.0, y_xi = 0.0, x_eta = 0.0, y_eta = 0.0;
  for (int m = 1; m <= METRIC_REACH; ++m) {
    const double cm = ms.d[m - 1];
    if (cm == 0.0) continue;
    double dx, dy;
    mb_diff(mb_point(tbl, X, b, a + m, c), mb_point(tbl, X, b, a - m, c), dx, dy);
    x_xi += cm * dx;
    y_xi += cm * dy;
    mb_diff(mb_point(tbl, X, b, a, c + m), mb_point(tbl, X, b, a, c - m), dx, dy);
    x_eta += cm * dx;
    y_eta += cm * dy;
  }
  const long long P = (long long)W * Hh, o = (long long)tb * W + ta;
  T[0 * P + o] = y_eta;
  T[1 * P + o] = -x_eta;
  T[2 * P + o] = -y_xi;
  T[3 * P + o] = x_xi;
  T[4 * P + o] = x_xi * y_eta - x_eta * y_xi;
}

// Line maxima of lines that cross blocks: every member of a group takes the
// group's maximum (raw bit patterns of non-negative doubles).
__global__ void group_max_kernel(unsigned long long* __restrict__ lam, const int* __restrict__ start,
                                 const int* __restrict__ mem, int ngroups) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ngroups) return;
  unsigned long long m = 0;
  for (int e = start[g]; e < start[g + 1]; ++e) m = max(m, lam[mem[e]]);
  for (int e = start[g]; e < start[g + 1]; ++e) lam[mem[e]] = m;
}

hipError_t launch_group_max(unsigned long long* lam, const int* start, const int* mem, int ngroups, hipStream_t st) {
  if (ngroups <= 0) return hipSuccess;
  hipLaunchKernelGGL(group_max_kernel, dim3((ngroups + 255) / 256), dim3(256), 0, st, lam, start, mem, ngroups);
  return hipGetLastError();
}

Dims mb_dims(const wiu_block& b) {
  Dims d;
  d.nx = b.nx; d.ny = b.ny; d.bcx = b.bc_x; d.bcy = b.bc_y;
  d.mpitch = b.nx + 2 * GHOST;
  d.mplane = (long long)(b.nx + 2 * GHOST) * (b.ny + 2 * GHOST);
  d.np = (long long)b.nx * b.ny;
  d.Lx = b.period_x; d.Ly = b.period_y;
  return d;
}

}  // namespace wiu

using namespace wiu;

namespace {

constexpr size_t MB_ALIGN = 256;
size_t mb_align(size_t v) { return (v + MB_ALIGN - 1) / MB_ALIGN * MB_ALIGN; }

size_t band_bytes(const wiu_block& b, int B) { return 5 * (size_t)(b.nx + 2 * B) * (b.ny + 2 * B) * sizeof(double); }

}  // namespace

extern "C" {

size_t wiu_blocks_metrics_work_size(const wiu_block* blocks, int nblocks, int scheme) {
  if (scheme < 0 || scheme > 7 || !mb_blocks_ok(blocks, nblocks)) return 0;
  const int B = metric_band(scheme);
  size_t band = 0;
  for (int b = 0; b < nblocks; ++b) band = band_bytes(blocks[b], B) > band ? band_bytes(blocks[b], B) : band;
  return MB_ALIGN + mb_align(sizeof(MbCoord) * nblocks) + band;
}

int wiu_blocks_metrics(const wiu_block* blocks, int nblocks, int scheme, const wiu_params* p, const double* X_all,
                       double* M_all, void* work, wiu_stream_t stream) {
  if (!X_all || !M_all || !work || scheme < 0 || scheme > 7) return WIU_EINVAL;
  if (!mb_blocks_ok(blocks, nblocks)) return WIU_EINVAL;
  const double ah = p ? p->alpha_h : 1.0;
  if (!(ah > 0.0 && ah < 1.0e300) ||
      (ah != 1.0 && scheme != WIU_3_1MP && scheme != WIU_5_1MP && scheme != WIU_7_1MP))
    return WIU_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  std::vector<MbCoord> tbl(nblocks);
  for (int b = 0; b < nblocks; ++b) {
    const wiu_block& k = blocks[b];
    MbCoord& c = tbl[b];
    c.nx = k.nx; c.ny = k.ny; c.bcx = k.bc_x; c.bcy = k.bc_y; c.Lx = k.period_x; c.Ly = k.period_y;
    c.offX = k.off_X;
    for (int s = 0; s < 4; ++s) {
      // sides of periodic directions are never crossed
      c.side[s] = periodic_dir(k, s) ? WIU_SIDE_TRANSMISSIVE : k.side[s];
      c.nbr[s] = c.side[s] == WIU_SIDE_INTERFACE ? k.nbr[s] : 0;
      c.nbr_side[s] = k.nbr_side[s];
      c.shift[s][0] = k.shift[s][0];
      c.shift[s][1] = k.shift[s][1];
    }
  }
  char* w = (char*)work;
  MbCoord* d_tbl = (MbCoord*)(w + MB_ALIGN);
  double* T = (double*)(w + MB_ALIGN + mb_align(sizeof(MbCoord) * nblocks));
  int* status = (int*)w;
  if (hipMemcpyAsync(d_tbl, tbl.data(), sizeof(MbCoord) * nblocks, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return WIU_EHIP;
  if (launch_zero_header(status, 1, st) != hipSuccess) return WIU_EHIP;
  const int B = metric_band(scheme);
  const MetricStencil ms = metric_stencil(scheme, ah);
  for (int b = 0; b < nblocks; ++b) {
    const Dims d = mb_dims(blocks[b]);
    dim3 blk(64, 4);
    dim3 grd((d.nx + 2 * B + 63) / 64, (d.ny + 2 * B + 3) / 4);
    hipLaunchKernelGGL(mb_metrics_nodal_kernel, grd, blk, 0, st, d_tbl, b, ms, B, X_all, T);
    if (hipGetLastError() != hipSuccess) return WIU_EHIP;
    if (launch_metrics_band(d, scheme, ah, B, T, M_all + blocks[b].off_M, status, st) != hipSuccess) return WIU_EHIP;
  }
  return WIU_OK;
}

}  // extern "C"
