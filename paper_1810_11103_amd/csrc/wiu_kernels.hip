// HIP kernels of libwenoiu for gfx950 (fp64 throughout, no MFMA: nothing on
// this path is a dense contraction).
//
//   metrics_nodal_kernel / metrics_band_kernel  grid metrics (Secs. 2.2-2.4)
//   wave_max_kernel                             line maxima of |U^| + c|k^| and
//                                               the CFL maximum (Sec. 2.3)
//   sweep_kernel<scheme, dir>                   residual of one direction (Sec. 3)
//                                               with the residual / RK epilogue
#include "wiu_kernels.hpp"
#include "wiu_sweep.hpp"

namespace wiu {

// ===========================================================================
// Metrics.  Coordinates are extended beyond the grid by the boundary rule
// (periodic: repeat shifted by the period; transmissive: linear extension
// from the last two nodes, applied per direction, so the extension is the
// bilinear tensor-product one).  Derivatives are taken on coordinate
// differences X(i+m) - X(i-m), never on absolute coordinates, so the metric
// keeps full relative accuracy on large or offset domains.
// ===========================================================================

// c[i1] - c[i0] + k L with i0, i1 inside [0, n): when the shift is non-zero
// the difference of the stored values is close to -k L and is corrected
// without rounding at the size of L.
WIU_DEV double shifted_diff(double c1, double c0, int k, double L) {
  if (k == 0) return c1 - c0;
  double s, e;
  two_sum(c1, -c0, s, e);
  return (s + (double)k * L) + e;
}

// Along one real line of n values c[stride * t]: difference X(a1) - X(a0)
// for arbitrary integer a1, a0 under the boundary rule.  `shift` says whether
// this coordinate is the one the period shifts (x along i, y along j).
struct LineDiff {
  const double* c;
  long long stride;
  int n, bc;
  double L;
  bool shift;
  WIU_DEV double at(int t) const { return c[stride * t]; }
  WIU_DEV double operator()(int a1, int a0) const {
    if (bc == 0) {
      int w1 = a1, k1 = 0, w0 = a0, k0 = 0;
      while (w1 < 0) { w1 += n; --k1; }
      while (w1 >= n) { w1 -= n; ++k1; }
      while (w0 < 0) { w0 += n; --k0; }
      while (w0 >= n) { w0 -= n; ++k0; }
      return shifted_diff(at(w1), at(w0), shift ? (k1 - k0) : 0, L);
    }
    // transmissive: X(a) = X(clamp(a)) + (a - clamp(a)) * step at that end
    int c1 = a1 < 0 ? 0 : (a1 >= n ? n - 1 : a1);
    int c0 = a0 < 0 ? 0 : (a0 >= n ? n - 1 : a0);
    double d = at(c1) - at(c0);
    if (a1 != c1) d += (double)(a1 - c1) * (a1 < 0 ? at(1) - at(0) : at(n - 1) - at(n - 2));
    if (a0 != c0) d -= (double)(a0 - c0) * (a0 < 0 ? at(1) - at(0) : at(n - 1) - at(n - 2));
    return d;
  }
};

// Difference along i of coordinate array c (x or y) on row b (any integer):
// rows outside a transmissive range extend linearly from the last two rows.
WIU_DEV double diff_i(const Dims& d, const double* c, bool is_x, int b, int a1, int a0) {
  auto row = [&](int r) {
    LineDiff ld{c + (long long)r * d.nx, 1, d.nx, d.bcx, d.Lx, is_x};
    return ld(a1, a0);
  };
  if (d.bcy == 0) return row(bc_index(b, d.ny, 0));
  if (b < 0) { double d0 = row(0), d1 = row(1); return d0 + (double)b * (d1 - d0); }
  if (b >= d.ny) {
    double dl = row(d.ny - 1), d2 = row(d.ny - 2);
    return dl + (double)(b - d.ny + 1) * (dl - d2);
  }
  return row(b);
}

WIU_DEV double diff_j(const Dims& d, const double* c, bool is_y, int a, int b1, int b0) {
  auto col = [&](int cidx) {
    LineDiff ld{c + cidx, d.nx, d.ny, d.bcy, d.Ly, is_y};
    return ld(b1, b0);
  };
  if (d.bcx == 0) return col(bc_index(a, d.nx, 0));
  if (a < 0) { double d0 = col(0), d1 = col(1); return d0 + (double)a * (d1 - d0); }
  if (a >= d.nx) {
    double dl = col(d.nx - 1), d2 = col(d.nx - 2);
    return dl + (double)(a - d.nx + 1) * (dl - d2);
  }
  return col(a);
}

// Each scheme's central operator delta^{c,(1)} (Eqs. 3.7, 3.9, 3.19, 3.21 and
// the Appendix) with the midpoint values replaced by the scheme's linear
// midpoint interpolation -- six points for the third- and fifth-order
// schemes, (3 g_{i-2} - 25 g_{i-1} + 150 g_i + 150 g_{i+1} - 25 g_{i+2} +
// 3 g_{i+3}) / 256, eight for the seventh-order ones, (-5 g_{i-3} + 49 g_{i-2}
// - 245 g_{i-1} + 1225 g_i + 1225 g_{i+1} - 245 g_{i+2} + 49 g_{i+3} -
// 5 g_{i+4}) / 2048 -- is an antisymmetric node stencil
// sum_m d_m (g_{i+m} - g_{i-m}), m = 1..7 (exact rationals):
const double kMetricStencil[8][METRIC_REACH] = {
    {557.0 / 768.0, -25.0 / 192.0, 3.0 / 256.0, 0.0, 0.0, 0.0, 0.0},                   // 3-1MP
    {1145.0 / 1536.0, -229.0 / 1536.0, 29.0 / 1536.0, -1.0 / 1024.0, 0.0, 0.0, 0.0},    // 3-2MP
    {3.0 / 4.0, -3.0 / 20.0, 1.0 / 60.0, 0.0, 0.0, 0.0, 0.0},                          // 5-1MP
    {487.0 / 640.0, -103.0 / 640.0, 41.0 / 1920.0, -1.0 / 1280.0, 0.0, 0.0, 0.0},      // 5-2MP
    {4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0, 0.0, 0.0, 0.0},                 // 7-1MP
    {773.0 / 960.0, -173.0 / 840.0, 557.0 / 13440.0, -23.0 / 5040.0, 1.0 / 8064.0, 0.0, 0.0},  // 7-2MP
    {114831.0 / 143360.0, -115271.0 / 573440.0, 4733.0 / 122880.0, -221.0 / 61440.0, -31.0 / 860160.0,
     1.0 / 114688.0, 0.0},                                                              // 7-4MP
    {5983587.0 / 7340032.0, -57115.0 / 262144.0, 153455.0 / 3145728.0, -1411.0 / 196608.0,
     10039.0 / 15728640.0, -89.0 / 1835008.0, 15.0 / 7340032.0},                        // 7-6MP
};

// The stencil for a scheme and free parameter a of the one-midpoint forms.
// Eq. 2.7 applied to Eq. 3.5 gives, with the six-point interpolation,
//   d = (2/3 + 15a/256, -1/12 - 3a/64, 3a/256)      (3-1MP; a = 1: the table row).
// For 5-1MP and 7-1MP the alpha term of h+ is a (F - P f), P the one-sided
// five- (seven-) point interpolation, whose mirror average is the six-
// (eight-) point central interpolation used here, so their operator does not
// depend on a.
MetricStencil metric_stencil(int scheme, double a) {
  MetricStencil s;
  for (int m = 0; m < METRIC_REACH; ++m) s.d[m] = kMetricStencil[scheme][m];
  if (scheme == 0 && a != 1.0) {
    s.d[0] = 2.0 / 3.0 + 15.0 * a / 256.0;
    s.d[1] = -1.0 / 12.0 - 3.0 * a / 64.0;
    s.d[2] = 3.0 * a / 256.0;
  }
  return s;
}

// Nodal-metric band beyond the stored ghost band: the reach of the midpoint
// interpolation (3 for six points, 4 for eight).
int metric_band(int scheme) { return GHOST + (scheme >= 4 ? 4 : 3); }

// Nodal metrics on the band of width B around the grid: T[5][(ny+2B)(nx+2B)].
// Periodic directions evaluate at the wrapped node so that band copies are
// bitwise equal to the interior values.
__global__ void metrics_nodal_kernel(Dims d, MetricStencil ms, int B, const double* __restrict__ x,
                                     const double* __restrict__ y, double* __restrict__ T) {
  const int W = d.nx + 2 * B, Hh = d.ny + 2 * B;
  const int ta = blockIdx.x * blockDim.x + threadIdx.x;
  const int tb = blockIdx.y * blockDim.y + threadIdx.y;
  if (ta >= W || tb >= Hh) return;
  int a = ta - B, b = tb - B;
  if (d.bcx == 0) a = bc_index(a, d.nx, 0);
  if (d.bcy == 0) b = bc_index(b, d.ny, 0);
  double x_xi = 0.0, y_xi = 0.0, x_eta = 0.0, y_eta = 0.0;
#pragma unroll
  for (int m = 1; m <= METRIC_REACH; ++m) {
    const double cm = ms.d[m - 1];
    if (cm == 0.0) continue;
    x_xi += cm * diff_i(d, x, true, b, a + m, a - m);
    y_xi += cm * diff_i(d, y, false, b, a + m, a - m);
    x_eta += cm * diff_j(d, x, false, a, b + m, b - m);
    y_eta += cm * diff_j(d, y, true, a, b + m, b - m);
  }
  const long long P = (long long)W * Hh, o = (long long)tb * W + ta;
  // Sec. 2.2 in two dimensions
  T[0 * P + o] = y_eta;                          // xi_x^
  T[1 * P + o] = -x_eta;                         // xi_y^
  T[2 * P + o] = -y_xi;                          // eta_x^
  T[3 * P + o] = x_xi;                           // eta_y^
  T[4 * P + o] = x_xi * y_eta - x_eta * y_xi;    // J^{-1}
}

// Nodal and midpoint metrics on the stored band (width GHOST) plus the tag.
__global__ void metrics_band_kernel(Dims d, int scheme, double ah, int B, const double* __restrict__ T,
                                    double* __restrict__ M, int* __restrict__ status) {
  const int W = d.nx + 2 * GHOST, Hh = d.ny + 2 * GHOST;
  const int ta = blockIdx.x * blockDim.x + threadIdx.x;
  const int tb = blockIdx.y * blockDim.y + threadIdx.y;
  if (ta == 0 && tb == 0) {
    double* tag = M + 9 * d.mplane;
    tag[0] = TAG_MAGIC; tag[1] = (double)scheme; tag[2] = (double)d.nx; tag[3] = (double)d.ny;
    tag[4] = (double)d.bcx; tag[5] = (double)d.bcy; tag[6] = ah; tag[7] = 0.0;
  }
  if (ta >= W || tb >= Hh) return;
  const int a = ta - GHOST, b = tb - GHOST;
  const int TW = d.nx + 2 * B;
  const long long TP = (long long)TW * (d.ny + 2 * B);
  auto t = [&](int p, int aa, int bb) { return T[p * TP + (long long)(bb + B) * TW + (aa + B)]; };
  const long long o = (long long)tb * W + ta;
  const long long P = d.mplane;
#pragma unroll
  for (int p = 0; p < 5; ++p) M[p * P + o] = t(p, a, b);
  // midpoint metrics: the same interpolation in the metric's own direction
  const bool eight = scheme >= 4;
  auto I = [&](int p, int di, int dj) {
    auto v = [&](int l) { return t(p, a + l * di, b + l * dj); };
    if (eight)
      return (-5.0 * (v(-3) + v(4)) + 49.0 * (v(-2) + v(3)) - 245.0 * (v(-1) + v(2)) + 1225.0 * (v(0) + v(1))) *
             (1.0 / 2048.0);
    return (3.0 * v(-2) - 25.0 * v(-1) + 150.0 * v(0) + 150.0 * v(1) - 25.0 * v(2) + 3.0 * v(3)) * (1.0 / 256.0);
  };
  M[5 * P + o] = I(0, 1, 0);
  M[6 * P + o] = I(1, 1, 0);
  M[7 * P + o] = I(2, 0, 1);
  M[8 * P + o] = I(3, 0, 1);
  if (a >= 0 && a < d.nx && b >= 0 && b < d.ny) {
    const double j = t(4, a, b);
    if (!(j > 0.0) || !(j < 1.0e300)) atomicOr(status, ST_JACOBIAN);
  }
}

// ===========================================================================
// Wave-speed maxima (Sec. 2.3): lam_xi[j] = max_i (|U^| + c|xi^|) over row j,
// lam_eta[i] over column i, and the CFL maximum of the sum over J^{-1}.
// Values are non-negative, so the order of their IEEE bit patterns as
// unsigned integers is their numeric order and an integer atomic max gives an
// order-independent (deterministic) result.  Non-physical or non-finite
// states latch ST_NONPHYS.
// ===========================================================================
__global__ void __launch_bounds__(256) wave_max_kernel(Dims d, const double* __restrict__ U,
                                                       const double* __restrict__ M, double gam,
                                                       unsigned long long* __restrict__ lam_xi,
                                                       unsigned long long* __restrict__ lam_eta,
                                                       unsigned long long* __restrict__ cfl_max,
                                                       int* __restrict__ status) {
  __shared__ WaveLds lds;
  wave_max_tile(d, U, M, gam, lam_xi, lam_eta, cfl_max, status, blockIdx.x, blockIdx.y, lds);
}

__global__ void fill_u64_kernel(unsigned long long* p, long long n, unsigned long long v) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

__global__ void cfl_dt_kernel(const unsigned long long* cfl_max, double cfl, double* dt) {
  if (threadIdx.x == 0 && blockIdx.x == 0) dt[0] = cfl / __longlong_as_double((long long)cfl_max[0]);
}

__global__ void lambda_out_kernel(Dims d, double alpha, const unsigned long long* lx, const unsigned long long* le,
                                  double* out_x, double* out_e) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < d.ny) out_x[t] = alpha * __longlong_as_double((long long)lx[t]);
  if (t < d.nx) out_e[t] = alpha * __longlong_as_double((long long)le[t]);
}

// ===========================================================================
// Direction sweep.  One block covers NB grid lines of one direction and a
// segment of OUT = NA - EXTRA output nodes along them.  Each thread owns one
// item k along its line: the split fluxes f^+-_k at node k and the midpoint
// fluxes F^+-_{k+1/2}; the items go to LDS, then the first OUT threads of
// each line form H_{i+1/2} - H_{i-1/2} for their output node.
//   DIR 0 (xi):  threadIdx.x runs along i, threadIdx.y across rows j.
//   DIR 1 (eta): threadIdx.x runs across columns i, threadIdx.y along j.
// Epilogue (SweepArgs::mode): rhs -- the xi sweep writes R^xi, the eta sweep
// dU/dt = -(R^xi + R^eta)/J^{-1}; RK stage -- the xi sweep writes its part of
// the update, P = a U0 + b (Us - dt R^xi/J^{-1}), the eta sweep completes it,
// U_out = P - b dt R^eta/J^{-1}, so U0 is read by the lighter xi epilogue.
// Launched for 4 waves per SIMD (at most 128 VGPRs).
// ===========================================================================
template <int SC, int DIR, int NA, int NB, bool OPT>
__global__ void __launch_bounds__(NA * NB, (sweep_waves<SC, OPT>())) sweep_kernel(SweepArgs s) {
  __shared__ SweepLds<SC, DIR, NA, NB, OPT> lds;
  // logical tile in XCD-aware order
  const int total = gridDim.x * gridDim.y;
  const int lid = xcd_remap(blockIdx.x + gridDim.x * blockIdx.y, total);
  sweep_tile<SC, DIR, NA, NB, OPT>(s, lid % gridDim.x, lid / gridDim.x, lds);
}

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------
template <int SC, int DIR, int NA, int NB, bool OPT>
hipError_t launch_sweep_t(const SweepArgs& a, hipStream_t st) {
  constexpr int OUT = NA - Range<SC>::EXTRA;
  const int n_al = DIR == 0 ? a.d.nx : a.d.ny;
  const int n_ac = DIR == 0 ? a.d.ny : a.d.nx;
  const int nseg = (n_al + OUT - 1) / OUT;
  const int nlin = (n_ac + NB - 1) / NB;
  dim3 grid = DIR == 0 ? dim3(nseg, nlin) : dim3(nlin, nseg);
  dim3 block = DIR == 0 ? dim3(NA, NB) : dim3(NB, NA);
  hipLaunchKernelGGL((sweep_kernel<SC, DIR, NA, NB, OPT>), grid, block, 0, st, a);
  return hipGetLastError();
}

// Tile shape `variant` of each direction (WIU_XI_TILES / WIU_ETA_TILES).
template <int SC, int DIR, bool OPT>
hipError_t launch_sweep_vo(int variant, const SweepArgs& a, hipStream_t st) {
#define WIU_CASE(v, na, nb) \
  case v: return launch_sweep_t<SC, DIR, na, nb, OPT>(a, st);
  if constexpr (DIR == 0) {
    switch (variant) {
      WIU_XI_TILES(WIU_CASE)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (variant) {
      WIU_ETA_TILES(WIU_CASE)
      default: return hipErrorInvalidValue;
    }
  }
#undef WIU_CASE
}

// the options kernels only when an option is in use
template <int SC, int DIR>
hipError_t launch_sweep_v(int variant, const SweepArgs& a, hipStream_t st) {
  if (a.vars != 0 || a.ah != 1.0 || a.weights != 0 || a.split != 0) return launch_sweep_vo<SC, DIR, true>(variant, a, st);
  return launch_sweep_vo<SC, DIR, false>(variant, a, st);
}

int sweep_variants(int dir) { return dir == 0 ? WIU_N_XI_TILES : WIU_N_ETA_TILES; }

hipError_t launch_sweep(int scheme, int dir, int variant, const SweepArgs& a, hipStream_t st) {
  switch (scheme * 2 + dir) {
    case 0: return launch_sweep_v<0, 0>(variant, a, st);
    case 1: return launch_sweep_v<0, 1>(variant, a, st);
    case 2: return launch_sweep_v<1, 0>(variant, a, st);
    case 3: return launch_sweep_v<1, 1>(variant, a, st);
    case 4: return launch_sweep_v<2, 0>(variant, a, st);
    case 5: return launch_sweep_v<2, 1>(variant, a, st);
    case 6: return launch_sweep_v<3, 0>(variant, a, st);
    case 7: return launch_sweep_v<3, 1>(variant, a, st);
    case 8: return launch_sweep_v<4, 0>(variant, a, st);
    case 9: return launch_sweep_v<4, 1>(variant, a, st);
    case 10: return launch_sweep_v<5, 0>(variant, a, st);
    case 11: return launch_sweep_v<5, 1>(variant, a, st);
    case 12: return launch_sweep_v<6, 0>(variant, a, st);
    case 13: return launch_sweep_v<6, 1>(variant, a, st);
    case 14: return launch_sweep_v<7, 0>(variant, a, st);
    case 15: return launch_sweep_v<7, 1>(variant, a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_wave_max(const Dims& d, const double* U, const double* M, double gam, unsigned long long* lx,
                           unsigned long long* le, unsigned long long* cfl, int* status, hipStream_t st) {
  // clear the maxima (a fill kernel, not a memset, so the sequence can be captured)
  const long long n = (long long)d.nx + d.ny + 1;
  // lx, le and cfl are contiguous in the workspace: lx[ny], le[nx], cfl[1]
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, lx, n, 0ull);
  dim3 grid((d.nx + 63) / 64, (d.ny + 15) / 16);
  hipLaunchKernelGGL(wave_max_kernel, grid, dim3(64, 4), 0, st, d, U, M, gam, lx, le, cfl, status);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, long long n, hipStream_t st) {
  hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, 0ull);
  return hipGetLastError();
}

hipError_t launch_metrics(const Dims& d, int scheme, double ah, const double* x, const double* y, double* M,
                          double* T, int* status, hipStream_t st) {
  const int B = metric_band(scheme);
  dim3 b1(64, 4);
  dim3 g1((d.nx + 2 * B + 63) / 64, (d.ny + 2 * B + 3) / 4);
  hipLaunchKernelGGL(metrics_nodal_kernel, g1, b1, 0, st, d, metric_stencil(scheme, ah), B, x, y, T);
  dim3 g2((d.nx + 2 * GHOST + 63) / 64, (d.ny + 2 * GHOST + 3) / 4);
  hipLaunchKernelGGL(metrics_band_kernel, g2, b1, 0, st, d, scheme, ah, B, T, M, status);
  return hipGetLastError();
}

hipError_t launch_metrics_band(const Dims& d, int scheme, double ah, int B, const double* T, double* M, int* status,
                               hipStream_t st) {
  dim3 b1(64, 4);
  dim3 g2((d.nx + 2 * GHOST + 63) / 64, (d.ny + 2 * GHOST + 3) / 4);
  hipLaunchKernelGGL(metrics_band_kernel, g2, b1, 0, st, d, scheme, ah, B, T, M, status);
  return hipGetLastError();
}

// One block: the maximum of n per-line CFL maxima (non-negative, so their
// bit patterns order as the values), then dt = cfl / max.
__global__ void __launch_bounds__(256) cfl_dt_lines_kernel(const unsigned long long* cfl_lines, int n, double cfl,
                                                            double* dt) {
  __shared__ unsigned long long part[4];
  unsigned long long m = 0;
  for (int k = threadIdx.x; k < n; k += 256) m = max(m, cfl_lines[k]);
  for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned long long)__shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) m = max(m, part[w]);
    m = max(m, part[0]);
    dt[0] = cfl / __longlong_as_double((long long)m);
  }
}

hipError_t launch_cfl_dt_lines(const unsigned long long* cfl_lines, int n, double cfl, double* dt, hipStream_t st) {
  hipLaunchKernelGGL(cfl_dt_lines_kernel, dim3(1), dim3(256), 0, st, cfl_lines, n, cfl, dt);
  return hipGetLastError();
}

hipError_t launch_cfl_dt(const unsigned long long* cfl_max, double cfl, double* dt, hipStream_t st) {
  hipLaunchKernelGGL(cfl_dt_kernel, dim3(1), dim3(64), 0, st, cfl_max, cfl, dt);
  return hipGetLastError();
}

hipError_t launch_lambda_out(const Dims& d, double alpha, const unsigned long long* lx, const unsigned long long* le,
                             double* ox, double* oe, hipStream_t st) {
  int n = d.nx > d.ny ? d.nx : d.ny;
  hipLaunchKernelGGL(lambda_out_kernel, dim3((n + 255) / 256), dim3(256), 0, st, d, alpha, lx, le, ox, oe);
  return hipGetLastError();
}

__global__ void set_tag_kernel(Dims d, int scheme, double ah, double* M) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double* tag = M + 9 * d.mplane;
    tag[0] = TAG_MAGIC; tag[1] = (double)scheme; tag[2] = (double)d.nx; tag[3] = (double)d.ny;
    tag[4] = (double)d.bcx; tag[5] = (double)d.bcy; tag[6] = ah; tag[7] = 0.0;
  }
}

hipError_t launch_set_tag(const Dims& d, int scheme, double ah, double* M, hipStream_t st) {
  hipLaunchKernelGGL(set_tag_kernel, dim3(1), dim3(64), 0, st, d, scheme, ah, M);
  return hipGetLastError();
}

__global__ void zero_int_kernel(int* p, int n) {
  int t = threadIdx.x;
  if (t < n) p[t] = 0;
}

hipError_t launch_zero_header(int* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(64), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace wiu
