// Batched multi-block kernels of libwenoiu (gfx950, fp64).
#include "wiu_kernels.hpp"
#include "wiu_sweep.hpp"

namespace wiu {

// ===========================================================================
// Batched multi-block stepping.  All blocks' tiles of one kind form one flat
// table (block by block); one launch per kernel kind per RK stage covers
// every block, one workgroup per table entry, in XCD-aware order so that
// each XCD works through one contiguous range of the table (tiles of the
// same block share that XCD's L2).  A persistent variant that walked the
// table with a fixed grid measured slower than letting the dispatcher
// place one workgroup per tile, so it was dropped.
// ===========================================================================

// The table entry of this workgroup, in scalar registers.
WIU_DEV int4 uniform_tile(const BatchArgs& b) {
  const int4 t = b.tiles[xcd_remap(blockIdx.x, gridDim.x)];
  return make_int4(ufirst(t.x), ufirst(t.y), ufirst(t.z), 0);
}

// RK stage st (0, 1, 2) of a block reads src and writes dst:
//   U -> U1, U1 -> U2, U2 -> U.
WIU_DEV double* stage_src(const BatchArgs& b, const BlockDev& B, int st) {
  return st == 0 ? b.U_all + ufirst(B.oU) : b.ws + ufirst(st == 1 ? B.oU1 : B.oU2);
}
WIU_DEV double* stage_dst(const BatchArgs& b, const BlockDev& B, int st) {
  return st == 2 ? b.U_all + ufirst(B.oU) : b.ws + ufirst(st == 0 ? B.oU1 : B.oU2);
}

template <int SC, int DIR, int NA, int NB, bool OPT>
__global__ void __launch_bounds__(NA * NB, (sweep_waves<SC, OPT>())) batched_sweep_kernel(BatchArgs b) {
  __shared__ SweepLds<SC, DIR, NA, NB, OPT> lds;
  {
    const int4 tl = uniform_tile(b);
    const BlockDev& B = b.blocks[tl.x];
    const int st = b.stage;
    SweepArgs s;
    s.d = ufirst(B.d);
    s.M = b.M_all + ufirst(B.oM);
    // stage 1 reads the maxima of the separate pass (lam) and accumulates
    // those of U1 into lam2; stage 2 reads lam2 and accumulates into lam;
    // stage 3 reads lam
    const unsigned long long* lam = b.lam + ufirst(st == 1 ? B.oLam2 : B.oLam);
    s.lam_xi = lam; s.lam_eta = lam + s.d.ny;
    unsigned long long* nlam = (DIR == 1 && st < 2) ? b.lam + ufirst(st == 0 ? B.oLam2 : B.oLam) : nullptr;
    s.nlam_xi = nlam; s.nlam_eta = nlam ? nlam + s.d.ny : nullptr;
    s.ncfl = nullptr;
    s.gamma = b.gamma; s.alpha = b.alpha; s.eps = b.eps; s.ppm = b.ppm; s.vars = b.vars; s.ah = b.ah;
    s.weights = b.weights; s.split = b.split;
    // the block's side rules; an interface reads the neighbour's state of
    // the same stage
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      s.side[k] = ufirst(B.side[k]);
#pragma unroll
      for (int c = 0; c < 4; ++c) s.fixed[k][c] = ufirst(B.fixed[k][c]);
    }
#pragma unroll
    for (int k = 2 * DIR; k < 2 * DIR + 2; ++k) {
      if (s.side[k] == WIU_SIDE_INTERFACE) {
        const BlockDev& N = b.blocks[ufirst(B.nbr[k])];
        s.nbU[k] = stage_src(b, N, st);
        s.nbnp[k] = ufirst(N.d.np);
        s.g0[k] = ufirst(B.g0[k]); s.gm[k] = ufirst(B.gm[k]); s.gl[k] = ufirst(B.gl[k]);
      }
    }
    s.Rxi = b.ws + ufirst(B.oRxi); s.U0 = b.U_all + ufirst(B.oU); s.dt = b.ws + ufirst(B.oDt);
    s.status = b.status;
    s.U = stage_src(b, B, st);
    s.out = stage_dst(b, B, st);
    s.ca = st == 0 ? 0.0 : (st == 1 ? 0.75 : 1.0 / 3.0);
    s.cb = st == 0 ? 1.0 : (st == 1 ? 0.25 : 2.0 / 3.0);
    s.mode = DIR == 0 ? b.xi_mode : 2;
    sweep_tile<SC, DIR, NA, NB, OPT>(s, tl.y, tl.z, lds);
  }
}

__global__ void __launch_bounds__(256) batched_wave_max_kernel(BatchArgs b) {
  __shared__ WaveLds lds;
  {
    const int4 tl = uniform_tile(b);
    const BlockDev& B = b.blocks[tl.x];
    const Dims d = ufirst(B.d);
    unsigned long long* lam = b.lam + ufirst(B.oLam);
    wave_max_tile(d, stage_src(b, B, b.stage), b.M_all + ufirst(B.oM), b.gamma, lam, lam + d.ny,
                  lam + d.ny + d.nx, b.status, tl.y, tl.z, lds);
  }
}

__global__ void batched_cfl_dt_kernel(BatchArgs b, int nblocks, double cfl) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nblocks) {
    const BlockDev& B = b.blocks[t];
    b.ws[B.oDt] = cfl / __longlong_as_double((long long)b.lam[B.oLam + B.d.ny + B.d.nx]);
  }
}

template <int SC, int DIR, int NA, int NB, bool OPT>
hipError_t launch_batched_sweep_t(const BatchArgs& a, hipStream_t st) {
  const int grid = a.ntiles;
  dim3 block = DIR == 0 ? dim3(NA, NB) : dim3(NB, NA);
  hipLaunchKernelGGL((batched_sweep_kernel<SC, DIR, NA, NB, OPT>), dim3(grid), block, 0, st, a);
  return hipGetLastError();
}

template <int SC, int DIR, bool OPT>
hipError_t launch_batched_sweep_vo(int variant, const BatchArgs& a, hipStream_t st) {
#define WIU_CASE(v, na, nb) \
  case v: return launch_batched_sweep_t<SC, DIR, na, nb, OPT>(a, st);
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
hipError_t launch_batched_sweep_v(int variant, const BatchArgs& a, hipStream_t st) {
  if (a.vars != 0 || a.ah != 1.0 || a.weights != 0 || a.split != 0)
    return launch_batched_sweep_vo<SC, DIR, true>(variant, a, st);
  return launch_batched_sweep_vo<SC, DIR, false>(variant, a, st);
}

hipError_t launch_batched_sweep(int scheme, int dir, int variant, const BatchArgs& a, hipStream_t st) {
  switch (scheme * 2 + dir) {
    case 0: return launch_batched_sweep_v<0, 0>(variant, a, st);
    case 1: return launch_batched_sweep_v<0, 1>(variant, a, st);
    case 2: return launch_batched_sweep_v<1, 0>(variant, a, st);
    case 3: return launch_batched_sweep_v<1, 1>(variant, a, st);
    case 4: return launch_batched_sweep_v<2, 0>(variant, a, st);
    case 5: return launch_batched_sweep_v<2, 1>(variant, a, st);
    case 6: return launch_batched_sweep_v<3, 0>(variant, a, st);
    case 7: return launch_batched_sweep_v<3, 1>(variant, a, st);
    case 8: return launch_batched_sweep_v<4, 0>(variant, a, st);
    case 9: return launch_batched_sweep_v<4, 1>(variant, a, st);
    case 10: return launch_batched_sweep_v<5, 0>(variant, a, st);
    case 11: return launch_batched_sweep_v<5, 1>(variant, a, st);
    case 12: return launch_batched_sweep_v<6, 0>(variant, a, st);
    case 13: return launch_batched_sweep_v<6, 1>(variant, a, st);
    case 14: return launch_batched_sweep_v<7, 0>(variant, a, st);
    case 15: return launch_batched_sweep_v<7, 1>(variant, a, st);
    default: return hipErrorInvalidValue;
  }
}

void sweep_tile_shape(int dir, int variant, int& na, int& nb) {
  na = nb = 0;
#define WIU_SHAPE(v, a_, b_) \
  if (variant == v) { na = a_; nb = b_; }
  if (dir == 0) { WIU_XI_TILES(WIU_SHAPE) }
  else { WIU_ETA_TILES(WIU_SHAPE) }
#undef WIU_SHAPE
}

int scheme_extra(int scheme) {
  switch (scheme) {
    case 0: return Range<0>::EXTRA;
    case 1: return Range<1>::EXTRA;
    case 2: return Range<2>::EXTRA;
    case 3: return Range<3>::EXTRA;
    case 4: return Range<4>::EXTRA;
    case 5: return Range<5>::EXTRA;
    case 6: return Range<6>::EXTRA;
    case 7: return Range<7>::EXTRA;
    default: return -1;
  }
}

hipError_t launch_batched_wave_max(const BatchArgs& a, hipStream_t st) {
  const int grid = a.ntiles;
  hipLaunchKernelGGL(batched_wave_max_kernel, dim3(grid), dim3(64, 4), 0, st, a);
  return hipGetLastError();
}


hipError_t launch_batched_cfl_dt(const BatchArgs& a, int nblocks, double cfl, hipStream_t st) {
  hipLaunchKernelGGL(batched_cfl_dt_kernel, dim3((nblocks + 63) / 64), dim3(64), 0, st, a, nblocks, cfl);
  return hipGetLastError();
}

}  // namespace wiu
