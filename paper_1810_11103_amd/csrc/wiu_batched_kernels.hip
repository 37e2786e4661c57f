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

WIU_DEV const double* stage_src(const BlockDev& B, int stage) {
  return stage == 0 ? B.U : (stage == 1 ? B.U1 : B.U2);
}

template <int SC, int DIR, int NA, int NB>
__global__ void __launch_bounds__(NA * NB, 4) batched_sweep_kernel(BatchArgs b) {
  __shared__ SweepLds<SC, DIR, NA, NB> lds;
  {
    const int4 tl = b.tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const BlockDev& B = b.blocks[tl.x];
    SweepArgs s;
    // stage 2 reads the maxima its predecessor accumulated in lam2; the eta
    // sweeps of stages 1 and 2 accumulate those of the state they write
    const unsigned long long* lam = b.stage == 1 ? B.lam2 : B.lam;
    s.d = B.d; s.M = B.M; s.lam_xi = lam; s.lam_eta = lam + B.d.ny;
    unsigned long long* nlam = (DIR == 1 && b.stage < 2) ? (b.stage == 0 ? B.lam2 : B.lam) : nullptr;
    s.nlam_xi = nlam; s.nlam_eta = nlam ? nlam + B.d.ny : nullptr;
    s.gamma = b.gamma; s.alpha = b.alpha; s.eps = b.eps; s.ppm = b.ppm;
    s.Rxi = B.Rxi; s.U0 = B.U; s.dt = B.dt; s.status = b.status;
    s.U = stage_src(B, b.stage);
    s.out = b.stage == 0 ? B.U1 : (b.stage == 1 ? B.U2 : B.U);
    s.ca = b.stage == 0 ? 0.0 : (b.stage == 1 ? 0.75 : 1.0 / 3.0);
    s.cb = b.stage == 0 ? 1.0 : (b.stage == 1 ? 0.25 : 2.0 / 3.0);
    s.mode = DIR == 0 ? 3 : 2;
    sweep_tile<SC, DIR, NA, NB>(s, tl.y, tl.z, lds);
  }
}

__global__ void __launch_bounds__(256) batched_wave_max_kernel(BatchArgs b) {
  __shared__ WaveLds lds;
  {
    const int4 tl = b.tiles[xcd_remap(blockIdx.x, gridDim.x)];
    const BlockDev& B = b.blocks[tl.x];
    wave_max_tile(B.d, stage_src(B, b.stage), B.M, b.gamma, B.lam, B.lam + B.d.ny, B.lam + B.d.ny + B.d.nx,
                  b.status, tl.y, tl.z, lds);
  }
}

__global__ void batched_cfl_dt_kernel(const BlockDev* blocks, int nblocks, double cfl) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nblocks) {
    const BlockDev& B = blocks[t];
    B.dt[0] = cfl / __longlong_as_double((long long)B.lam[B.d.ny + B.d.nx]);
  }
}

template <int SC, int DIR, int NA, int NB>
hipError_t launch_batched_sweep_t(const BatchArgs& a, hipStream_t st) {
  const int grid = a.ntiles;
  dim3 block = DIR == 0 ? dim3(NA, NB) : dim3(NB, NA);
  hipLaunchKernelGGL((batched_sweep_kernel<SC, DIR, NA, NB>), dim3(grid), block, 0, st, a);
  return hipGetLastError();
}

template <int SC, int DIR>
hipError_t launch_batched_sweep_v(int variant, const BatchArgs& a, hipStream_t st) {
#define WIU_CASE(v, na, nb) \
  case v: return launch_batched_sweep_t<SC, DIR, na, nb>(a, st);
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

hipError_t launch_batched_sweep(int scheme, int dir, int variant, const BatchArgs& a, hipStream_t st) {
  switch (scheme * 2 + dir) {
    case 0: return launch_batched_sweep_v<0, 0>(variant, a, st);
    case 1: return launch_batched_sweep_v<0, 1>(variant, a, st);
    case 2: return launch_batched_sweep_v<1, 0>(variant, a, st);
    case 3: return launch_batched_sweep_v<1, 1>(variant, a, st);
    case 4: return launch_batched_sweep_v<2, 0>(variant, a, st);
    case 5: return launch_batched_sweep_v<2, 1>(variant, a, st);
    case 6: return launch_batched_sweep_v<3, 0>(variant, a, st);
    default: return launch_batched_sweep_v<3, 1>(variant, a, st);
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
    default: return Range<3>::EXTRA;
  }
}

hipError_t launch_batched_wave_max(const BatchArgs& a, hipStream_t st) {
  const int grid = a.ntiles;
  hipLaunchKernelGGL(batched_wave_max_kernel, dim3(grid), dim3(64, 4), 0, st, a);
  return hipGetLastError();
}


hipError_t launch_batched_cfl_dt(const BlockDev* blocks, int nblocks, double cfl, hipStream_t st) {
  hipLaunchKernelGGL(batched_cfl_dt_kernel, dim3((nblocks + 63) / 64), dim3(64), 0, st, blocks, nblocks, cfl);
  return hipGetLastError();
}

}  // namespace wiu
