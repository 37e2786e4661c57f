// Batched multi-block stepping: plan construction, graph capture and the
// C ABI entry points declared in include/wenoiu.h.
#include "wenoiu.h"
#include "wiu_kernels.hpp"

#include <new>
#include <vector>

using namespace wiu;

struct wiu_plan {
  int scheme = 0;
  int nblocks = 0;
  int variant[2] = {0, 0};
  wiu_params params{};
  long long cells = 0;
  // device memory owned by the plan
  BlockDev* d_blocks = nullptr;
  int4* d_tiles = nullptr;       // xi tiles, then eta tiles, then wave-max tiles
  int n_xi = 0, n_eta = 0, n_wm = 0;
  char* d_ws = nullptr;          // per-block lam, R^xi, U1, U2, dt; status
  unsigned long long* d_lam = nullptr;   // line maxima of all blocks (stages 1 and 3)
  unsigned long long* d_lam2 = nullptr;  // second set (stage 2), filled by stage 1's eta sweep
  long long lam_len = 0;
  double* d_dt = nullptr;
  double* U_all = nullptr;        // caller's states and metrics (offsets in the block table)
  const double* M_all = nullptr;
  int* d_status = nullptr;
  // captured step
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

bool block_ok(const wiu_block& b) {
  if (b.nx < 1 || b.ny < 1) return false;
  if (b.bc_x < 0 || b.bc_x > 1 || b.bc_y < 0 || b.bc_y > 1) return false;
  if (b.bc_x == WIU_BC_TRANSMISSIVE && b.nx < 2) return false;
  if (b.bc_y == WIU_BC_TRANSMISSIVE && b.ny < 2) return false;
  if (b.bc_x == WIU_BC_PERIODIC && !(b.period_x > 0.0)) return false;
  if (b.bc_y == WIU_BC_PERIODIC && !(b.period_y > 0.0)) return false;
  if (b.off_U < 0 || b.off_M < 0) return false;
  if (b.ny > 65535 * 4 || b.nx > (1 << 28)) return false;
  return true;
}

Dims dims_of(const wiu_block& b) {
  Dims d;
  d.nx = b.nx; d.ny = b.ny; d.bcx = b.bc_x; d.bcy = b.bc_y;
  d.mpitch = b.nx + 2 * GHOST;
  d.mplane = (long long)(b.nx + 2 * GHOST) * (b.ny + 2 * GHOST);
  d.np = (long long)b.nx * b.ny;
  d.Lx = b.period_x; d.Ly = b.period_y;
  return d;
}

void free_plan(wiu_plan* p) {
  if (!p) return;
  if (p->exec) hipGraphExecDestroy(p->exec);
  if (p->graph) hipGraphDestroy(p->graph);
  if (p->d_blocks) hipFree(p->d_blocks);
  if (p->d_tiles) hipFree(p->d_tiles);
  if (p->d_ws) hipFree(p->d_ws);
  delete p;
}

BatchArgs base_args(const wiu_plan* p) {
  BatchArgs a;
  a.blocks = p->d_blocks;
  a.tiles = p->d_tiles;
  a.ntiles = 0;
  a.stage = 0;
  a.gamma = p->params.gamma; a.alpha = p->params.alpha_lf; a.eps = p->params.eps; a.ppm = p->params.ppm;
  a.vars = p->params.vars; a.ah = p->params.alpha_h;
  a.weights = p->params.weights; a.split = p->params.split;
  for (int k = 0; k < 4; ++k) {  // blocks have periodic or transmissive sides
    a.side[k] = WIU_SIDE_TRANSMISSIVE;
    for (int c = 0; c < 4; ++c) a.fixed[k][c] = 0.0;
  }
  a.status = p->d_status;
  a.U_all = p->U_all;
  a.M_all = p->M_all;
  a.ws = (double*)p->d_ws;
  a.lam = p->d_lam;
  a.xi_mode = 3;
  return a;
}

int launch_step(wiu_plan* p, hipStream_t st) {
  BatchArgs a = base_args(p);
  // Line maxima: a separate pass for the step's state only; the eta sweeps
  // of stages 1 and 2 accumulate the maxima of the stage state they write
  // (into lam2, then back into lam), which the next stage reads.
  for (int stage = 0; stage < 3; ++stage) {
    a.stage = stage;
    if (stage == 0) {
      if (launch_fill_u64(p->d_lam, p->lam_len, st) != hipSuccess) return WIU_EHIP;
      a.tiles = p->d_tiles + p->n_xi + p->n_eta; a.ntiles = p->n_wm;
      if (launch_batched_wave_max(a, st) != hipSuccess) return WIU_EHIP;
    }
    a.tiles = p->d_tiles; a.ntiles = p->n_xi;
    if (launch_batched_sweep(p->scheme, 0, p->variant[0], a, st) != hipSuccess) return WIU_EHIP;
    if (stage < 2 && launch_fill_u64(stage == 0 ? p->d_lam2 : p->d_lam, p->lam_len, st) != hipSuccess)
      return WIU_EHIP;
    a.tiles = p->d_tiles + p->n_xi; a.ntiles = p->n_eta;
    if (launch_batched_sweep(p->scheme, 1, p->variant[1], a, st) != hipSuccess) return WIU_EHIP;
  }
  return WIU_OK;
}

}  // namespace

extern "C" {

int wiu_batched_plan(const wiu_block* blocks, int nblocks, int scheme, const wiu_params* params, int xi_variant,
                     int eta_variant, double* U_all, const double* M_all, wiu_plan** out) {
  if (!out) return WIU_EINVAL;
  *out = nullptr;
  if (!blocks || nblocks < 1 || scheme < 0 || scheme > 7 || !params || !U_all || !M_all) return WIU_EINVAL;
  if (!(params->gamma > 1.0) || !(params->alpha_lf > 0.0) || !(params->eps >= 0.0)) return WIU_EINVAL;
  if (params->ppm != 0 && params->ppm != 1) return WIU_EINVAL;
  if (params->vars < WIU_VARS_CHARACTERISTIC || params->vars > WIU_VARS_PRIMITIVE) return WIU_EINVAL;
  if (params->weights < 0 || params->weights > 1 || params->split < 0 || params->split > 2) return WIU_EINVAL;
  if (!(params->alpha_h > 0.0) || !(params->alpha_h < 1.0e300)) return WIU_EINVAL;
  if (params->alpha_h != 1.0 && scheme != WIU_3_1MP && scheme != WIU_5_1MP && scheme != WIU_7_1MP) return WIU_EINVAL;
  if (xi_variant < 0 || xi_variant >= wiu_tuning_variants(0)) return WIU_EINVAL;
  if (eta_variant < 0 || eta_variant >= wiu_tuning_variants(1)) return WIU_EINVAL;
  for (int b = 0; b < nblocks; ++b)
    if (!block_ok(blocks[b])) return WIU_EINVAL;

  wiu_plan* p = new (std::nothrow) wiu_plan();
  if (!p) return WIU_EINVAL;
  p->scheme = scheme;
  p->nblocks = nblocks;
  p->variant[0] = xi_variant;
  p->variant[1] = eta_variant;
  p->params = *params;

  // workspace: [status | lam, lam2 of all blocks | dt of all blocks | per block R^xi, U1, U2]
  std::vector<size_t> off_lam(nblocks), off_st(nblocks);
  size_t lam_total = 0;
  for (int b = 0; b < nblocks; ++b) {
    off_lam[b] = lam_total;
    lam_total += (size_t)blocks[b].nx + blocks[b].ny + 1;
  }
  size_t pos = ALIGN;                                   // status
  const size_t lam_pos = pos;
  pos += align_up(lam_total * 8);
  const size_t lam2_pos = pos;
  pos += align_up(lam_total * 8);
  const size_t dt_pos = pos;
  pos += align_up((size_t)nblocks * 8);
  for (int b = 0; b < nblocks; ++b) {
    off_st[b] = pos;
    pos += 3 * align_up(4 * (size_t)blocks[b].nx * blocks[b].ny * 8);
    p->cells += (long long)blocks[b].nx * blocks[b].ny;
  }
  if (hipMalloc(&p->d_ws, pos) != hipSuccess) { free_plan(p); return WIU_EHIP; }
  if (hipMemset(p->d_ws, 0, ALIGN + 2 * align_up(lam_total * 8) + align_up((size_t)nblocks * 8)) != hipSuccess) {
    free_plan(p);
    return WIU_EHIP;
  }
  p->d_status = (int*)p->d_ws;
  p->d_lam = (unsigned long long*)(p->d_ws + lam_pos);
  p->d_lam2 = (unsigned long long*)(p->d_ws + lam2_pos);
  p->lam_len = (long long)lam_total;
  p->d_dt = (double*)(p->d_ws + dt_pos);

  p->U_all = U_all;
  p->M_all = M_all;

  // block table: element offsets into U_all, M_all, the workspace (as
  // doubles) and the maxima (as 64-bit words from d_lam)
  std::vector<BlockDev> hb(nblocks);
  for (int b = 0; b < nblocks; ++b) {
    BlockDev& B = hb[b];
    B.d = dims_of(blocks[b]);
    B.oU = blocks[b].off_U;
    B.oM = blocks[b].off_M;
    const size_t plane4 = align_up(4 * (size_t)blocks[b].nx * blocks[b].ny * 8);
    B.oRxi = (long long)(off_st[b] / 8);
    B.oU1 = (long long)((off_st[b] + plane4) / 8);
    B.oU2 = (long long)((off_st[b] + 2 * plane4) / 8);
    B.oDt = (long long)(dt_pos / 8) + b;
    B.oLam = (long long)off_lam[b];
    B.oLam2 = (long long)((lam2_pos - lam_pos) / 8 + off_lam[b]);
  }
  // tile tables, block by block (so each XCD's contiguous range stays local)
  std::vector<int4> tx, te, tw;
  const int extra = scheme_extra(scheme);
  int na, nb;
  sweep_tile_shape(0, xi_variant, na, nb);
  for (int b = 0; b < nblocks; ++b) {
    const int out = na - extra;
    const int nseg = (blocks[b].nx + out - 1) / out, nlin = (blocks[b].ny + nb - 1) / nb;
    for (int y = 0; y < nlin; ++y)
      for (int x = 0; x < nseg; ++x) tx.push_back(make_int4(b, x, y, 0));
  }
  sweep_tile_shape(1, eta_variant, na, nb);
  for (int b = 0; b < nblocks; ++b) {
    const int out = na - extra;
    const int nseg = (blocks[b].ny + out - 1) / out, nlin = (blocks[b].nx + nb - 1) / nb;
    for (int y = 0; y < nseg; ++y)
      for (int x = 0; x < nlin; ++x) te.push_back(make_int4(b, x, y, 0));
  }
  for (int b = 0; b < nblocks; ++b) {
    const int gx = (blocks[b].nx + 63) / 64, gy = (blocks[b].ny + 15) / 16;
    for (int y = 0; y < gy; ++y)
      for (int x = 0; x < gx; ++x) tw.push_back(make_int4(b, x, y, 0));
  }
  p->n_xi = (int)tx.size();
  p->n_eta = (int)te.size();
  p->n_wm = (int)tw.size();
  std::vector<int4> all;
  all.reserve(tx.size() + te.size() + tw.size());
  all.insert(all.end(), tx.begin(), tx.end());
  all.insert(all.end(), te.begin(), te.end());
  all.insert(all.end(), tw.begin(), tw.end());
  if (hipMalloc(&p->d_blocks, sizeof(BlockDev) * nblocks) != hipSuccess ||
      hipMalloc(&p->d_tiles, sizeof(int4) * all.size()) != hipSuccess ||
      hipMemcpy(p->d_blocks, hb.data(), sizeof(BlockDev) * nblocks, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(p->d_tiles, all.data(), sizeof(int4) * all.size(), hipMemcpyHostToDevice) != hipSuccess) {
    free_plan(p);
    return WIU_EHIP;
  }
  *out = p;
  return WIU_OK;
}

int wiu_batched_info(const wiu_plan* p, long long* cells, int* tiles_xi, int* tiles_eta) {
  if (!p) return WIU_EINVAL;
  if (cells) *cells = p->cells;
  if (tiles_xi) *tiles_xi = p->n_xi;
  if (tiles_eta) *tiles_eta = p->n_eta;
  return WIU_OK;
}

int wiu_batched_set_dt(wiu_plan* p, const double* dt_host, wiu_stream_t stream) {
  if (!p || !dt_host) return WIU_EINVAL;
  if (hipMemcpyAsync(p->d_dt, dt_host, sizeof(double) * p->nblocks, hipMemcpyHostToDevice, (hipStream_t)stream) !=
      hipSuccess)
    return WIU_EHIP;
  return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? WIU_OK : WIU_EHIP;
}

int wiu_batched_get_dt(const wiu_plan* p, double* dt_host, wiu_stream_t stream) {
  if (!p || !dt_host) return WIU_EINVAL;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return WIU_EHIP;
  return hipMemcpy(dt_host, p->d_dt, sizeof(double) * p->nblocks, hipMemcpyDeviceToHost) == hipSuccess ? WIU_OK
                                                                                                        : WIU_EHIP;
}

int wiu_batched_cfl_dt(wiu_plan* p, double cfl, wiu_stream_t stream) {
  if (!p || !(cfl > 0.0)) return WIU_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  BatchArgs a = base_args(p);
  a.tiles = p->d_tiles + p->n_xi + p->n_eta;
  a.ntiles = p->n_wm;
  if (launch_fill_u64(p->d_lam, p->lam_len, st) != hipSuccess) return WIU_EHIP;
  if (launch_batched_wave_max(a, st) != hipSuccess) return WIU_EHIP;
  return launch_batched_cfl_dt(a, p->nblocks, cfl, st) == hipSuccess ? WIU_OK : WIU_EHIP;
}

int wiu_batched_rk3_step(wiu_plan* p, int use_graph, wiu_stream_t stream) {
  if (!p) return WIU_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (!use_graph) return launch_step(p, st);
  if (!p->exec) {
    // capture the launches of one step on a private stream
    hipStream_t cap;
    if (hipStreamCreate(&cap) != hipSuccess) return WIU_EHIP;
    int rc = WIU_OK;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = WIU_EHIP;
    if (rc == WIU_OK) {
      rc = launch_step(p, cap);
      hipGraph_t g = nullptr;
      if (hipStreamEndCapture(cap, &g) != hipSuccess || !g) rc = WIU_EHIP;
      if (rc == WIU_OK) {
        p->graph = g;
        if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) rc = WIU_EHIP;
      } else if (g) {
        hipGraphDestroy(g);
      }
    }
    hipStreamDestroy(cap);
    if (rc != WIU_OK) return rc;
  }
  return hipGraphLaunch(p->exec, st) == hipSuccess ? WIU_OK : WIU_EHIP;
}

int wiu_batched_status(wiu_plan* p, wiu_stream_t stream, int* status, int clear) {
  if (!p || !status) return WIU_EINVAL;
  return wiu_status(p->d_ws, stream, status, clear);
}

int wiu_plan_destroy(wiu_plan* p) {
  if (!p) return WIU_EINVAL;
  hipDeviceSynchronize();
  free_plan(p);
  return WIU_OK;
}

}  // extern "C"
