// Batched multi-block stepping: plan construction, graph capture and the
// C ABI entry points declared in include/wenoiu.h.
#include "wenoiu.h"
#include "wiu_kernels.hpp"
#include "wiu_mb.hpp"

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
  // groups of line maxima joined through interfaces (lines crossing blocks,
  // and the CFL maxima of blocks joined into one set): offsets into d_lam
  int* d_gstart = nullptr;
  int* d_gmem = nullptr;
  int ngroups = 0;
  // captured step
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Ghost layer m >= 1 on line l beyond interface side s of block b, as an
// element offset g0 + m gm + l gl in the neighbour's state planes (an affine
// map: the side frames are).  False if some layer 1 <= m < WIU_MB_REACH of
// some line would fall outside the neighbour.
bool ghost_map(const wiu_block* blocks, int b, int s, long long& g0, long long& gm, long long& gl) {
  const wiu_block& k = blocks[b];
  const wiu_block& h = blocks[k.nbr[s]];
  auto off = [&](int m, int l) {
    int a, c, a2, c2;
    if (s == 0) { a = -m; c = l; }
    else if (s == 1) { a = k.nx - 1 + m; c = l; }
    else if (s == 2) { a = l; c = -m; }
    else { a = l; c = k.ny - 1 + m; }
    mb_through(s, k.nx, k.ny, k.nbr_side[s], h.nx, h.ny, a, c, a2, c2);
    if (a2 < 0 || a2 >= h.nx || c2 < 0 || c2 >= h.ny) return -1LL;
    return (long long)c2 * h.nx + a2;
  };
  const int n = mb_side_len(s, k.nx, k.ny), mmax = WIU_MB_REACH - 1;
  gm = off(2, 0) - off(1, 0);
  gl = n > 1 ? off(1, 1) - off(1, 0) : 0;
  g0 = off(1, 0) - gm;
  for (int m : {1, mmax})
    for (int l : {0, n - 1}) {
      const long long o = off(m, l);
      if (o < 0 || o != g0 + m * gm + l * gl) return false;
    }
  return true;
}

int uf_root(std::vector<int>& p, int v) {
  while (p[v] != v) { p[v] = p[p[v]]; v = p[v]; }
  return v;
}

// Groups of line maxima to be joined (only groups of two or more): the
// lines that continue through interfaces, and the CFL maxima of the blocks
// of each set joined by interfaces.  Uploaded to the plan.
bool line_groups(const wiu_block* blocks, int n, const std::vector<size_t>& off_lam, wiu_plan* p) {
  const int total = (int)(off_lam[n - 1] + blocks[n - 1].nx + blocks[n - 1].ny + 1);
  std::vector<int> par(total);
  for (int v = 0; v < total; ++v) par[v] = v;
  auto join = [&](int u, int v) {
    u = uf_root(par, u); v = uf_root(par, v);
    if (u != v) par[u] = v;
  };
  // line through node (a, c) normal to side s: xi line (row c) or eta line (column a)
  auto line_of = [&](int b, int s, int a, int c) { return (int)off_lam[b] + (s < 2 ? c : blocks[b].ny + a); };
  auto cfl_of = [&](int b) { return (int)off_lam[b] + blocks[b].ny + blocks[b].nx; };
  bool any = false;
  for (int b = 0; b < n; ++b)
    for (int s = 0; s < 4; ++s) {
      const wiu_block& k = blocks[b];
      if ((s < 2 ? k.bc_x : k.bc_y) == WIU_BC_PERIODIC || k.side[s] != WIU_SIDE_INTERFACE) continue;
      const wiu_block& h = blocks[k.nbr[s]];
      const int len = mb_side_len(s, k.nx, k.ny);
      for (int t = 0; t < len; ++t) {
        int a, c, a2, c2;
        mb_side_node(s, k.nx, k.ny, t, 0, a, c);
        mb_side_node(k.nbr_side[s], h.nx, h.ny, len - 1 - t, 0, a2, c2);
        join(line_of(b, s, a, c), line_of(k.nbr[s], k.nbr_side[s], a2, c2));
      }
      join(cfl_of(b), cfl_of(k.nbr[s]));
      any = true;
    }
  if (!any) return true;
  std::vector<std::vector<int>> members(total);
  for (int v = 0; v < total; ++v) members[uf_root(par, v)].push_back(v);
  std::vector<int> start{0}, mem;
  for (int v = 0; v < total; ++v)
    if (members[v].size() > 1) {
      mem.insert(mem.end(), members[v].begin(), members[v].end());
      start.push_back((int)mem.size());
    }
  p->ngroups = (int)start.size() - 1;
  if (p->ngroups == 0) return true;
  // one allocation: starts, then members
  const size_t bytes = sizeof(int) * (start.size() + mem.size());
  if (hipMalloc(&p->d_gstart, bytes) != hipSuccess) return false;
  p->d_gmem = p->d_gstart + start.size();
  return hipMemcpy(p->d_gstart, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(p->d_gmem, mem.data(), sizeof(int) * mem.size(), hipMemcpyHostToDevice) == hipSuccess;
}

void free_plan(wiu_plan* p) {
  if (!p) return;
  // teardown: nothing useful can be done with a failure here
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->d_blocks) (void)hipFree(p->d_blocks);
  if (p->d_tiles) (void)hipFree(p->d_tiles);
  if (p->d_ws) (void)hipFree(p->d_ws);
  if (p->d_gstart) (void)hipFree(p->d_gstart);
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
      if (launch_group_max(p->d_lam, p->d_gstart, p->d_gmem, p->ngroups, st) != hipSuccess) return WIU_EHIP;
    }
    a.tiles = p->d_tiles; a.ntiles = p->n_xi;
    if (launch_batched_sweep(p->scheme, 0, p->variant[0], a, st) != hipSuccess) return WIU_EHIP;
    if (stage < 2 && launch_fill_u64(stage == 0 ? p->d_lam2 : p->d_lam, p->lam_len, st) != hipSuccess)
      return WIU_EHIP;
    a.tiles = p->d_tiles + p->n_xi; a.ntiles = p->n_eta;
    if (launch_batched_sweep(p->scheme, 1, p->variant[1], a, st) != hipSuccess) return WIU_EHIP;
    if (stage < 2 &&
        launch_group_max(stage == 0 ? p->d_lam2 : p->d_lam, p->d_gstart, p->d_gmem, p->ngroups, st) != hipSuccess)
      return WIU_EHIP;
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
  if (!mb_blocks_ok(blocks, nblocks)) return WIU_EINVAL;

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
    B.d = mb_dims(blocks[b]);
    B.oU = blocks[b].off_U;
    B.oM = blocks[b].off_M;
    const size_t plane4 = align_up(4 * (size_t)blocks[b].nx * blocks[b].ny * 8);
    B.oRxi = (long long)(off_st[b] / 8);
    B.oU1 = (long long)((off_st[b] + plane4) / 8);
    B.oU2 = (long long)((off_st[b] + 2 * plane4) / 8);
    B.oDt = (long long)(dt_pos / 8) + b;
    B.oLam = (long long)off_lam[b];
    B.oLam2 = (long long)((lam2_pos - lam_pos) / 8 + off_lam[b]);
    for (int s = 0; s < 4; ++s) {
      const bool per = (s < 2 ? blocks[b].bc_x : blocks[b].bc_y) == WIU_BC_PERIODIC;
      B.side[s] = per ? WIU_SIDE_TRANSMISSIVE : blocks[b].side[s];
      B.nbr[s] = 0;
      B.g0[s] = B.gm[s] = B.gl[s] = 0;
      for (int c = 0; c < 4; ++c) B.fixed[s][c] = blocks[b].fixed[s][c];
      if (B.side[s] == WIU_SIDE_INTERFACE) {
        B.nbr[s] = blocks[b].nbr[s];
        if (!ghost_map(blocks, b, s, B.g0[s], B.gm[s], B.gl[s])) { free_plan(p); return WIU_EINVAL; }
      }
    }
  }
  if (!line_groups(blocks, nblocks, off_lam, p)) { free_plan(p); return WIU_EHIP; }
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
  if (launch_group_max(p->d_lam, p->d_gstart, p->d_gmem, p->ngroups, st) != hipSuccess) return WIU_EHIP;
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
        (void)hipGraphDestroy(g);
      }
    }
    if (hipStreamDestroy(cap) != hipSuccess) rc = WIU_EHIP;
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
  // work queued on the plan's buffers ends before they are freed; a failed
  // wait is reported, the plan is freed either way
  const bool ok = hipDeviceSynchronize() == hipSuccess;
  free_plan(p);
  return ok ? WIU_OK : WIU_EHIP;
}

}  // extern "C"
