"""Thin ctypes binding of libwenoiu (include/wenoiu.h).

Argument marshalling only: every step of the path runs in the HIP kernels of
libwenoiu.so.  Tensors are torch tensors on the ROCm device (fp64,
contiguous); the current torch stream is passed as the HIP stream.  There is
no CPU fallback: if the library is missing the import of this module fails.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwenoiu.so")

SCHEMES = {"3-1MP": 0, "3-2MP": 1, "5-1MP": 2, "5-2MP": 3, "7-1MP": 4, "7-2MP": 5, "7-4MP": 6, "7-6MP": 7}
BC = {"periodic": 0, "transmissive": 1}
GHOST = 4
ST_JACOBIAN, ST_NONPHYS, ST_SCHEME, ST_ARGMAX = 1, 2, 4, 8
WIU_OK, WIU_EINVAL, WIU_EHIP = 0, -1, -2

EXPORTS = [
    "wiu_metrics_size", "wiu_workspace_bytes", "wiu_workspace_init", "wiu_metrics", "wiu_set_metrics_tag",
    "wiu_line_eigenvalues", "wiu_rhs", "wiu_cfl_dt", "wiu_rk3_step", "wiu_status", "wiu_strerror",
    "wiu_profile_enable", "wiu_profile_read", "wiu_tuning_variants", "wiu_set_tuning", "wiu_get_tuning",
    "wiu_batched_plan", "wiu_batched_info", "wiu_batched_set_dt", "wiu_batched_cfl_dt", "wiu_batched_get_dt",
    "wiu_batched_rk3_step", "wiu_batched_status", "wiu_plan_destroy", "wiu_blocks_metrics_work_size",
    "wiu_blocks_metrics", "wiu3_metrics_size", "wiu3_workspace_bytes", "wiu3_metrics", "wiu3_rhs", "wiu3_cfl_dt",
    "wiu3_rk3_step", "wiu3_rk3_step_cfl", "wiu3_rk3_steps_cfl",
    "wiu_rhs_vjp", "wiu_rk3_step_stages", "wiu_rk3_step_vjp", "wiu_rk3_step_cfl", "wiu_rk3_steps_cfl", "wiu_rk3_steps_stages", "wiu_step_record_bytes",
    "wiu_noalloc_bytes", "wiu_rk3_step_noalloc",
]
KERNELS = {"wave_max": 0, "sweep_xi": 1, "sweep_eta": 2, "metrics": 3, "sweep3": 4}


class WiuGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int),
                ("period_x", ctypes.c_double), ("period_y", ctypes.c_double), ("side", ctypes.c_int * 4),
                ("fixed", (ctypes.c_double * 4) * 4)]


class WiuBlock(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int),
                ("period_x", ctypes.c_double), ("period_y", ctypes.c_double),
                ("off_U", ctypes.c_longlong), ("off_M", ctypes.c_longlong),
                ("side", ctypes.c_int * 4), ("nbr", ctypes.c_int * 4), ("nbr_side", ctypes.c_int * 4),
                ("shift", (ctypes.c_double * 2) * 4), ("fixed", (ctypes.c_double * 4) * 4),
                ("off_X", ctypes.c_longlong)]


class WiuGrid3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("bc", ctypes.c_int * 3),
                ("period", ctypes.c_double * 3), ("side", ctypes.c_int * 6), ("fixed", (ctypes.c_double * 5) * 6)]


class WiuParams(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("alpha_lf", ctypes.c_double), ("eps", ctypes.c_double),
                ("ppm", ctypes.c_int), ("vars", ctypes.c_int), ("alpha_h", ctypes.c_double),
                ("weights", ctypes.c_int), ("split", ctypes.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libwenoiu.so not built ({LIB_PATH}); run paper_1810_11103_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    G = ctypes.POINTER(WiuGrid)
    PR = ctypes.POINTER(WiuParams)
    I = ctypes.c_int
    sig = {
        "wiu_metrics_size": (ctypes.c_size_t, [G]),
        "wiu_workspace_bytes": (ctypes.c_size_t, [G]),
        "wiu_workspace_init": (I, [P, P]),
        "wiu_metrics": (I, [G, I, PR, P, P, P, P, P]),
        "wiu_set_metrics_tag": (I, [G, I, PR, P, P]),
        "wiu_line_eigenvalues": (I, [G, PR, P, P, P, P, P, P]),
        "wiu_rhs": (I, [G, I, PR, P, P, P, P, P]),
        "wiu_cfl_dt": (I, [G, PR, P, P, ctypes.c_double, P, P, P]),
        "wiu_rk3_step": (I, [G, I, PR, P, P, P, P, P]),
        "wiu_rk3_step_cfl": (I, [G, I, PR, P, P, ctypes.c_double, P, P, P]),
        "wiu_rk3_steps_cfl": (I, [G, I, PR, P, P, ctypes.c_double, I, P, P, P]),
        "wiu_noalloc_bytes": (ctypes.c_size_t, [G]),
        "wiu_rk3_step_noalloc": (I, [G, I, PR, P, P, P, P, P]),
        "wiu_status": (I, [P, P, ctypes.POINTER(I), I]),
        "wiu_strerror": (ctypes.c_char_p, [I]),
        "wiu_profile_enable": (I, [I]),
        "wiu_batched_plan": (I, [ctypes.POINTER(WiuBlock), I, I, PR, I, I, P, P, ctypes.POINTER(P)]),
        "wiu_blocks_metrics_work_size": (ctypes.c_size_t, [ctypes.POINTER(WiuBlock), I, I]),
        "wiu3_metrics_size": (ctypes.c_size_t, [ctypes.POINTER(WiuGrid3)]),
        "wiu3_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(WiuGrid3)]),
        "wiu3_metrics": (I, [ctypes.POINTER(WiuGrid3), I, I, PR, P, P, P, P, P, P]),
        "wiu3_rhs": (I, [ctypes.POINTER(WiuGrid3), I, PR, P, P, P, P, P]),
        "wiu3_cfl_dt": (I, [ctypes.POINTER(WiuGrid3), PR, P, P, ctypes.c_double, P, P, P]),
        "wiu3_rk3_step": (I, [ctypes.POINTER(WiuGrid3), I, PR, P, P, P, P, P]),
        "wiu3_rk3_step_cfl": (I, [ctypes.POINTER(WiuGrid3), I, PR, P, P, ctypes.c_double, P, P, P]),
        "wiu3_rk3_steps_cfl": (I, [ctypes.POINTER(WiuGrid3), I, PR, P, P, ctypes.c_double, I, P, P, P]),
        "wiu_blocks_metrics": (I, [ctypes.POINTER(WiuBlock), I, I, PR, P, P, P, P]),
        "wiu_batched_info": (I, [P, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(I), ctypes.POINTER(I)]),
        "wiu_batched_set_dt": (I, [P, P, P]),
        "wiu_batched_cfl_dt": (I, [P, ctypes.c_double, P]),
        "wiu_batched_get_dt": (I, [P, P, P]),
        "wiu_batched_rk3_step": (I, [P, I, P]),
        "wiu_batched_status": (I, [P, P, ctypes.POINTER(I), I]),
        "wiu_plan_destroy": (I, [P]),
        "wiu_rhs_vjp": (I, [G, I, PR, P, P, P, P, P, P]),
        "wiu_rk3_step_stages": (I, [G, I, PR, P, P, P, P, P, P, P, P]),
        "wiu_rk3_steps_stages": (I, [G, I, PR, P, P, P, I, P, P, P, P]),
        "wiu_rk3_step_vjp": (I, [G, I, PR, P, P, P, P, P, P, P, P, P, P]),
        "wiu_step_record_bytes": (ctypes.c_size_t, [G]),
        "wiu_tuning_variants": (I, [I]),
        "wiu_set_tuning": (I, [I, I]),
        "wiu_get_tuning": (I, [I]),
        "wiu_profile_read": (I, [I, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()


class WiuError(RuntimeError):
    pass


def _check(rc):
    if rc != WIU_OK:
        raise WiuError(f"libwenoiu: {lib.wiu_strerror(rc).decode()} ({rc})")


def scheme_id(s):
    return SCHEMES[s] if isinstance(s, str) else int(s)


SIDES = {"transmissive": 0, "wall": 1, "fixed": 2, "interface": 3}


def make_grid(nx, ny, bc=("periodic", "periodic"), period=(0.0, 0.0), sides=None, fixed=None):
    """Grid description; sides: rules of (x low, x high, y low, y high) of the
    non-periodic directions ("transmissive", "wall", "fixed"), fixed: their
    conservative states [4][4] for "fixed" sides."""
    bx = BC[bc[0]] if isinstance(bc[0], str) else int(bc[0])
    by = BC[bc[1]] if isinstance(bc[1], str) else int(bc[1])
    g = WiuGrid(int(nx), int(ny), bx, by, float(period[0]), float(period[1]))
    if sides is not None:
        for k, v in enumerate(sides):
            g.side[k] = SIDES[v] if isinstance(v, str) else int(v)
    if fixed is not None:
        for k in range(4):
            for q in range(4):
                g.fixed[k][q] = float(fixed[k][q])
    return g


VARS = {"characteristic": 0, "conservative": 1, "primitive": 2}


WEIGHTS = {"js": 0, "z": 1}
SPLITS = {"lf": 0, "sw": 1, "vl": 2}


def make_params(gamma=1.4, alpha_lf=1.1, eps=1e-40, ppm=1, vars="characteristic", alpha_h=1.0, weights="js",
                split="lf"):
    """Scheme parameters; vars: interpolation variables (Sec. 2.4), alpha_h:
    free parameter of the one-midpoint families (Eqs. 3.5, 3.17, Appendix),
    weights: "js" (Eqs. 3.12-3.13) or "z" (WENO-Z), split: splitting of the
    leading midpoint flux, "lf", "sw" (Steger-Warming) or "vl" (van Leer)."""
    v = VARS[vars] if isinstance(vars, str) else int(vars)
    w = WEIGHTS[weights] if isinstance(weights, str) else int(weights)
    sp = SPLITS[split] if isinstance(split, str) else int(split)
    return WiuParams(float(gamma), float(alpha_lf), float(eps), int(ppm), v, float(alpha_h), w, sp)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), "fp64 contiguous device tensor expected"
    return ctypes.c_void_p(t.data_ptr())


def metrics_size(grid):
    return lib.wiu_metrics_size(ctypes.byref(grid))


def workspace_bytes(grid):
    return lib.wiu_workspace_bytes(ctypes.byref(grid))


def workspace(grid, device="cuda"):
    """A zero-initialised workspace tensor for `grid` (uint8)."""
    n = workspace_bytes(grid)
    if n == 0:
        raise WiuError("invalid grid")
    ws = torch.zeros(n, dtype=torch.uint8, device=device)
    return ws


def metrics_tensor(grid, device="cuda"):
    n = metrics_size(grid)
    if n == 0:
        raise WiuError("invalid grid")
    return torch.empty(n // 8, dtype=torch.float64, device=device)


def metric_planes(M, grid):
    """View of the nine metric planes (9, ny + 2G, nx + 2G)."""
    H, W = grid.ny + 2 * GHOST, grid.nx + 2 * GHOST
    return M[: 9 * H * W].view(9, H, W)


def workspace_init(ws, stream=None):
    _check(lib.wiu_workspace_init(ctypes.c_void_p(ws.data_ptr()), _stream(stream)))


def _pref(params):
    return ctypes.byref(params) if params is not None else None


def metrics(grid, scheme, x, y, M, ws, stream=None, params=None):
    _check(lib.wiu_metrics(ctypes.byref(grid), scheme_id(scheme), _pref(params), _ptr(x), _ptr(y), _ptr(M),
                           ctypes.c_void_p(ws.data_ptr()), _stream(stream)))
    return M


def set_metrics_tag(grid, scheme, M, stream=None, params=None):
    _check(lib.wiu_set_metrics_tag(ctypes.byref(grid), scheme_id(scheme), _pref(params), _ptr(M),
                                   _stream(stream)))


def line_eigenvalues(grid, params, U, M, lam_xi, lam_eta, ws, stream=None):
    _check(lib.wiu_line_eigenvalues(ctypes.byref(grid), ctypes.byref(params), _ptr(U), _ptr(M), _ptr(lam_xi),
                                    _ptr(lam_eta), ctypes.c_void_p(ws.data_ptr()), _stream(stream)))


def rhs(grid, scheme, params, U, M, dUdt, ws, stream=None):
    _check(lib.wiu_rhs(ctypes.byref(grid), scheme_id(scheme), ctypes.byref(params), _ptr(U), _ptr(M), _ptr(dUdt),
                       ctypes.c_void_p(ws.data_ptr()), _stream(stream)))
    return dUdt


def cfl_dt(grid, params, U, M, cfl, dt_dev, ws, stream=None):
    _check(lib.wiu_cfl_dt(ctypes.byref(grid), ctypes.byref(params), _ptr(U), _ptr(M), float(cfl), _ptr(dt_dev),
                          ctypes.c_void_p(ws.data_ptr()), _stream(stream)))
    return dt_dev


def rk3_step(grid, scheme, params, U, M, dt_dev, ws, stream=None):
    _check(lib.wiu_rk3_step(ctypes.byref(grid), scheme_id(scheme), ctypes.byref(params), _ptr(U), _ptr(M),
                            _ptr(dt_dev), ctypes.c_void_p(ws.data_ptr()), _stream(stream)))
    return U


def rk3_step_cfl(grid, scheme, params, U, M, cfl, dt_dev, ws, stream=None):
    _check(lib.wiu_rk3_step_cfl(ctypes.byref(grid), scheme_id(scheme), ctypes.byref(params), _ptr(U), _ptr(M),
                                float(cfl), _ptr(dt_dev), ctypes.c_void_p(ws.data_ptr()), _stream(stream)))
    return U


def rk3_steps_cfl(grid, scheme, params, U, M, cfl, nsteps, dt_dev, ws, stream=None):
    """nsteps RK3 steps, each at the CFL time step of its state; dt_dev
    (float64, >= nsteps entries) receives the step sizes."""
    if dt_dev.numel() < nsteps or dt_dev.dtype != torch.float64 or not dt_dev.is_contiguous():
        raise ValueError("dt_dev: a contiguous float64 tensor of at least nsteps entries")
    _check(lib.wiu_rk3_steps_cfl(ctypes.byref(grid), scheme_id(scheme), ctypes.byref(params), _ptr(U), _ptr(M),
                                 float(cfl), int(nsteps), _ptr(dt_dev), ctypes.c_void_p(ws.data_ptr()),
                                 _stream(stream)))
    return U


def noalloc_bytes(grid):
    return lib.wiu_noalloc_bytes(ctypes.byref(grid))


def rk3_step_noalloc(grid, scheme, params, U, M, dt_dev, status_dev, stream=None):
    """wiu_rk3_step without a workspace: scratch in the library's static
    device array; device-side status bits are OR-ed into status_dev (int32)."""
    assert status_dev.is_cuda and status_dev.dtype == torch.int32, "int32 device tensor expected"
    _check(lib.wiu_rk3_step_noalloc(ctypes.byref(grid), scheme_id(scheme), ctypes.byref(params), _ptr(U), _ptr(M),
                                    _ptr(dt_dev), ctypes.c_void_p(status_dev.data_ptr()), _stream(stream)))
    return U


def rhs_vjp(grid, scheme, params, U, M, Gbar, Ubar, ws, stream=None):
    _check(lib.wiu_rhs_vjp(ctypes.byref(grid), scheme_id(scheme), ctypes.byref(params), _ptr(U), _ptr(M), _ptr(Gbar),
                           _ptr(Ubar), ctypes.c_void_p(ws.data_ptr()), _stream(stream)))
    return Ubar


def step_record_bytes(grid):
    return lib.wiu_step_record_bytes(ctypes.byref(grid))


def _rec(rec):
    if rec is None:
        return None
    assert rec.is_cuda and rec.is_contiguous() and rec.numel() * rec.element_size() >= 8
    return ctypes.c_void_p(rec.data_ptr())


def rk3_step_stages(grid, scheme, params, U, M, dt_dev, U1, U2, ws, rec=None, stream=None):
    _check(lib.wiu_rk3_step_stages(ctypes.byref(grid), scheme_id(scheme), ctypes.byref(params), _ptr(U), _ptr(M),
                                   _ptr(dt_dev), _ptr(U1), _ptr(U2), _rec(rec), ctypes.c_void_p(ws.data_ptr()),
                                   _stream(stream)))
    return U


def rk3_steps_stages(grid, scheme, params, U, M, dt_dev, stages, recs, ws, stream=None):
    """len(stages) steps of rk3_step_stages in one call: stages [n, 3, 4, ny, nx]
    (U_n, U1, U2 of each step), recs [n, record words] (step records)."""
    n = int(stages.shape[0])
    if (stages.dim() != 5 or tuple(stages.shape[1:]) != (3,) + tuple(U.shape) or stages.dtype != torch.float64
            or not stages.is_contiguous()):
        raise ValueError("stages: a contiguous float64 tensor [n, 3, 4, ny, nx]")
    if (recs.dim() != 2 or recs.shape[0] < n or recs.shape[1] * recs.element_size() < step_record_bytes(grid)
            or not recs.is_contiguous() or not recs.is_cuda):
        raise ValueError("recs: a contiguous device tensor of at least n step records")
    _check(lib.wiu_rk3_steps_stages(ctypes.byref(grid), scheme_id(scheme), ctypes.byref(params), _ptr(U), _ptr(M),
                                    _ptr(dt_dev), n, _ptr(stages), ctypes.c_void_p(recs.data_ptr()),
                                    ctypes.c_void_p(ws.data_ptr()), _stream(stream)))
    return U


def rk3_step_vjp(grid, scheme, params, U_n, U1, U2, M, dt_dev, Ubar_np1, Ubar_n, ws, rec=None, stream=None):
    _check(lib.wiu_rk3_step_vjp(ctypes.byref(grid), scheme_id(scheme), ctypes.byref(params), _ptr(U_n), _ptr(U1),
                                _ptr(U2), _rec(rec), _ptr(M), _ptr(dt_dev), _ptr(Ubar_np1), _ptr(Ubar_n),
                                ctypes.c_void_p(ws.data_ptr()), _stream(stream)))
    return Ubar_n


def status(ws, clear=True, stream=None):
    v = ctypes.c_int(0)
    _check(lib.wiu_status(ctypes.c_void_p(ws.data_ptr()), _stream(stream), ctypes.byref(v), int(clear)))
    return v.value


def tuning_variants(direction):
    return lib.wiu_tuning_variants(int(direction))


def set_tuning(direction, variant):
    _check(lib.wiu_set_tuning(int(direction), int(variant)))


def get_tuning(direction):
    return lib.wiu_get_tuning(int(direction))


def profile_enable(on=True):
    _check(lib.wiu_profile_enable(int(bool(on))))


def profile_read(kernel):
    """(launch count, mean duration in ms) of a library kernel since the last read."""
    n = ctypes.c_longlong(0)
    ms = ctypes.c_double(0.0)
    _check(lib.wiu_profile_read(KERNELS[kernel] if isinstance(kernel, str) else int(kernel), ctypes.byref(n),
                                ctypes.byref(ms)))
    return n.value, ms.value


class Solver:
    """Device-resident grid, metrics and workspace for one WENOIU problem."""

    def __init__(self, x, y, scheme="5-2MP", bc=("periodic", "periodic"), period=(0.0, 0.0), params=None,
                 device="cuda", sides=None, fixed=None):
        x = torch.as_tensor(x, dtype=torch.float64).to(device).contiguous()
        y = torch.as_tensor(y, dtype=torch.float64).to(device).contiguous()
        ny, nx = x.shape
        self.scheme = scheme
        self.grid = make_grid(nx, ny, bc, period, sides, fixed)
        self.params = params or make_params()
        self.device = device
        self.ws = workspace(self.grid, device)
        workspace_init(self.ws)
        self.M = metrics_tensor(self.grid, device)
        metrics(self.grid, scheme, x, y, self.M, self.ws, params=self.params)
        self.x, self.y = x, y
        self.dt = torch.zeros(1, dtype=torch.float64, device=device)

    def rhs(self, U, out=None):
        out = torch.empty_like(U) if out is None else out
        return rhs(self.grid, self.scheme, self.params, U, self.M, out, self.ws)

    def cfl_dt(self, U, cfl):
        return cfl_dt(self.grid, self.params, U, self.M, cfl, self.dt, self.ws)

    def rk3_step(self, U, dt=None):
        if dt is not None:
            self.dt.fill_(float(dt))
        return rk3_step(self.grid, self.scheme, self.params, U, self.M, self.dt, self.ws)

    def rk3_step_cfl(self, U, cfl):
        """CFL time step of U (into self.dt) and one RK3 step of that size."""
        return rk3_step_cfl(self.grid, self.scheme, self.params, U, self.M, cfl, self.dt, self.ws)

    def rk3_steps_cfl(self, U, cfl, nsteps, dts=None):
        """nsteps CFL-limited RK3 steps in one call; returns the device
        tensor of the step sizes (dts, or a new one)."""
        dts = torch.empty(int(nsteps), dtype=torch.float64, device=self.device) if dts is None else dts
        rk3_steps_cfl(self.grid, self.scheme, self.params, U, self.M, cfl, int(nsteps), dts, self.ws)
        return dts

    def rhs_vjp(self, U, Gbar, out=None):
        out = torch.empty_like(U) if out is None else out
        return rhs_vjp(self.grid, self.scheme, self.params, U, self.M, Gbar, out, self.ws)

    def rk3_step_stages(self, U, U1, U2, ws=None, rec=None):
        return rk3_step_stages(self.grid, self.scheme, self.params, U, self.M, self.dt, U1, U2,
                               self.ws if ws is None else ws, rec)

    def rk3_steps_stages(self, U, stages, recs, ws=None):
        return rk3_steps_stages(self.grid, self.scheme, self.params, U, self.M, self.dt, stages, recs,
                                self.ws if ws is None else ws)

    def step_record(self, n=None):
        """Device buffer for one step record (or `n` of them, as rows)."""
        nb = step_record_bytes(self.grid)
        shape = (nb // 8,) if n is None else (n, nb // 8)
        return torch.empty(shape, dtype=torch.int64, device=self.device)

    def side_workspace(self):
        """A second workspace of this grid (lazily created), for work issued
        on another stream concurrently with calls that use self.ws."""
        if getattr(self, "_ws2", None) is None:
            self._ws2 = workspace(self.grid, self.device)
            workspace_init(self._ws2)
        return self._ws2

    def rk3_step_vjp(self, U_n, Ubar_np1, U1=None, U2=None, out=None, rec=None):
        out = torch.empty_like(U_n) if out is None else out
        return rk3_step_vjp(self.grid, self.scheme, self.params, U_n, U1, U2, self.M, self.dt, Ubar_np1, out, self.ws,
                            rec)

    def line_eigenvalues(self, U):
        lx = torch.empty(self.grid.ny, dtype=torch.float64, device=self.device)
        le = torch.empty(self.grid.nx, dtype=torch.float64, device=self.device)
        line_eigenvalues(self.grid, self.params, U, self.M, lx, le, self.ws)
        return lx, le

    def status(self, clear=True):
        st = status(self.ws, clear)
        if getattr(self, "_ws2", None) is not None:
            st |= status(self._ws2, clear)
        return st

    def planes(self):
        return metric_planes(self.M, self.grid)


class BatchedPlan:
    """Many blocks stepped together (wiu_batched_*).

    blocks: either (x, y, bc, period) node-coordinate arrays per block
    (independent blocks, each with its own boundary rule), or objects with
    attributes x, y, bc, period, sides, nbr, nbr_side, shift, fixed (a
    multi-block grid: per-side rules, "interface" sides coupling the blocks
    as stated with wiu_block in wenoiu.h; metrics from wiu_blocks_metrics).
    U_all and M_all are flat device tensors owned here; block b's state is
    U_all[off_U[b] : off_U[b] + 4 ny nx] viewed as (4, ny, nx)."""

    def __init__(self, blocks, scheme="5-2MP", params=None, xi_variant=None, eta_variant=None, device="cuda"):
        self.scheme = scheme
        self.params = params or make_params()
        self.device = device
        self.shapes = []
        self.coupled = any(hasattr(b, "sides") for b in blocks)
        descs = []
        offU = offM = offX = 0
        for blk in blocks:
            x, y, bc, period = (blk.x, blk.y, blk.bc, blk.period) if self.coupled else blk
            ny, nx = x.shape
            g = make_grid(nx, ny, bc, period)
            d = WiuBlock(nx, ny, g.bc_x, g.bc_y, g.period_x, g.period_y, offU, offM)
            if self.coupled:
                for s_ in range(4):
                    v = blk.sides[s_]
                    d.side[s_] = SIDES[v] if isinstance(v, str) else int(v)
                    d.nbr[s_] = int(blk.nbr[s_])
                    d.nbr_side[s_] = int(blk.nbr_side[s_])
                    for c in range(2):
                        d.shift[s_][c] = float(blk.shift[s_][c])
                    for q in range(4):
                        d.fixed[s_][q] = float(blk.fixed[s_][q])
                d.off_X = offX
                offX += 2 * nx * ny
            descs.append(d)
            self.shapes.append((ny, nx))
            offU += 4 * nx * ny
            offM += metrics_size(g) // 8
        self.off_U = [d.off_U for d in descs]
        self.U_all = torch.zeros(offU, dtype=torch.float64, device=device)
        self.M_all = torch.zeros(offM, dtype=torch.float64, device=device)
        self._descs = (WiuBlock * len(descs))(*descs)
        if self.coupled:
            # metrics of all blocks on their coupled coordinates (one-time)
            X = torch.cat([torch.as_tensor(a, dtype=torch.float64).reshape(-1)
                           for blk in blocks for a in (blk.x, blk.y)]).to(device).contiguous()
            n = lib.wiu_blocks_metrics_work_size(self._descs, len(descs), scheme_id(scheme))
            if n == 0:
                raise WiuError("invalid multi-block grid")
            work = torch.zeros(n, dtype=torch.uint8, device=device)
            _check(lib.wiu_blocks_metrics(self._descs, len(descs), scheme_id(scheme), ctypes.byref(self.params),
                                          ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(self.M_all.data_ptr()),
                                          ctypes.c_void_p(work.data_ptr()), _stream()))
            if status(work):
                raise WiuError("metrics reported a folded cell")
        else:
            # metrics of every block with the single-grid entry point (one-time)
            for d, (x, y, bc, period) in zip(descs, blocks):
                g = make_grid(d.nx, d.ny, bc, period)
                ws = workspace(g, device)
                xx = torch.as_tensor(x, dtype=torch.float64).to(device).contiguous()
                yy = torch.as_tensor(y, dtype=torch.float64).to(device).contiguous()
                Mb = self.M_all[d.off_M: d.off_M + metrics_size(g) // 8]
                metrics(g, scheme, xx, yy, Mb, ws, params=self.params)
                if status(ws):
                    raise WiuError("metrics reported a folded cell")
        self.plan = ctypes.c_void_p()
        self.retune(get_tuning(0) if xi_variant is None else xi_variant,
                    get_tuning(1) if eta_variant is None else eta_variant)

    def retune(self, xi_variant, eta_variant):
        """(Re)create the device plan with other tile shapes; the state,
        metrics and time steps are kept."""
        dt = self.get_dt() if self.plan else None
        self.close()
        _check(lib.wiu_batched_plan(self._descs, len(self._descs), scheme_id(self.scheme), ctypes.byref(self.params),
                                    int(xi_variant), int(eta_variant), ctypes.c_void_p(self.U_all.data_ptr()),
                                    ctypes.c_void_p(self.M_all.data_ptr()), ctypes.byref(self.plan)))
        self.variant = (int(xi_variant), int(eta_variant))
        if dt is not None:
            self.set_dt(dt)

    def state(self, b):
        ny, nx = self.shapes[b]
        return self.U_all[self.off_U[b]: self.off_U[b] + 4 * nx * ny].view(4, ny, nx)

    def metric_array(self, b):
        d = self._descs[b]
        g = make_grid(d.nx, d.ny, (d.bc_x, d.bc_y), (d.period_x, d.period_y))
        return self.M_all[d.off_M: d.off_M + metrics_size(g) // 8]

    def info(self):
        c = ctypes.c_longlong(0)
        a = ctypes.c_int(0)
        b = ctypes.c_int(0)
        _check(lib.wiu_batched_info(self.plan, ctypes.byref(c), ctypes.byref(a), ctypes.byref(b)))
        return c.value, a.value, b.value

    def set_dt(self, dt):
        import numpy as np
        arr = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (len(self.shapes),)))
        _check(lib.wiu_batched_set_dt(self.plan, arr.ctypes.data_as(ctypes.c_void_p), _stream()))

    def cfl_dt(self, cfl):
        _check(lib.wiu_batched_cfl_dt(self.plan, float(cfl), _stream()))

    def get_dt(self):
        import numpy as np
        arr = np.zeros(len(self.shapes))
        _check(lib.wiu_batched_get_dt(self.plan, arr.ctypes.data_as(ctypes.c_void_p), _stream()))
        return arr

    def step(self, graph=True):
        _check(lib.wiu_batched_rk3_step(self.plan, int(bool(graph)), _stream()))

    def status(self, clear=True):
        v = ctypes.c_int(0)
        _check(lib.wiu_batched_status(self.plan, _stream(), ctypes.byref(v), int(clear)))
        return v.value

    def close(self):
        if self.plan:
            lib.wiu_plan_destroy(self.plan)
            self.plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- three-dimensional grids (wiu3_*) -------------------------------------------

def make_grid3(nx, ny, nz, bc=("periodic",) * 3, period=(0.0, 0.0, 0.0), sides=None, fixed=None):
    """3-D grid description; sides: rules of x low .. z high of the
    non-periodic directions ("transmissive", "wall", "fixed"), fixed: their
    conservative states [6][5]."""
    g = WiuGrid3(int(nx), int(ny), int(nz))
    for a in range(3):
        g.bc[a] = BC[bc[a]] if isinstance(bc[a], str) else int(bc[a])
        g.period[a] = float(period[a])
    if sides is not None:
        for k, v in enumerate(sides):
            g.side[k] = SIDES[v] if isinstance(v, str) else int(v)
    if fixed is not None:
        for k in range(6):
            for q in range(5):
                g.fixed[k][q] = float(fixed[k][q])
    return g


class Solver3:
    """A 3-D grid on the device: coordinates (nz, ny, nx) arrays, metrics
    computed once for `scheme` (J^{-1} by Eq. 2.5 or, jform=6, Eq. 2.6), a
    workspace; states are (5, nz, ny, nx) fp64 device tensors."""

    def __init__(self, x, y, z, scheme="5-2MP", bc=("periodic",) * 3, period=(0.0, 0.0, 0.0), params=None,
                 device="cuda", jform=5, sides=None, fixed=None):
        nz, ny, nx = x.shape
        self.grid = make_grid3(nx, ny, nz, bc, period, sides, fixed)
        self.scheme = scheme
        self.params = params or make_params()
        nm = lib.wiu3_metrics_size(ctypes.byref(self.grid))
        nw = lib.wiu3_workspace_bytes(ctypes.byref(self.grid))
        if nm == 0 or nw == 0:
            raise WiuError("invalid 3-D grid")
        self.M = torch.zeros(nm // 8, dtype=torch.float64, device=device)
        self.ws = torch.zeros(nw, dtype=torch.uint8, device=device)
        self.dt = torch.zeros(1, dtype=torch.float64, device=device)
        xyz = [torch.as_tensor(a, dtype=torch.float64).to(device).contiguous() for a in (x, y, z)]
        _check(lib.wiu3_metrics(ctypes.byref(self.grid), scheme_id(scheme), int(jform), ctypes.byref(self.params),
                                *[_ptr(a) for a in xyz],
                                _ptr(self.M),
                                ctypes.c_void_p(self.ws.data_ptr()), _stream()))
        if status(self.ws):
            raise WiuError("metrics reported a folded cell")

    def planes(self):
        g = self.grid
        P = (g.nx + 8) * (g.ny + 8) * (g.nz + 8)
        return self.M[:19 * P].view(19, g.nz + 8, g.ny + 8, g.nx + 8)

    def rhs(self, U, out=None):
        out = torch.empty_like(U) if out is None else out
        _check(lib.wiu3_rhs(ctypes.byref(self.grid), scheme_id(self.scheme), ctypes.byref(self.params), _ptr(U),
                            _ptr(self.M), _ptr(out), ctypes.c_void_p(self.ws.data_ptr()), _stream()))
        return out

    def cfl_dt(self, U, cfl):
        _check(lib.wiu3_cfl_dt(ctypes.byref(self.grid), ctypes.byref(self.params), _ptr(U), _ptr(self.M), float(cfl),
                               _ptr(self.dt), ctypes.c_void_p(self.ws.data_ptr()), _stream()))
        return self.dt

    def rk3_step(self, U, dt=None):
        if dt is not None:
            self.dt.fill_(float(dt))
        _check(lib.wiu3_rk3_step(ctypes.byref(self.grid), scheme_id(self.scheme), ctypes.byref(self.params), _ptr(U),
                                 _ptr(self.M), _ptr(self.dt), ctypes.c_void_p(self.ws.data_ptr()), _stream()))

    def rk3_step_cfl(self, U, cfl):
        """cfl_dt then rk3_step with one shared pass over U; returns the
        device time step."""
        _check(lib.wiu3_rk3_step_cfl(ctypes.byref(self.grid), scheme_id(self.scheme), ctypes.byref(self.params),
                                     _ptr(U), _ptr(self.M), float(cfl), _ptr(self.dt),
                                     ctypes.c_void_p(self.ws.data_ptr()), _stream()))
        return self.dt

    def rk3_steps_cfl(self, U, cfl, nsteps, dts=None):
        """nsteps CFL-limited RK3 steps in one call; returns the device
        tensor of the step sizes (dts, or a new one)."""
        dts = torch.empty(int(nsteps), dtype=torch.float64, device=self.M.device) if dts is None else dts
        if dts.numel() < nsteps or dts.dtype != torch.float64 or not dts.is_contiguous():
            raise ValueError("dts: a contiguous float64 tensor of at least nsteps entries")
        _check(lib.wiu3_rk3_steps_cfl(ctypes.byref(self.grid), scheme_id(self.scheme), ctypes.byref(self.params),
                                      _ptr(U), _ptr(self.M), float(cfl), int(nsteps), _ptr(dts),
                                      ctypes.c_void_p(self.ws.data_ptr()), _stream()))
        return dts

    def status(self, clear=True):
        return status(self.ws, clear)
