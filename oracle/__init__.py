"""ctypes binding of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

The oracle is a plain scalar C++ implementation of the WENOIU method written
from the paper (see ``wenoiu_oracle.hpp``).  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark may use it; the product path
(the HIP library and its Python binding) never imports this package.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

SCHEMES = {"3-1MP": 0, "3-2MP": 1, "5-1MP": 2, "5-2MP": 3, "7-1MP": 4, "7-2MP": 5, "7-4MP": 6, "7-6MP": 7}
BC = {"periodic": 0, "transmissive": 1}
G = 4  # metric ghost band

_D = ctypes.c_double
_I = ctypes.c_int
_P = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        # ORACLE_LIB: another build of the same source (the sanitizer build of
        # tests/test_oracle_sanitizers.py); otherwise the regular library
        path = os.environ.get("ORACLE_LIB") or _build.LIB
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        L.orc_weno.restype = _D
        L.orc_weno.argtypes = [_I, _P, _D, _I, _I]
        L.orc_ppm.restype = _D
        L.orc_ppm.argtypes = [_I, _D, _D]
        L.orc_is.restype = _D
        L.orc_is.argtypes = [_I, _D, _D, _D]
        L.orc_is4.restype = _D
        L.orc_is4.argtypes = [_I, _D, _D, _D, _D]
        L.orc_hplus.restype = _D
        L.orc_hplus.argtypes = [_I, _D, _P, _P]
        L.orc_delta_c.restype = _D
        L.orc_delta_c.argtypes = [_I, _D, _P, _P]
        L.orc_delta_c_eq27.restype = _D
        L.orc_delta_c_eq27.argtypes = [_I, _D, _P, _P]
        L.orc_interp_mid.restype = _D
        L.orc_interp_mid.argtypes = [_I, _P]
        L.orc_metric_derivative.restype = _D
        L.orc_metric_derivative.argtypes = [_I, _D, _P]
        L.orc_eigenvectors.restype = None
        L.orc_eigenvectors.argtypes = [_P, _D, _D, _D, _P, _P]
        L.orc_flux_hat.restype = None
        L.orc_flux_hat.argtypes = [_P, _D, _D, _D, _P]
        L.orc_midpoint_flux.restype = _I
        L.orc_midpoint_flux.argtypes = [_I, _D, _D, _I, _I, _I, _I, _P, _P, _P, _P, _D, _P, _P]
        L.orc_metrics_size.restype = ctypes.c_longlong
        L.orc_metrics_size.argtypes = [_I, _I]
        L.orc_metrics.restype = _I
        L.orc_metrics.argtypes = [_I, _D, _I, _I, _I, _I, _D, _D, _P, _P, _P]
        L.orc_rhs.restype = _I
        L.orc_rhs.argtypes = [_I, _I, _I, _I, _I, _P, _P, _D, _D, _D, _I, _I, _D, _I, _I, _P, _P, _P, _P, _P]
        L.orc_cfl_dt.restype = _D
        L.orc_cfl_dt.argtypes = [_I, _I, _D, _P, _P, _D]
        L.orc_rk3_step.restype = _I
        L.orc_rk3_step.argtypes = [_I, _I, _I, _I, _I, _P, _P, _D, _D, _D, _I, _I, _D, _I, _I, _P, _P, _D]
        L.orc_rk3_run.restype = _I
        L.orc_rk3_run.argtypes = [_I, _I, _I, _I, _I, _P, _P, _D, _D, _D, _I, _I, _D, _I, _I, _P, _P, _D, _I]
        L.orc_adv1d_rhs.restype = None
        L.orc_adv1d_rhs.argtypes = [_I, _I, _D, _I, _D, _D, _I, _D, _I, _P, _P]
        L.orc_adv1d_run.restype = _I
        L.orc_adv1d_run.argtypes = [_I, _I, _I, _D, _D, _I, _D, _I, _D, _D, _P, _P]
        for nm in ("orc_rhs_jvp", "orc_rk3_step_jvp"):
            f = getattr(L, nm)
            f.restype = _I
        L.orc_rhs_jvp.argtypes = [_I, _I, _I, _I, _I, _P, _P, _D, _D, _D, _I, _I, _D, _I, _I, _P, _P, _P, _P, _P]
        L.orc_rk3_step_jvp.argtypes = [_I, _I, _I, _I, _I, _P, _P, _D, _D, _D, _I, _I, _D, _I, _I, _P, _P, _P, _D, _P, _P]
        L.orc_rhs_vjp.restype = _I
        L.orc_rhs_vjp.argtypes = [_I, _I, _I, _I, _I, _P, _P, _D, _D, _D, _I, _I, _D, _I, _I, _P, _P, _P, _P]
        L.orc_rk3_step_vjp.restype = _I
        L.orc_rk3_step_vjp.argtypes = [_I, _I, _I, _I, _I, _P, _P, _D, _D, _D, _I, _I, _D, _I, _I, _P, _P, _D, _P, _P]
        L.orc_count_rhs_flops.restype = _I
        L.orc_count_rhs_flops.argtypes = [_I, _I, _I, _I, _I, _P, _P, _D, _D, _D, _I, _I, _D, _I, _I, _P, _P, _P]
        for f in ("orc_mb_metrics", "orc_mb_rhs", "orc_mb_rk3_step", "orc_mb_cfl_dt"):
            getattr(L, f).restype = _I
        L.orc_mb_metrics.argtypes = [_I, _D, _I, _P, _P, _P, _P, _P, _P]
        L.orc_mb_rhs.argtypes = [_I, _I, _P, _P, _D, _D, _D, _I, _I, _D, _I, _I, _P, _P, _P, _P, _P]
        L.orc_mb_rk3_step.argtypes = [_I, _I, _P, _P, _D, _D, _D, _I, _I, _D, _I, _I, _P, _P, _P, _P, _P]
        L.orc_mb_cfl_dt.argtypes = [_I, _P, _P, _D, _P, _P, _P, _P, _D, _P]
        L.orc3_metrics_size.restype = ctypes.c_longlong
        L.orc3_metrics_size.argtypes = [_P]
        L.orc3_metrics.argtypes = [_I, _P, _P, _P, _P, _P, _P, _P, _I, _D]
        L.orc3_rhs.argtypes = [_I, _P, _P, _P, _P, _D, _D, _D, _I, _I, _D, _I, _I, _P, _P, _P]
        L.orc3_cfl_dt.restype = _D
        L.orc3_cfl_dt.argtypes = [_P, _D, _P, _P, _D]
        L.orc3_rk3_step.argtypes = [_I, _P, _P, _P, _P, _D, _D, _D, _I, _I, _D, _I, _I, _P, _P, _D]
        L.orc3_eigenvectors.restype = None
        L.orc3_eigenvectors.argtypes = [_P, _D, _P, _P, _P]
        L.orc3_flux_hat.restype = None
        L.orc3_flux_hat.argtypes = [_P, _D, _P, _P]
        L.orc3_count_line_flops.argtypes = [_I, _I, _D, _P, _P, _P]
        L.orc3_midpoint_split.restype = None
        L.orc3_midpoint_split.argtypes = [_I, _D, _P, _P, _I, _P]
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [_I]
        L.orc_get_threads.restype = _I
        L.orc_get_threads.argtypes = []
        _lib = L
    return _lib


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


VARS = {"characteristic": 0, "conservative": 1, "primitive": 2}


def vars_id(v):
    """Interpolation variables (Sec. 2.4): name or 0/1/2."""
    return VARS[v] if isinstance(v, str) else int(v)


WEIGHTS = {"js": 0, "z": 1}
SPLITS = {"lf": 0, "sw": 1, "vl": 2}


def weights_id(w):
    """Nonlinear weights: "js" (Jiang-Shu, Eqs. 3.12-3.13) or "z" (WENO-Z)."""
    return WEIGHTS[w] if isinstance(w, str) else int(w)


def split_id(s):
    """Midpoint flux split: "lf" (Lax-Friedrichs), "sw" (Steger-Warming), "vl" (van Leer)."""
    return SPLITS[s] if isinstance(s, str) else int(s)


SIDES = {"transmissive": 0, "wall": 1, "fixed": 2}


def _sides(sides, fixed):
    """(side kinds, fixed states) of the four sides (x lo, x hi, y lo, y hi) as
    ctypes pointers, or nulls for all-transmissive.  sides: names or 0/1/2;
    fixed: conservative states [4][4] used by "fixed" sides."""
    if sides is None:
        return None, None
    k = np.ascontiguousarray([SIDES[v] if isinstance(v, str) else int(v) for v in sides], dtype=np.int32)
    f = np.zeros((4, 4)) if fixed is None else np.ascontiguousarray(fixed, dtype=np.float64).reshape(4, 4)
    _sides.keep = (k, f)  # alive for the duration of the call
    return k.ctypes.data_as(ctypes.c_void_p), f.ctypes.data_as(ctypes.c_void_p)


def scheme_id(s):
    return SCHEMES[s] if isinstance(s, str) else int(s)


def bc_id(b):
    return BC[b] if isinstance(b, str) else int(b)


def set_threads(n):
    lib().orc_set_threads(int(n))


def get_threads():
    return lib().orc_get_threads()


# ---- component probes ------------------------------------------------------------

def weno(r, v, eps=1e-40, ppm=1, weights=0):
    v = _f64(v)
    return lib().orc_weno(r, _ptr(v), eps, ppm, weights_id(weights))


def ppm(order, w, C):
    return lib().orc_ppm(order, w, C)


def smoothness(k, a, b, c):
    return lib().orc_is(k, a, b, c)


def smoothness4(k, a, b, c, d):
    """r = 4 indicator of stencil k (0 = leftmost) on four values."""
    return lib().orc_is4(k, a, b, c, d)


def hplus(scheme, f, F, alpha_h=1.0):
    """h^+_{i+1/2}; f = f_{i-3..i+3} (7 values), F = f_{i-5/2..i+5/2} (6 values;
    4 values f_{i-3/2..i+3/2} are accepted and padded with zeros).  alpha_h:
    free parameter of the one-midpoint families."""
    f, F = _f64(f), _f64(F)
    if F.size == 4:
        F = np.concatenate([[0.0], F, [0.0]])
    return lib().orc_hplus(scheme_id(scheme), float(alpha_h), _ptr(f), _ptr(F))


def delta_c(scheme, g, gm, alpha_h=1.0):
    """delta^{c,(1)} at i; g = g_{i-4..i+4} (9), gm = g_{i-7/2..i+7/2} (8)."""
    g, gm = _f64(g), _f64(gm)
    return lib().orc_delta_c(scheme_id(scheme), float(alpha_h), _ptr(g), _ptr(gm))


def delta_c_eq27(scheme, g, gm, alpha_h=1.0):
    """The central operator built by Eq. 2.7 from h^+ (any alpha_h)."""
    g, gm = _f64(g), _f64(gm)
    return lib().orc_delta_c_eq27(scheme_id(scheme), float(alpha_h), _ptr(g), _ptr(gm))


def interp_mid(g):
    """Midpoint value g_{i+1/2} from g_{i-2..i+3} (6 values) or g_{i-3..i+4} (8)."""
    g = _f64(g)
    if g.size not in (6, 8):
        raise ValueError("interp_mid takes 6 or 8 values")
    return lib().orc_interp_mid(g.size, _ptr(g))


def metric_derivative(scheme, r, alpha_h=1.0):
    r = _f64(r)
    return lib().orc_metric_derivative(scheme_id(scheme), float(alpha_h), _ptr(r))


def eigenvectors(Q, gamma, nx, ny):
    Q = _f64(Q)
    L = np.zeros((4, 4))
    R = np.zeros((4, 4))
    lib().orc_eigenvectors(_ptr(Q), gamma, nx, ny, _ptr(L), _ptr(R))
    return L, R


def flux_hat(Q, gamma, kx, ky):
    Q = _f64(Q)
    out = np.zeros(4)
    lib().orc_flux_hat(_ptr(Q), gamma, kx, ky, _ptr(out))
    return out


def midpoint_flux(scheme, Qs, k0, k1, mk, lam, gamma=1.4, eps=1e-40, ppm=1, vars=0, weights=0, split=0):
    """F^+, F^- at k+1/2 from Qs = Q_{k-3..k+4} (8 states; 6 states Q_{k-2..k+3}
    are accepted for the third- and fifth-order schemes)."""
    Qs, k0, k1, mk = _f64(Qs), _f64(k0), _f64(k1), _f64(mk)
    if Qs.shape[0] == 6:
        Qs = np.ascontiguousarray(np.concatenate([Qs[:1], Qs, Qs[-1:]]))
    Fp, Fm = np.zeros(4), np.zeros(4)
    rc = lib().orc_midpoint_flux(scheme_id(scheme), gamma, eps, ppm, vars_id(vars), weights_id(weights),
                                 split_id(split), _ptr(Qs), _ptr(k0), _ptr(k1),
                                 _ptr(mk), lam, _ptr(Fp), _ptr(Fm))
    assert rc == 0
    return Fp, Fm


# ---- 2-D Euler ----------------------------------------------------------------------

def metrics(scheme, x, y, bc=("periodic", "periodic"), period=(0.0, 0.0), alpha_h=1.0):
    """Nine metric planes with the ghost band: shape (9, ny+2G, nx+2G)."""
    x, y = _f64(x), _f64(y)
    ny, nx = x.shape
    M = np.zeros((9, ny + 2 * G, nx + 2 * G))
    rc = lib().orc_metrics(scheme_id(scheme), float(alpha_h), nx, ny, bc_id(bc[0]), bc_id(bc[1]), float(period[0]),
                           float(period[1]), _ptr(x), _ptr(y), _ptr(M))
    if rc:
        raise ValueError("orc_metrics failed")
    return M


def rhs(scheme, U, M, bc=("periodic", "periodic"), gamma=1.4, alpha=1.1, eps=1e-40, ppm=1, vars=0, alpha_h=1.0, weights=0, split=0,
        sides=None, fixed=None,
        return_lambda=False):
    U, M = _f64(U), _f64(M)
    _, ny, nx = U.shape
    out = np.zeros_like(U)
    lx = np.zeros(ny)
    le = np.zeros(nx)
    rc = lib().orc_rhs(scheme_id(scheme), nx, ny, bc_id(bc[0]), bc_id(bc[1]), *_sides(sides, fixed), gamma, alpha, eps, ppm, vars_id(vars), float(alpha_h), weights_id(weights), split_id(split),
                       _ptr(U), _ptr(M), _ptr(out), _ptr(lx), _ptr(le))
    if rc:
        raise ValueError("orc_rhs failed")
    if return_lambda:
        return out, lx, le
    return out


def count_rhs_flops(scheme, U, M, bc=("periodic", "periodic"), gamma=1.4, alpha=1.1, eps=1e-40, ppm=1, vars=0, alpha_h=1.0, weights=0, split=0,
        sides=None, fixed=None):
    """Operation counts of one rhs: (xi sweep, eta sweep, final combination)."""
    U, M = _f64(U), _f64(M)
    _, ny, nx = U.shape
    c = np.zeros(3, dtype=np.int64)
    rc = lib().orc_count_rhs_flops(scheme_id(scheme), nx, ny, bc_id(bc[0]), bc_id(bc[1]), *_sides(sides, fixed), gamma, alpha, eps, ppm, vars_id(vars), float(alpha_h), weights_id(weights), split_id(split),
                                   _ptr(U), _ptr(M), _ptr(c))
    if rc:
        raise ValueError("orc_count_rhs_flops failed")
    return tuple(int(v) for v in c)


def rhs_jvp(scheme, U, V, M, bc=("periodic", "periodic"), gamma=1.4, alpha=1.1, eps=1e-40, ppm=1, vars=0, alpha_h=1.0, weights=0, split=0,
        sides=None, fixed=None):
    """(rhs(U), (d rhs/dU) V) by forward-mode dual numbers."""
    U, V, M = _f64(U), _f64(V), _f64(M)
    _, ny, nx = U.shape
    val, tan = np.zeros_like(U), np.zeros_like(U)
    rc = lib().orc_rhs_jvp(scheme_id(scheme), nx, ny, bc_id(bc[0]), bc_id(bc[1]), *_sides(sides, fixed), gamma, alpha, eps, ppm, vars_id(vars), float(alpha_h), weights_id(weights), split_id(split),
                           _ptr(U), _ptr(V), _ptr(M), _ptr(val), _ptr(tan))
    if rc:
        raise ValueError("orc_rhs_jvp failed")
    return val, tan


def rhs_vjp(scheme, U, M, Gbar, bc=("periodic", "periodic"), gamma=1.4, alpha=1.1, eps=1e-40, ppm=1, vars=0, alpha_h=1.0, weights=0, split=0,
        sides=None, fixed=None):
    """(d rhs/dU)^T Gbar by reverse mode on a tape."""
    U, M, Gbar = _f64(U), _f64(M), _f64(Gbar)
    _, ny, nx = U.shape
    out = np.zeros_like(U)
    rc = lib().orc_rhs_vjp(scheme_id(scheme), nx, ny, bc_id(bc[0]), bc_id(bc[1]), *_sides(sides, fixed), gamma, alpha, eps, ppm, vars_id(vars), float(alpha_h), weights_id(weights), split_id(split),
                           _ptr(U), _ptr(M), _ptr(Gbar), _ptr(out))
    if rc:
        raise ValueError("orc_rhs_vjp failed")
    return out


def rk3_step_jvp(scheme, U, V, M, dt, bc=("periodic", "periodic"), gamma=1.4, alpha=1.1, eps=1e-40, ppm=1, vars=0, alpha_h=1.0, weights=0, split=0,
        sides=None, fixed=None):
    U, V, M = _f64(U), _f64(V), _f64(M)
    _, ny, nx = U.shape
    val, tan = np.zeros_like(U), np.zeros_like(U)
    rc = lib().orc_rk3_step_jvp(scheme_id(scheme), nx, ny, bc_id(bc[0]), bc_id(bc[1]), *_sides(sides, fixed), gamma, alpha, eps, ppm, vars_id(vars), float(alpha_h), weights_id(weights), split_id(split),
                                _ptr(U), _ptr(V), _ptr(M), dt, _ptr(val), _ptr(tan))
    if rc:
        raise ValueError("orc_rk3_step_jvp failed")
    return val, tan


def rk3_step_vjp(scheme, U, M, dt, Ubar, bc=("periodic", "periodic"), gamma=1.4, alpha=1.1, eps=1e-40, ppm=1, vars=0, alpha_h=1.0, weights=0, split=0,
        sides=None, fixed=None):
    U, M, Ubar = _f64(U), _f64(M), _f64(Ubar)
    _, ny, nx = U.shape
    out = np.zeros_like(U)
    rc = lib().orc_rk3_step_vjp(scheme_id(scheme), nx, ny, bc_id(bc[0]), bc_id(bc[1]), *_sides(sides, fixed), gamma, alpha, eps, ppm, vars_id(vars), float(alpha_h), weights_id(weights), split_id(split),
                                _ptr(U), _ptr(M), dt, _ptr(Ubar), _ptr(out))
    if rc:
        raise ValueError("orc_rk3_step_vjp failed")
    return out


def cfl_dt(U, M, cfl, gamma=1.4):
    U, M = _f64(U), _f64(M)
    _, ny, nx = U.shape
    return lib().orc_cfl_dt(nx, ny, gamma, _ptr(U), _ptr(M), cfl)


def rk3_step(scheme, U, M, dt, bc=("periodic", "periodic"), gamma=1.4, alpha=1.1, eps=1e-40, ppm=1, vars=0, alpha_h=1.0, weights=0, split=0,
        sides=None, fixed=None):
    U = np.array(U, dtype=np.float64, copy=True, order="C")
    M = _f64(M)
    _, ny, nx = U.shape
    rc = lib().orc_rk3_step(scheme_id(scheme), nx, ny, bc_id(bc[0]), bc_id(bc[1]), *_sides(sides, fixed), gamma, alpha, eps, ppm, vars_id(vars), float(alpha_h), weights_id(weights), split_id(split),
                            _ptr(U), _ptr(M), dt)
    if rc:
        raise ValueError("orc_rk3_step failed")
    return U


def rk3_run(scheme, U, M, dt, nsteps, bc=("periodic", "periodic"), gamma=1.4, alpha=1.1, eps=1e-40, ppm=1, vars=0, alpha_h=1.0, weights=0, split=0,
        sides=None, fixed=None):
    U = np.array(U, dtype=np.float64, copy=True, order="C")
    M = _f64(M)
    _, ny, nx = U.shape
    rc = lib().orc_rk3_run(scheme_id(scheme), nx, ny, bc_id(bc[0]), bc_id(bc[1]), *_sides(sides, fixed), gamma, alpha, eps, ppm, vars_id(vars), float(alpha_h), weights_id(weights), split_id(split),
                           _ptr(U), _ptr(M), dt, int(nsteps))
    if rc:
        raise ValueError("orc_rk3_run failed")
    return U


# ---- Sec. 5.1 scalar advection ------------------------------------------------------------

def adv1d_rhs(scheme, u, dx, split=0, alpha=1.1, eps=1e-40, ppm=1, alpha_h=1.0, weights=0):
    u = _f64(u)
    out = np.zeros_like(u)
    lib().orc_adv1d_rhs(scheme_id(scheme), u.size, dx, split, alpha, eps, ppm, float(alpha_h), weights_id(weights),
                        _ptr(u), _ptr(out))
    return out


def adv1d_run(scheme, N, split=0, alpha=1.1, eps=1e-40, ppm=1, tend=2.0, dtpow=1.25, alpha_h=1.0, weights=0):
    l2 = ctypes.c_double()
    li = ctypes.c_double()
    rc = lib().orc_adv1d_run(scheme_id(scheme), N, split, alpha, eps, ppm, float(alpha_h), weights_id(weights), tend,
                             dtpow, ctypes.byref(l2), ctypes.byref(li))
    if rc:
        raise ValueError("orc_adv1d_run failed")
    return l2.value, li.value


# ---- multi-block grids (multiblock.hpp) -----------------------------------------

SIDE_KINDS = {"transmissive": 0, "wall": 1, "fixed": 2, "interface": 3}


def _mb_desc(blocks):
    """Block descriptors: idesc[b] = nx, ny, bcx, bcy, side[4], nbr[4],
    nbr_side[4]; fdesc[b] = Lx, Ly, shift[4][2], fixed[4][4]."""
    I = np.zeros((len(blocks), 16), dtype=np.int32)
    F = np.zeros((len(blocks), 26))
    for b, k in enumerate(blocks):
        ny, nx = k.x.shape
        I[b, :4] = nx, ny, bc_id(k.bc[0]), bc_id(k.bc[1])
        I[b, 4:8] = [SIDE_KINDS[v] if isinstance(v, str) else int(v) for v in k.sides]
        I[b, 8:12] = k.nbr
        I[b, 12:16] = k.nbr_side
        F[b, :2] = k.period
        F[b, 2:10] = np.asarray(k.shift, dtype=np.float64).reshape(8)
        F[b, 10:26] = np.asarray(k.fixed, dtype=np.float64).reshape(16)
    return I, F


def _concat(arrays):
    arrays = [_f64(a) for a in arrays]
    off = np.zeros(len(arrays), dtype=np.int64)
    pos = 0
    for b, a in enumerate(arrays):
        off[b] = pos
        pos += a.size
    return np.concatenate([a.ravel() for a in arrays]) if arrays else np.zeros(0), off


def _split(flat, off, like):
    return [flat[o:o + a.size].reshape(a.shape).copy() for o, a in zip(off, like)]


def mb_metrics(scheme, blocks, alpha_h=1.0):
    """Metric arrays (9, ny+2G, nx+2G) of every block, coupled through the
    blocks' interfaces."""
    I, F = _mb_desc(blocks)
    X, offX = _concat([np.concatenate([_f64(k.x).ravel(), _f64(k.y).ravel()]) for k in blocks])
    shapes = [np.zeros((9, k.x.shape[0] + 2 * G, k.x.shape[1] + 2 * G)) for k in blocks]
    M, offM = _concat(shapes)
    rc = lib().orc_mb_metrics(scheme_id(scheme), float(alpha_h), len(blocks), _ptr(I), _ptr(F), _ptr(X), _ptr(offX),
                              _ptr(M), _ptr(offM))
    if rc:
        raise ValueError("orc_mb_metrics: invalid scheme or connectivity")
    return _split(M, offM, shapes)


def mb_rhs(scheme, blocks, Us, Ms, gamma=1.4, alpha=1.1, eps=1e-40, ppm=1, vars=0, alpha_h=1.0, weights=0, split=0):
    I, F = _mb_desc(blocks)
    U, offU = _concat(Us)
    M, offM = _concat(Ms)
    out = np.zeros_like(U)
    rc = lib().orc_mb_rhs(scheme_id(scheme), len(blocks), _ptr(I), _ptr(F), gamma, alpha, eps, ppm, vars_id(vars),
                          float(alpha_h), weights_id(weights), split_id(split), _ptr(U), _ptr(offU), _ptr(M),
                          _ptr(offM), _ptr(out))
    if rc:
        raise ValueError("orc_mb_rhs: invalid options or connectivity")
    return _split(out, offU, Us)


def mb_rk3_step(scheme, blocks, Us, Ms, dts, gamma=1.4, alpha=1.1, eps=1e-40, ppm=1, vars=0, alpha_h=1.0, weights=0,
                split=0):
    I, F = _mb_desc(blocks)
    U, offU = _concat(Us)
    M, offM = _concat(Ms)
    dt = _f64(np.broadcast_to(np.asarray(dts, dtype=np.float64), (len(blocks),)))
    rc = lib().orc_mb_rk3_step(scheme_id(scheme), len(blocks), _ptr(I), _ptr(F), gamma, alpha, eps, ppm,
                               vars_id(vars), float(alpha_h), weights_id(weights), split_id(split), _ptr(U),
                               _ptr(offU), _ptr(M), _ptr(offM), _ptr(dt))
    if rc:
        raise ValueError("orc_mb_rk3_step: invalid options or connectivity")
    return _split(U, offU, Us)


def mb_cfl_dt(blocks, Us, Ms, cfl, gamma=1.4):
    """Per-block CFL time step, the minimum over each set of blocks joined
    by interfaces."""
    I, F = _mb_desc(blocks)
    U, offU = _concat(Us)
    M, offM = _concat(Ms)
    dt = np.zeros(len(blocks))
    rc = lib().orc_mb_cfl_dt(len(blocks), _ptr(I), _ptr(F), gamma, _ptr(U), _ptr(offU), _ptr(M), _ptr(offM),
                             float(cfl), _ptr(dt))
    if rc:
        raise ValueError("orc_mb_cfl_dt: invalid connectivity")
    return dt


# ---- three-dimensional grids (euler3d.hpp) --------------------------------------

def _i3(v):
    return np.ascontiguousarray(v, dtype=np.int32)


def metrics3(scheme, x, y, z, bc=("periodic",) * 3, period=(0.0, 0.0, 0.0), jform=5, alpha_h=1.0):
    """19 metric planes with the ghost band: shape (19, nz+2G, ny+2G, nx+2G);
    jform 5 or 6: the Jacobian by Eq. 2.5 or Eq. 2.6."""
    x, y, z = _f64(x), _f64(y), _f64(z)
    nz, ny, nx = x.shape
    n = _i3([nx, ny, nz])
    b = _i3([bc_id(v) for v in bc])
    L = _f64(period)
    M = np.zeros((19, nz + 2 * G, ny + 2 * G, nx + 2 * G))
    if lib().orc3_metrics(scheme_id(scheme), _ptr(n), _ptr(b), _ptr(L), _ptr(x), _ptr(y), _ptr(z), _ptr(M),
                          int(jform), float(alpha_h)):
        raise ValueError("orc3_metrics failed")
    return M


def _sides3(sides, fixed):
    """(side kinds, fixed states) of the six sides (x lo, x hi, y lo, y hi,
    z lo, z hi) as ctypes pointers, or nulls for all-transmissive."""
    if sides is None:
        return None, None
    k = np.ascontiguousarray([SIDES[v] if isinstance(v, str) else int(v) for v in sides], dtype=np.int32)
    f = np.zeros((6, 5)) if fixed is None else np.ascontiguousarray(fixed, dtype=np.float64).reshape(6, 5)
    _sides3.keep = (k, f)
    return k.ctypes.data_as(ctypes.c_void_p), f.ctypes.data_as(ctypes.c_void_p)


def rhs3(scheme, U, M, bc=("periodic",) * 3, gamma=1.4, alpha=1.1, eps=1e-40, ppm=1, sides=None, fixed=None,
         vars=0, alpha_h=1.0, weights=0, split=0):
    U, M = _f64(U), _f64(M)
    _, nz, ny, nx = U.shape
    out = np.zeros_like(U)
    if lib().orc3_rhs(scheme_id(scheme), _ptr(_i3([nx, ny, nz])), _ptr(_i3([bc_id(v) for v in bc])),
                      *_sides3(sides, fixed), gamma, alpha, eps, ppm, vars_id(vars), float(alpha_h),
                      weights_id(weights), split_id(split), _ptr(U), _ptr(M), _ptr(out)):
        raise ValueError("orc3_rhs failed")
    return out


def cfl_dt3(U, M, cfl, gamma=1.4):
    U, M = _f64(U), _f64(M)
    _, nz, ny, nx = U.shape
    return lib().orc3_cfl_dt(_ptr(_i3([nx, ny, nz])), gamma, _ptr(U), _ptr(M), float(cfl))


def rk3_step3(scheme, U, M, dt, bc=("periodic",) * 3, gamma=1.4, alpha=1.1, eps=1e-40, ppm=1, sides=None, fixed=None,
              vars=0, alpha_h=1.0, weights=0, split=0):
    U = _f64(U).copy()
    M = _f64(M)
    _, nz, ny, nx = U.shape
    if lib().orc3_rk3_step(scheme_id(scheme), _ptr(_i3([nx, ny, nz])), _ptr(_i3([bc_id(v) for v in bc])),
                           *_sides3(sides, fixed), gamma, alpha, eps, ppm, vars_id(vars), float(alpha_h),
                           weights_id(weights), split_id(split), _ptr(U), _ptr(M), float(dt)):
        raise ValueError("orc3_rk3_step failed")
    return U


def eigenvectors3(Q, gamma, n):
    Q, n = _f64(Q), _f64(n)
    L = np.zeros((5, 5))
    R = np.zeros((5, 5))
    lib().orc3_eigenvectors(_ptr(Q), gamma, _ptr(n), _ptr(L), _ptr(R))
    return L, R


def flux_hat3(Q, gamma, k):
    Q, k = _f64(Q), _f64(k)
    out = np.zeros(5)
    lib().orc3_flux_hat(_ptr(Q), gamma, _ptr(k), _ptr(out))
    return out


def count_line_flops3(scheme, Q, K, gamma=1.4):
    """Operation counts of one 3-D line (Q [5][n], K [6][n+8]) by phase:
    line maximum, nodal split fluxes, midpoint split fluxes, combination."""
    Q, K = _f64(Q), _f64(K)
    n = Q.shape[1]
    c = np.zeros(4, dtype=np.int64)
    if lib().orc3_count_line_flops(scheme_id(scheme), n, gamma, _ptr(Q), _ptr(K), _ptr(c)):
        raise ValueError("orc3_count_line_flops failed")
    return c


def midpoint_split3(split, Q, k, side, gamma=1.4):
    """F+ (side 0) or F- (side 1) of the 3-D Steger-Warming or van Leer split."""
    Q, k = _f64(Q), _f64(k)
    out = np.zeros(5)
    lib().orc3_midpoint_split(split_id(split), gamma, _ptr(Q), _ptr(k), int(side), _ptr(out))
    return out
