"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/wenoiu.h, sizes are as documented and
argument errors are caught on the host before anything is launched."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wenoiu.h")
LIB = os.path.join(ROOT, "paper_1810_11103_amd", "libwenoiu.so")


@pytest.fixture(scope="module")
def wiu():
    if not os.path.exists(LIB):
        from paper_1810_11103_amd import build
        build.build()
    from paper_1810_11103_amd import wenoiu
    return wenoiu


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wiu3?_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("wiu_metrics", "wiu_rhs", "wiu_rk3_step", "wiu_cfl_dt", "wiu_status", "wiu_workspace_bytes"):
        assert n in names


def test_library_exports_every_declared_symbol(wiu):
    # immediate binding: every symbol the library references must resolve
    lib = ctypes.CDLL(LIB, mode=os.RTLD_NOW)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert sorted(wiu.EXPORTS) == sorted(declared_functions())


def test_sizes(wiu):
    g = wiu.make_grid(100, 60, ("periodic", "transmissive"), (1.0, 0.0))
    assert wiu.metrics_size(g) == (9 * 108 * 68 + 8) * 8
    ws = wiu.workspace_bytes(g)
    assert ws % 256 == 0 and ws >= 12 * 100 * 60 * 8


@pytest.mark.parametrize("nx,ny,bc,period", [
    (0, 10, ("periodic", "periodic"), (1, 1)),
    (10, -1, ("periodic", "periodic"), (1, 1)),
    (1, 10, ("transmissive", "periodic"), (0, 1)),
    (10, 10, ("periodic", "periodic"), (0, 1)),
    (10, 10, (2, 0), (1, 1)),
])
def test_bad_grids_rejected_on_host(wiu, nx, ny, bc, period):
    g = wiu.make_grid(nx, ny, bc, period)
    assert wiu.metrics_size(g) == 0
    assert wiu.workspace_bytes(g) == 0
    p = wiu.make_params()
    rc = wiu.lib.wiu_rhs(ctypes.byref(g), 3, ctypes.byref(p), ctypes.c_void_p(8), ctypes.c_void_p(8),
                         ctypes.c_void_p(16), ctypes.c_void_p(8), None)
    assert rc == wiu.WIU_EINVAL


def test_bad_scheme_params_and_pointers_rejected(wiu):
    g = wiu.make_grid(16, 16, ("periodic", "periodic"), (1.0, 1.0))
    p = wiu.make_params()
    dummy = ctypes.c_void_p(256)
    other = ctypes.c_void_p(512)
    assert wiu.lib.wiu_rhs(ctypes.byref(g), 8, ctypes.byref(p), dummy, dummy, other, dummy, None) == wiu.WIU_EINVAL
    # the adjoint covers the third- and fifth-order schemes only
    assert wiu.lib.wiu_rhs_vjp(ctypes.byref(g), 4, ctypes.byref(p), dummy, dummy, other, ctypes.c_void_p(768),
                               dummy, None) == wiu.WIU_EINVAL
    assert wiu.lib.wiu_rhs(ctypes.byref(g), 3, ctypes.byref(p), dummy, dummy, dummy, dummy, None) == wiu.WIU_EINVAL
    assert wiu.lib.wiu_rhs(ctypes.byref(g), 3, ctypes.byref(p), None, dummy, other, dummy, None) == wiu.WIU_EINVAL
    # interpolation variables 0..2; alpha_h != 1 only for the one-midpoint schemes
    for kw, scheme in ((dict(vars=3), 3), (dict(alpha_h=0.9), 3), (dict(alpha_h=-1.0), 0), (dict(alpha_h=0.9), 7),
                       (dict(weights=2), 3), (dict(split=3), 3)):
        q = wiu.make_params(**kw)
        assert wiu.lib.wiu_rhs(ctypes.byref(g), scheme, ctypes.byref(q), dummy, dummy, other, dummy,
                               None) == wiu.WIU_EINVAL, kw
    assert wiu.lib.wiu_metrics(ctypes.byref(g), 3, ctypes.byref(wiu.make_params(alpha_h=0.9)), dummy, dummy, other,
                               dummy, None) == wiu.WIU_EINVAL
    # the adjoint: the paper's configuration only
    for kw in (dict(vars=1), dict(alpha_h=0.9), dict(weights="z"), dict(split="sw")):
        q = wiu.make_params(**kw)
        assert wiu.lib.wiu_rhs_vjp(ctypes.byref(g), 0, ctypes.byref(q), dummy, dummy, other, ctypes.c_void_p(768),
                                   dummy, None) == wiu.WIU_EINVAL
    bad = wiu.make_params(gamma=1.0)
    assert wiu.lib.wiu_rhs(ctypes.byref(g), 3, ctypes.byref(bad), dummy, dummy, other, dummy, None) == wiu.WIU_EINVAL
    assert wiu.lib.wiu_metrics(ctypes.byref(g), -1, None, dummy, dummy, dummy, dummy, None) == wiu.WIU_EINVAL
    assert wiu.lib.wiu_cfl_dt(ctypes.byref(g), ctypes.byref(p), dummy, dummy, ctypes.c_double(-1.0), dummy, dummy,
                              None) == wiu.WIU_EINVAL
    # several CFL-limited steps: at least one step, a positive CFL number
    for n, c in ((0, 0.5), (-3, 0.5), (2, 0.0)):
        assert wiu.lib.wiu_rk3_steps_cfl(ctypes.byref(g), 3, ctypes.byref(p), dummy, other, ctypes.c_double(c), n,
                                         ctypes.c_void_p(768), ctypes.c_void_p(1024), None) == wiu.WIU_EINVAL
    # several stage-storing steps: at least one step, stages and records required
    for n, st, rc in ((0, dummy, dummy), (2, None, dummy), (2, dummy, None)):
        assert wiu.lib.wiu_rk3_steps_stages(ctypes.byref(g), 3, ctypes.byref(p), dummy, other, ctypes.c_void_p(768),
                                            n, st, rc, ctypes.c_void_p(1024), None) == wiu.WIU_EINVAL
    assert wiu.lib.wiu_strerror(wiu.WIU_EINVAL) == b"invalid argument"


def test_side_rules_are_validated(wiu):
    """Side rules of non-periodic directions must be 0..2 and fixed states
    physical; periodic directions ignore them."""
    g = wiu.make_grid(16, 12, ("transmissive", "transmissive"), sides=("wall", "fixed", 0, 0),
                      fixed=[[1.0, 0.1, 0.0, 2.5], [1.0, 0.0, 0.0, 2.5], [0] * 4, [0] * 4])
    assert wiu.metrics_size(g) > 0
    g.fixed[1][0] = -1.0
    assert wiu.metrics_size(g) == 0
    g = wiu.make_grid(16, 12, ("transmissive", "transmissive"), sides=(0, 0, 3, 0))
    assert wiu.metrics_size(g) == 0
    g = wiu.make_grid(16, 12, ("periodic", "periodic"), (1.0, 1.0), sides=(3, 3, 3, 3))
    assert wiu.metrics_size(g) > 0


def _descs(wiu, blocks):
    """wiu_block array for multi-block grid blocks (offsets left at zero:
    validation does not look at them)."""
    out = (wiu.WiuBlock * len(blocks))()
    for d, b in zip(out, blocks):
        ny, nx = b.x.shape
        d.nx, d.ny, d.bc_x, d.bc_y = nx, ny, 1, 1
        for s in range(4):
            d.side[s], d.nbr[s], d.nbr_side[s] = int(b.sides[s]), int(b.nbr[s]), int(b.nbr_side[s])
            d.shift[s][0], d.shift[s][1] = float(b.shift[s][0]), float(b.shift[s][1])
    return out


def test_block_sets_are_validated(wiu):
    """Interfaces must point back, match in length and lead into blocks at
    least WIU_MB_REACH nodes deep; seam shifts must cancel; a rejected set
    fails on the host before anything is allocated or launched."""
    import numpy as np
    from paper_1810_11103_amd import workloads as W
    g = W.periodic_grid(60, 40, A=0.2, seed=1)
    P = wiu.make_params()
    plan = ctypes.c_void_p()

    def ok(blocks):
        d = _descs(wiu, blocks)
        n = wiu.lib.wiu_blocks_metrics_work_size(d, len(blocks), 3)
        return n > 0

    good, _ = W.cut_blocks(g, [], icuts=[30], turns=[1, 2])
    assert ok(good)
    cases = []
    b, _ = W.cut_blocks(g, [], icuts=[30], turns=[1, 2]); b[0].nbr_side[0] = (b[0].nbr_side[0] + 1) % 4; cases.append(b)
    b, _ = W.cut_blocks(g, [], icuts=[30], turns=[1, 2]); b[1].shift = np.ones((4, 2)); cases.append(b)
    b, _ = W.cut_blocks(g, [], icuts=[30], turns=[1, 2]); b[1].nbr = [5, 5, 5, 5]; cases.append(b)
    b, _ = W.cut_blocks(g, [], icuts=[50], turns=[0, 0]); cases.append(b)  # neighbour 10 nodes deep
    for b in cases:
        assert not ok(b)
        d = _descs(wiu, b)
        rc = wiu.lib.wiu_batched_plan(d, len(b), 3, ctypes.byref(P), 0, 0, ctypes.c_void_p(8), ctypes.c_void_p(8),
                                      ctypes.byref(plan))
        assert rc == wiu.WIU_EINVAL and not plan.value


def test_3d_grids_and_options_are_validated(wiu):
    """3-D grids need positive sizes (two nodes in transmissive directions,
    positive periods in periodic ones); out-of-range options are rejected on
    the host."""
    g = wiu.make_grid3(16, 12, 10, ("periodic", "transmissive", "periodic"), (1.0, 0.0, 1.0))
    assert wiu.lib.wiu3_metrics_size(ctypes.byref(g)) == (19 * 24 * 20 * 18 + 8) * 8
    assert wiu.lib.wiu3_workspace_bytes(ctypes.byref(g)) > 0
    for bad in (wiu.make_grid3(0, 12, 10), wiu.make_grid3(16, 1, 10, (1, 1, 1)),
                wiu.make_grid3(16, 12, 10, ("periodic",) * 3, (1.0, 0.0, 1.0))):
        assert wiu.lib.wiu3_metrics_size(ctypes.byref(bad)) == 0
    dummy = ctypes.c_void_p(8)
    # options as in 2-D: alpha_h only for one-midpoint schemes, enums in range
    for scheme, opts in ((3, dict(split=3)), (3, dict(vars=3)), (3, dict(alpha_h=0.9))):
        P = wiu.make_params(**opts)
        rc = wiu.lib.wiu3_rhs(ctypes.byref(g), scheme, ctypes.byref(P), dummy, dummy, dummy, dummy, None)
        assert rc == wiu.WIU_EINVAL
    # side rules of bounded directions: 0..2, fixed states physical
    bad = wiu.make_grid3(16, 12, 10, ("periodic", "transmissive", "periodic"), (1.0, 0.0, 1.0),
                         sides=(0, 0, 3, 0, 0, 0))
    assert wiu.lib.wiu3_metrics_size(ctypes.byref(bad)) == 0
    fx = [[0.0] * 5 for _ in range(6)]
    fx[3] = [-1.0, 0.0, 0.0, 0.0, 2.5]
    bad = wiu.make_grid3(16, 12, 10, ("periodic", "transmissive", "periodic"), (1.0, 0.0, 1.0),
                         sides=(0, 0, 0, 2, 0, 0), fixed=fx)
    assert wiu.lib.wiu3_metrics_size(ctypes.byref(bad)) == 0
    ok = wiu.make_grid3(16, 12, 10, ("periodic", "transmissive", "periodic"), (1.0, 0.0, 1.0),
                        sides=(3, 3, 1, 0, 3, 3))  # periodic directions ignore their sides
    assert wiu.lib.wiu3_metrics_size(ctypes.byref(ok)) > 0
    # the Jacobian form is 5 or 6
    assert wiu.lib.wiu3_metrics(ctypes.byref(g), 3, 4, None, dummy, dummy, dummy, dummy, dummy, None) == wiu.WIU_EINVAL
    P = wiu.make_params(alpha_h=0.9)
    assert wiu.lib.wiu3_metrics(ctypes.byref(g), 3, 5, ctypes.byref(P), dummy, dummy, dummy, dummy, dummy,
                                None) == wiu.WIU_EINVAL
    P = wiu.make_params()
    assert wiu.lib.wiu3_rhs(ctypes.byref(g), 8, ctypes.byref(P), dummy, dummy, dummy, dummy, None) == wiu.WIU_EINVAL
    # the combined CFL step needs a positive CFL number and the step's own checks
    for cfl, scheme in ((0.0, 3), (-0.5, 3), (float("nan"), 3), (0.5, 8)):
        assert wiu.lib.wiu3_rk3_step_cfl(ctypes.byref(g), scheme, ctypes.byref(P), dummy, dummy, cfl, dummy, dummy,
                                         None) == wiu.WIU_EINVAL
    # several steps per call: also at least one step
    for cfl, scheme, n in ((0.0, 3, 2), (float("nan"), 3, 2), (0.5, 8, 2), (0.5, 3, 0), (0.5, 3, -1)):
        assert wiu.lib.wiu3_rk3_steps_cfl(ctypes.byref(g), scheme, ctypes.byref(P), dummy, dummy, cfl, n, dummy,
                                          dummy, None) == wiu.WIU_EINVAL
