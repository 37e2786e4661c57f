"""The allocation-free RK3 step (wiu_rk3_step_noalloc) against the
workspace entry point wiu_rk3_step, through the C ABI: the same kernels on
the same inputs, so the states must agree bit for bit; two calls in a row,
the second on a smaller grid (the static scratch keeps the first call's
contents), and each against the oracle's RK3 step at the parity bar of the
step tests (1e-11 of the step's change, per component).  Host-side
rejection of grids beyond the scratch needs no GPU."""
import ctypes
import sys

import numpy as np
import pytest

from paper_1810_11103_amd import workloads as W


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def wiu():
    from paper_1810_11103_amd import wenoiu
    return wenoiu


def test_grid_beyond_scratch_rejected_on_host(wiu):
    p = wiu.make_params()
    small = wiu.make_grid(1024, 1024, ("periodic", "periodic"), (1.0, 1.0))
    big = wiu.make_grid(1200, 1024, ("periodic", "periodic"), (1.0, 1.0))
    limit = 72 << 20
    assert 0 < wiu.noalloc_bytes(small) <= limit < wiu.noalloc_bytes(big)
    d = ctypes.c_void_p(256)
    assert wiu.lib.wiu_rk3_step_noalloc(ctypes.byref(big), 3, ctypes.byref(p), d, d, d, d, None) == wiu.WIU_EINVAL
    # null status pointer, bad scheme
    assert wiu.lib.wiu_rk3_step_noalloc(ctypes.byref(small), 3, ctypes.byref(p), d, d, d, None, None) == wiu.WIU_EINVAL
    assert wiu.lib.wiu_rk3_step_noalloc(ctypes.byref(small), 9, ctypes.byref(p), d, d, d, d, None) == wiu.WIU_EINVAL


def _case(kind):
    if kind == "vortex":
        g = W.periodic_grid(300, 260, (0, 10, 0, 10), A=0.2, seed=11)
        return g, W.vortex_periodic_state(g), "5-2MP"
    g = W.bounded_grid(130, 97, (0, 1, 0, 1), A=0.2, seed=12)
    return g, W.riemann_state(g), "3-1MP"


@pytest.mark.gpu
def test_noalloc_step_equals_workspace_step(wiu, orc):
    import torch
    for kind in ("vortex", "riemann"):  # the second call is on a smaller grid
        g, U0, s = _case(kind)
        say("noalloc step:", kind, s, g.shape)
        sol = wiu.Solver(g.x, g.y, s, g.bc, g.period)
        M = orc.metrics(s, g.x, g.y, g.bc, g.period)
        dt = 0.8 * orc.cfl_dt(U0, M, 0.5)
        Ua = torch.as_tensor(U0).cuda().contiguous()
        Ub = Ua.clone()
        sol.rk3_step(Ua, dt)
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        wiu.rk3_step_noalloc(sol.grid, s, sol.params, Ub, sol.M, sol.dt, st)
        torch.cuda.synchronize()
        a, b = Ua.cpu().numpy(), Ub.cpu().numpy()
        assert np.array_equal(a, b), f"{kind}: max diff {np.abs(a - b).max():.3e}"
        assert int(st.item()) == 0
        assert sol.status() == 0
        ref = orc.rk3_step(s, U0, M, dt, g.bc)
        for c in range(4):
            d_ref = ref[c] - U0[c]
            assert np.abs((b[c] - U0[c]) - d_ref).max() <= 1e-11 * np.abs(d_ref).max(), (kind, c)


@pytest.mark.gpu
def test_noalloc_status_latches_nonphysical_state(wiu):
    """A negative density is reported through the caller's status word."""
    import torch
    g, U0, s = _case("riemann")
    U0 = U0.copy()
    U0[0, 40, 50] = -1.0
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period)
    sol.dt.fill_(1e-5)
    U = torch.as_tensor(U0).cuda().contiguous()
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    wiu.rk3_step_noalloc(sol.grid, s, sol.params, U, sol.M, sol.dt, st)
    torch.cuda.synchronize()
    assert int(st.item()) & wiu.ST_NONPHYS
