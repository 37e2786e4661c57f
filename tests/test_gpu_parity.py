"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bar (written per test): metrics and line eigenvalues within 1e-13 of the
plane's magnitude; rhs within 1e-12 normwise per conservative component
(max |gpu - oracle| <= 1e-12 max |oracle|); free-stream preservation
max |dU/dt| < 1e-11 for uniform flow on randomized grids."""
import sys

import numpy as np
import pytest

from paper_1810_11103_amd import workloads as W

pytestmark = pytest.mark.gpu

SCHEMES = ["3-1MP", "3-2MP", "5-1MP", "5-2MP", "7-1MP", "7-2MP", "7-4MP", "7-6MP"]
G = 4


@pytest.fixture(scope="module")
def wiu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1810_11103_amd import wenoiu
    return wenoiu


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).cuda()


def _host(t):
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def normwise(gpu, ref):
    """max_ij |gpu - ref| / max_ij |ref| per conservative component."""
    return np.array([np.abs(gpu[c] - ref[c]).max() / max(np.abs(ref[c]).max(), 1e-300) for c in range(4)])


def make_case(kind, nx, ny, seed=0):
    if kind == "vortex":
        g = W.periodic_grid(nx, ny, (0, 10, 0, 10), A=0.2, seed=seed)
        U = W.vortex_periodic_state(g)
    elif kind == "smooth":
        g = W.periodic_grid(nx, ny, (0, 10, 0, 10), A=0.2, seed=seed)
        U = W.random_smooth_state(g, seed=seed)
    elif kind == "riemann":
        g = W.bounded_grid(nx, ny, (0, 1, 0, 1), A=0.2, seed=seed)
        U = W.riemann_state(g)
    elif kind == "strip":
        g = W.strip_grid(nx)
        U = W.sod_state(g)
    else:
        raise ValueError(kind)
    return g, U


CASES = [("vortex", 300, 70), ("smooth", 131, 67), ("riemann", 260, 90), ("strip", 203, 1)]


@pytest.mark.parametrize("s", SCHEMES)
@pytest.mark.parametrize("kind,nx,ny", CASES)
def test_metrics_parity(orc, wiu, s, kind, nx, ny):
    say("metrics parity", s, kind, nx, ny)
    g, _ = make_case(kind, nx, ny, seed=11)
    Mo = orc.metrics(s, g.x, g.y, g.bc, g.period)
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period)
    Mg = _host(sol.planes())
    assert sol.status() == 0
    for p in range(9):
        scale = np.abs(Mo[p]).max()
        err = np.abs(Mg[p] - Mo[p]).max()
        assert err <= 1e-13 * scale, (p, err, scale)


@pytest.mark.parametrize("kind,nx,ny", CASES)
def test_line_eigenvalue_parity(orc, wiu, kind, nx, ny):
    say("lambda parity", kind, nx, ny)
    g, U = make_case(kind, nx, ny, seed=3)
    s = "5-2MP"
    Mo = orc.metrics(s, g.x, g.y, g.bc, g.period)
    _, lx, le = orc.rhs(s, U, Mo, g.bc, return_lambda=True)
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period)
    gx, ge = sol.line_eigenvalues(_dev(U))
    np.testing.assert_allclose(_host(gx), lx, rtol=1e-13)
    np.testing.assert_allclose(_host(ge), le, rtol=1e-13)


def _gpu_rhs_with_metrics(wiu, g, s, U, M_planes):
    """rhs on the GPU with externally supplied metric planes (tagged)."""
    import torch
    grid = wiu.make_grid(g.x.shape[1], g.x.shape[0], g.bc, g.period)
    M = wiu.metrics_tensor(grid)
    H, Wd = grid.ny + 2 * G, grid.nx + 2 * G
    M[: 9 * H * Wd] = _dev(M_planes).reshape(-1)
    wiu.set_metrics_tag(grid, s, M)
    ws = wiu.workspace(grid)
    Ud = _dev(U)
    out = torch.empty_like(Ud)
    wiu.rhs(grid, s, wiu.make_params(), Ud, M, out, ws)
    st = wiu.status(ws)
    return _host(out), st


@pytest.mark.parametrize("s", SCHEMES)
@pytest.mark.parametrize("kind,nx,ny", CASES)
def test_rhs_parity_same_metrics(orc, wiu, s, kind, nx, ny):
    """rhs alone: both sides consume the oracle's metric planes."""
    say("rhs parity (oracle metrics)", s, kind, nx, ny)
    g, U = make_case(kind, nx, ny, seed=5)
    Mo = orc.metrics(s, g.x, g.y, g.bc, g.period)
    ref = orc.rhs(s, U, Mo, g.bc)
    out, st = _gpu_rhs_with_metrics(wiu, g, s, U, Mo)
    assert st == 0
    err = normwise(out, ref)
    assert np.all(err <= 1e-12), err


@pytest.mark.parametrize("s", SCHEMES)
@pytest.mark.parametrize("kind,nx,ny", CASES)
def test_rhs_parity_full_path(orc, wiu, s, kind, nx, ny):
    """metrics + rhs on the GPU against metrics + rhs in the oracle."""
    say("rhs parity (full path)", s, kind, nx, ny)
    g, U = make_case(kind, nx, ny, seed=7)
    Mo = orc.metrics(s, g.x, g.y, g.bc, g.period)
    ref = orc.rhs(s, U, Mo, g.bc)
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period)
    out = _host(sol.rhs(_dev(U)))
    assert sol.status() == 0
    err = normwise(out, ref)
    assert np.all(err <= 1e-12), err


@pytest.mark.parametrize("s", SCHEMES)
@pytest.mark.parametrize("n", [64, 128, 256, 512])
def test_free_stream_preservation_on_gpu(wiu, s, n):
    """Sec. 5.2 on the GPU: uniform Mach-0.5 flow on the randomized periodic
    [0,10]^2 grid (A = 0.2) keeps max |dU/dt| < 1e-11."""
    say("FSP", s, n)
    g, U = W.fsp_problem(n, A=0.2)
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period)
    d = _host(sol.rhs(_dev(U)))
    assert sol.status() == 0
    assert np.abs(d).max() < 1e-11, np.abs(d).max()


@pytest.mark.parametrize("s", SCHEMES)
def test_rk3_step_parity(orc, wiu, s):
    say("rk3 parity", s)
    g, U = make_case("vortex", 160, 96, seed=2)
    Mo = orc.metrics(s, g.x, g.y, g.bc, g.period)
    dt = orc.cfl_dt(U, Mo, 0.5)
    ref = orc.rk3_step(s, U, Mo, dt, g.bc)
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period)
    Ud = _dev(U)
    sol.cfl_dt(Ud, 0.5)
    assert float(sol.dt.item()) == pytest.approx(dt, rel=1e-13)
    sol.dt.fill_(dt)
    sol.rk3_step(Ud)
    out = _host(Ud)
    assert sol.status() == 0
    err = normwise(out - U, ref - U)
    assert np.all(err <= 1e-11), err


def test_rk3_steps_track_oracle_on_sod_strip(orc, wiu):
    """20 CFL-driven RK3 steps of the Sod strip stay with the oracle (the
    state is re-synchronised each step, so only one step's rounding counts)."""
    g = W.strip_grid(200)
    U = W.sod_state(g)
    s = "5-2MP"
    Mo = orc.metrics(s, g.x, g.y, g.bc, g.period)
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period)
    for k in range(20):
        dt = orc.cfl_dt(U, Mo, 0.5)
        ref = orc.rk3_step(s, U, Mo, dt, g.bc)
        Ud = _dev(U)
        sol.rk3_step(Ud, dt)
        out = _host(Ud)
        err = normwise(out - U, ref - U)
        assert np.all(err <= 1e-11), (k, err)
        U = ref
    assert sol.status() == 0


def test_status_flags(orc, wiu):
    import torch
    g, U = make_case("vortex", 64, 64, seed=1)
    sol = wiu.Solver(g.x, g.y, "5-2MP", g.bc, g.period)
    assert sol.status() == 0
    # non-physical state: negative pressure at one node
    Ub = U.copy()
    Ub[3, 10, 10] = 0.1 * Ub[3, 10, 10] - 5.0
    sol.rhs(_dev(Ub))
    assert sol.status() & wiu.ST_NONPHYS
    # metrics of another scheme: flagged, nothing written
    other = wiu.Solver(g.x, g.y, "3-1MP", g.bc, g.period)
    out = torch.full((4, 64, 64), 7.0, dtype=torch.float64, device="cuda")
    wiu.rhs(sol.grid, "5-2MP", sol.params, _dev(U), other.M, out, sol.ws)
    assert sol.status() & wiu.ST_SCHEME
    assert float(out.min()) == 7.0 and float(out.max()) == 7.0
    # folded grid (node displaced past its neighbour): J^{-1} <= 0 flagged
    gf = W.periodic_grid(32, 32, (0, 10, 0, 10))
    x = gf.x.copy()
    x[10, 10] += 1.6 * (10 / 32)
    bad = wiu.Solver(x, gf.y, "5-2MP", gf.bc, gf.period)
    assert bad.status() & wiu.ST_JACOBIAN


def test_rhs_is_deterministic(wiu):
    g, U = make_case("riemann", 300, 200, seed=8)
    sol = wiu.Solver(g.x, g.y, "5-2MP", g.bc, g.period)
    Ud = _dev(U)
    a = _host(sol.rhs(Ud))
    b = _host(sol.rhs(Ud))
    assert np.array_equal(a, b)


def test_full_size_riemann_parity(orc, wiu):
    """The throughput workload itself (2048^2 randomized Riemann grid, 5-2MP,
    transmissive): GPU rhs and one RK3 step against the oracle, everywhere."""
    s = "5-2MP"
    say("full-size parity: metrics")
    g, U = W.riemann_problem(2048)
    Mo = orc.metrics(s, g.x, g.y, g.bc, g.period)
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period)
    Mg = _host(sol.planes())
    for p in range(9):
        assert np.abs(Mg[p] - Mo[p]).max() <= 1e-13 * np.abs(Mo[p]).max(), p
    say("full-size parity: rhs")
    ref = orc.rhs(s, U, Mo, g.bc)
    Ud = _dev(U)
    out = _host(sol.rhs(Ud))
    err = normwise(out, ref)
    assert np.all(err <= 1e-12), err
    say("full-size parity: rk3 step")
    dt = orc.cfl_dt(U, Mo, 0.5)
    refs = orc.rk3_step(s, U, Mo, dt, g.bc)
    sol.rk3_step(Ud, dt)
    outs = _host(Ud)
    err = normwise(outs - U, refs - U)
    assert np.all(err <= 1e-11), err
    assert sol.status() == 0


def test_full_size_steps_cfl_equal_single_steps(wiu):
    """The timed configuration: several CFL-limited steps per call on the
    2048^2 randomized Riemann workload (A = 0.2, seed 2048), bitwise equal to
    one wiu_rk3_step_cfl call per step, states and time steps."""
    say("full-size: rk3_steps_cfl against single steps")
    g, U = W.riemann_problem(2048, A=0.2, seed=2048)
    sol = wiu.Solver(g.x, g.y, "5-2MP", g.bc, g.period)
    Ua, Ub = _dev(U), _dev(U)
    dts = []
    for _ in range(3):
        sol.rk3_step_cfl(Ua, 0.5)
        dts.append(float(sol.dt.item()))
    got = _host(sol.rk3_steps_cfl(Ub, 0.5, 3)).tolist()
    assert sol.status() == 0
    assert got == dts
    assert np.array_equal(_host(Ua), _host(Ub))


def test_tile_shapes_give_identical_results(wiu):
    """Every compiled tile shape of both sweeps gives bitwise the same rhs
    (each item is computed by the same code whatever the tiling)."""
    g, U = make_case("riemann", 301, 203, seed=4)
    Ud = _dev(U)
    ref = None
    saved = (wiu.get_tuning(0), wiu.get_tuning(1))
    try:
        for s in SCHEMES:
            sol = wiu.Solver(g.x, g.y, s, g.bc, g.period)
            ref = None
            for vx in range(wiu.tuning_variants(0)):
                for ve in range(wiu.tuning_variants(1)):
                    wiu.set_tuning(0, vx)
                    wiu.set_tuning(1, ve)
                    out = _host(sol.rhs(Ud))
                    if ref is None:
                        ref = out
                    else:
                        assert np.array_equal(out, ref), (s, vx, ve)
            assert sol.status() == 0
    finally:
        wiu.set_tuning(0, saved[0])
        wiu.set_tuning(1, saved[1])


@pytest.mark.parametrize("s", SCHEMES)
def test_rk3_step_parity_ragged_transmissive(orc, wiu, s):
    """RK3 step on a ragged transmissive Riemann grid: stages 2 and 3 take
    their line eigenvalues from the maxima the previous stage's eta sweep
    accumulated, so wrong maxima would show here against the oracle."""
    say("rk3 parity ragged riemann", s)
    g, U = make_case("riemann", 260, 90, seed=5)
    Mo = orc.metrics(s, g.x, g.y, g.bc, g.period)
    dt = orc.cfl_dt(U, Mo, 0.5)
    ref = orc.rk3_step(s, U, Mo, dt, g.bc)
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period)
    Ud = _dev(U)
    sol.rk3_step(Ud, dt)
    out = _host(Ud)
    assert sol.status() == 0
    err = normwise(out - U, ref - U)
    assert np.all(err <= 1e-11), err


def test_rk3_step_cfl_equals_cfl_dt_then_step(wiu):
    """The combined entry point gives bitwise the dt and state of wiu_cfl_dt
    followed by wiu_rk3_step."""
    g, U = make_case("riemann", 301, 203, seed=6)
    sol = wiu.Solver(g.x, g.y, "5-2MP", g.bc, g.period)
    Ua, Ub = _dev(U), _dev(U)
    for _ in range(3):
        sol.cfl_dt(Ua, 0.5)
        dta = float(sol.dt.item())
        sol.rk3_step(Ua)
        sol.rk3_step_cfl(Ub, 0.5)
        assert float(sol.dt.item()) == dta
        assert np.array_equal(_host(Ua), _host(Ub))
    assert sol.status() == 0


STEPS_CASES = [
    ("5-2MP", "riemann", None, {}),
    ("3-1MP", "vortex", None, {}),
    ("7-4MP", "riemann", None, {}),
    ("5-2MP", "riemann", ("wall", "transmissive", "wall", "wall"), {}),
    ("5-1MP", "riemann", None, dict(vars="conservative", alpha_h=0.8)),
]


@pytest.mark.parametrize("s,kind,sides,opts", STEPS_CASES)
def test_rk3_steps_cfl_equals_single_steps(wiu, s, kind, sides, opts):
    """Several CFL-limited steps in one call give bitwise the states and time
    steps of as many wiu_rk3_step_cfl calls: the line eigenvalues and CFL
    maximum that the last stage's eta sweep accumulates for the next step
    equal those of the separate maxima pass."""
    say("rk3_steps_cfl vs single steps", s, kind, sides, opts)
    g, U = make_case(kind, 301, 203, seed=8) if kind == "riemann" else make_case(kind, 300, 70, seed=8)
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period, params=wiu.make_params(**opts), sides=sides)
    Ua, Ub = _dev(U), _dev(U)
    dts = []
    for _ in range(4):
        sol.rk3_step_cfl(Ua, 0.5)
        dts.append(float(sol.dt.item()))
    got = _host(sol.rk3_steps_cfl(Ub, 0.5, 4)).tolist()
    assert sol.status() == 0
    assert got == dts
    assert np.array_equal(_host(Ua), _host(Ub))
    one = sol.rk3_steps_cfl(Ub, 0.5, 1)  # a single step: the separate pass only
    sol.rk3_step_cfl(Ua, 0.5)
    assert float(one[0].item()) == float(sol.dt.item())
    assert np.array_equal(_host(Ua), _host(Ub))



DEGENERATE_STEPS = [("strip", 203, 1), ("smooth", 7, 5), ("bounded", 3, 2), ("periodic1", 9, 1)]



def test_steps_cfl_replayed_from_a_captured_graph(wiu):
    """Several CFL steps per call captured once in a HIP graph (the library
    clears its maxima with fill kernels, never memsets) and replayed three
    times, with eager steps and synchronisations between the replays: every
    replay gives the eager call's states and time steps bit for bit."""
    import torch
    say("rk3_steps_cfl graph replays")
    g, U = make_case("riemann", 301, 203, seed=8)
    sol = wiu.Solver(g.x, g.y, "5-2MP", g.bc, g.period)
    U0 = _dev(U)
    K = 4
    Ue = U0.clone()
    dte = sol.rk3_steps_cfl(Ue, 0.5, K)
    torch.cuda.synchronize()
    Ug = U0.clone()
    dtg = torch.empty(K, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # one call before capture, as torch asks
        sol.rk3_steps_cfl(Ug, 0.5, K, dtg)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        sol.rk3_steps_cfl(Ug, 0.5, K, dtg)
    for r in range(3):
        Ug.copy_(U0)
        dtg.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(Ug, Ue), r
        assert torch.equal(dtg, dte), r
        Uw = U0.clone()  # eager work between the replays
        sol.rk3_steps_cfl(Uw, 0.5, 2)
        torch.cuda.synchronize()
    assert sol.status() == 0

@pytest.mark.parametrize("kind,nx,ny", DEGENERATE_STEPS)
def test_rk3_steps_cfl_degenerate_shapes(wiu, kind, nx, ny):
    """Several steps per call on a one-row strip, a one-node periodic
    direction and grids of a few nodes, where the per-line CFL partials
    cover only a handful of lines: states and time steps equal those of
    single wiu_rk3_step_cfl calls, bit for bit."""
    say("rk3_steps_cfl degenerate", kind, nx, ny)
    if kind == "bounded":
        g = W.bounded_grid(nx, ny, (0, 1, 0, 1), A=0.1, seed=4, layers=1)
        U = W.random_smooth_state(g, seed=4)
    elif kind == "periodic1":
        g = W.periodic_grid(nx, ny, (0, 10, 0, 10), A=0.0, seed=3)
        U = W.random_smooth_state(g, seed=3)
    else:
        g, U = make_case(kind, nx, ny, seed=4)
    a = wiu.Solver(g.x, g.y, "5-2MP", g.bc, g.period)
    b = wiu.Solver(g.x, g.y, "5-2MP", g.bc, g.period)
    Ua, Ub = _dev(U), _dev(U)
    dts = []
    for _ in range(3):
        a.rk3_step_cfl(Ua, 0.5)
        dts.append(float(a.dt.item()))
    got = _host(b.rk3_steps_cfl(Ub, 0.5, 3)).tolist()
    assert a.status() == 0 and b.status() == 0
    assert got == dts
    assert np.array_equal(_host(Ua), _host(Ub))

def test_rk3_steps_cfl_across_tile_shapes(wiu):
    """The CFL maximum reduced in the eta tiles does not depend on their
    lane layout (2 to 16 lines per wave): same steps for every eta shape."""
    g, U = make_case("riemann", 301, 203, seed=9)
    saved = wiu.get_tuning(1)
    try:
        sol = wiu.Solver(g.x, g.y, "5-2MP", g.bc, g.period)
        ref = None
        for ve in range(wiu.tuning_variants(1)):
            wiu.set_tuning(1, ve)
            Ud = _dev(U)
            dts = _host(sol.rk3_steps_cfl(Ud, 0.5, 3))
            out = (_host(Ud), dts)
            if ref is None:
                ref = out
            else:
                assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), ve
        assert sol.status() == 0
    finally:
        wiu.set_tuning(1, saved)


def test_rk3_steps_cfl_track_oracle(orc, wiu):
    """Three CFL-limited steps in one call against the oracle's CFL rule and
    RK3 step applied three times (ragged transmissive Riemann grid)."""
    g, U = make_case("riemann", 260, 90, seed=10)
    Mo = orc.metrics("5-2MP", g.x, g.y, g.bc, g.period)
    ref = U.copy()
    ref_dts = []
    for _ in range(3):
        dt = orc.cfl_dt(ref, Mo, 0.5)
        ref_dts.append(dt)
        ref = orc.rk3_step("5-2MP", ref, Mo, dt, g.bc)
    sol = wiu.Solver(g.x, g.y, "5-2MP", g.bc, g.period)
    Ud = _dev(U)
    dts = _host(sol.rk3_steps_cfl(Ud, 0.5, 3))
    assert sol.status() == 0
    assert np.allclose(dts, ref_dts, rtol=1e-12, atol=0.0), (dts, ref_dts)
    err = normwise(_host(Ud) - U, ref - U)
    assert np.all(err <= 1e-11), err


def test_rk3_step_identical_across_tile_shapes(wiu):
    """RK3 steps are bitwise the same for every pair of tile shapes: the eta
    tiles reduce the next stage's line maxima over their own lane layout
    (2 to 16 lines per wave), and maxima do not depend on the order."""
    g, U = make_case("riemann", 301, 203, seed=7)
    saved = (wiu.get_tuning(0), wiu.get_tuning(1))
    try:
        for s in ("3-1MP", "5-2MP", "7-6MP"):
            sol = wiu.Solver(g.x, g.y, s, g.bc, g.period)
            ref = None
            for vx in range(wiu.tuning_variants(0)):
                for ve in range(wiu.tuning_variants(1)):
                    wiu.set_tuning(0, vx)
                    wiu.set_tuning(1, ve)
                    Ud = _dev(U)
                    sol.rk3_step(Ud, 2e-4)
                    sol.rk3_step(Ud, 2e-4)
                    out = _host(Ud)
                    if ref is None:
                        ref = out
                    else:
                        assert np.array_equal(out, ref), (s, vx, ve)
            assert sol.status() == 0
    finally:
        wiu.set_tuning(0, saved[0])
        wiu.set_tuning(1, saved[1])


def test_adjoint_rejects_seventh_order(wiu):
    """The adjoint entry points cover the third- and fifth-order schemes and
    reject the seventh-order ones with WIU_EINVAL (no silent result)."""
    import torch
    g, U = make_case("smooth", 64, 48, seed=1)
    sol = wiu.Solver(g.x, g.y, "7-2MP", g.bc, g.period)
    Ud = _dev(U)
    with pytest.raises(RuntimeError):
        sol.rhs_vjp(Ud, torch.ones_like(Ud))
