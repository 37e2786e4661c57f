"""GPU parity of multi-block grids coupled through interfaces.

The paper motivates multi-block grids (Sec. 1) but defines no coupling; the
library's rule (lines continue across an interface: states, coordinates,
and each line's Lax-Friedrichs eigenvalue of Sec. 2.3) is implemented by
wiu_blocks_metrics and the batched plan with interface sides, and compared
here with the oracle's multi-block grids on grids cut into blocks whose
index frames are turned by multiples of 90 degrees (periodic grids with
seams; bounded grids with wall, fixed and transmissive sides).

Bar, as for single grids: metrics within 1e-13 of each plane's magnitude,
time steps within 1e-13, RK3 increments within 1e-11 normwise per
component over the whole grid; graph replays equal eager stepping bit for
bit."""
import sys

import numpy as np
import pytest

from paper_1810_11103_amd import workloads as W
from test_gpu_parity import normwise

pytestmark = pytest.mark.gpu
G = 4


@pytest.fixture(scope="module")
def wiu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1810_11103_amd import wenoiu
    return wenoiu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


FIXED = np.array([[1.2, 0.3, -0.1, 2.9], [0.9, 0.1, 0.0, 2.4], [1.0, 0.0, 0.2, 2.6], [1.1, -0.2, 0.1, 2.7]])

# (grid kind, nx, ny, icuts, jcuts, turns, sides): several tiles per block
# along both directions and ragged tails
CONFIGS = {
    "periodic4": ("periodic", 300, 200, [130], [90], [0, 1, 2, 3], None),
    "periodic6": ("periodic", 300, 200, [130, 210], [90], [3, 0, 2, 1, 1, 2], None),
    "bounded6": ("bounded", 300, 200, [130, 210], [90], [1, 2, 0, 3, 2, 1], ("wall", "fixed", "wall", "transmissive")),
    "strip3": ("bounded", 260, 40, [90, 170], [], [2, 1, 3], ("fixed", "transmissive", "wall", "wall")),
}


def make(name, state="smooth", seed=7):
    kind, nx, ny, ic, jc, turns, sides = CONFIGS[name]
    if kind == "periodic":
        g = W.periodic_grid(nx, ny, box=(0.0, nx / 20.0, 0.0, ny / 20.0), A=0.3, seed=seed)
    else:
        g = W.bounded_grid(nx, ny, box=(0.0, nx / 20.0, 0.0, ny / 20.0), A=0.3, seed=seed)
    U = W.random_smooth_state(g, seed=seed, amp=0.2) if state == "smooth" else W.riemann_state(g)
    kw = {} if sides is None else dict(sides=sides, fixed=FIXED)
    blocks, (Ub,) = W.cut_blocks(g, [U], icuts=ic, jcuts=jc, turns=turns, **kw)
    return g, U, blocks, Ub


def mb_normwise(outs, refs):
    """Per component: max |out - ref| over all blocks relative to max |ref|
    over all blocks (as for one grid: a block inside a uniform region has a
    reference increment of pure round-off, so a per-block ratio means
    nothing there)."""
    num = np.max([[np.abs(o[q] - r[q]).max() for q in range(4)] for o, r in zip(outs, refs)], axis=0)
    den = np.max([[np.abs(r[q]).max() for q in range(4)] for r in refs], axis=0)
    return num / den


def plan_for(wiu, blocks, Ub, s, params=None):
    import torch
    plan = wiu.BatchedPlan(blocks, s, params=params)
    for b, u in enumerate(Ub):
        plan.state(b).copy_(torch.as_tensor(u))
    return plan


def gpu_metrics(plan, b):
    ny, nx = plan.shapes[b]
    M = plan.metric_array(b).cpu().numpy()
    return M[:9 * (ny + 2 * G) * (nx + 2 * G)].reshape(9, ny + 2 * G, nx + 2 * G)


@pytest.mark.parametrize("s", ["3-1MP", "5-2MP", "7-2MP"])
@pytest.mark.parametrize("name", ["periodic6", "bounded6"])
def test_coupled_metrics_parity(orc, wiu, s, name):
    say("multi-block metrics", s, name)
    g, U, blocks, Ub = make(name)
    Mo = orc.mb_metrics(s, blocks)
    plan = plan_for(wiu, blocks, Ub, s)
    for b in range(len(blocks)):
        Mg = gpu_metrics(plan, b)
        for p in range(9):
            assert np.abs(Mg[p] - Mo[b][p]).max() <= 1e-13 * np.abs(Mo[b][p]).max(), (b, p)
    plan.close()


@pytest.mark.parametrize("s", ["3-2MP", "5-2MP", "7-1MP"])
@pytest.mark.parametrize("name", list(CONFIGS))
@pytest.mark.parametrize("state", ["smooth", "riemann"])
def test_rk3_step_parity(orc, wiu, s, name, state):
    say("multi-block rk3", s, name, state)
    g, U, blocks, Ub = make(name, state)
    Mo = orc.mb_metrics(s, blocks)
    plan = plan_for(wiu, blocks, Ub, s)
    plan.cfl_dt(0.5)
    dts = plan.get_dt()
    ref_dt = orc.mb_cfl_dt(blocks, Ub, Mo, 0.5)
    assert np.allclose(dts, ref_dt, rtol=1e-13, atol=0.0), (dts, ref_dt)
    # blocks joined by interfaces share one step
    assert np.all(dts == dts[0])
    ref = orc.mb_rk3_step(s, blocks, Ub, Mo, dts)
    plan.step(graph=False)
    assert plan.status() == 0
    outs = [plan.state(b).cpu().numpy() - Ub[b] for b in range(len(blocks))]
    err = mb_normwise(outs, [r - u for r, u in zip(ref, Ub)])
    assert np.all(err <= 1e-11), err
    plan.close()


@pytest.mark.parametrize("s,opts", [("5-1MP", dict(vars="primitive", alpha_h=0.9)),
                                    ("5-2MP", dict(weights="z", split="vl")),
                                    ("7-4MP", dict(vars="conservative"))])
def test_rk3_step_parity_with_options(orc, wiu, s, opts):
    say("multi-block rk3 options", s, opts)
    g, U, blocks, Ub = make("periodic6", "riemann", seed=3)
    Mo = orc.mb_metrics(s, blocks, alpha_h=opts.get("alpha_h", 1.0))
    plan = plan_for(wiu, blocks, Ub, s, params=wiu.make_params(**opts))
    plan.cfl_dt(0.4)
    dts = plan.get_dt()
    ref = orc.mb_rk3_step(s, blocks, Ub, Mo, dts, **opts)
    plan.step(graph=False)
    assert plan.status() == 0
    outs = [plan.state(b).cpu().numpy() - Ub[b] for b in range(len(blocks))]
    err = mb_normwise(outs, [r - u for r, u in zip(ref, Ub)])
    assert np.all(err <= 1e-11), err
    plan.close()


def test_graph_replays_equal_eager_steps(wiu):
    import torch
    g, U, blocks, Ub = make("bounded6", "riemann")
    a = plan_for(wiu, blocks, Ub, "5-2MP")
    b = plan_for(wiu, blocks, Ub, "5-2MP")
    a.cfl_dt(0.5)
    b.set_dt(a.get_dt())
    for k in range(3):
        a.step(graph=False)
        b.step(graph=True)
        torch.cuda.synchronize()
        for i in range(len(blocks)):
            assert torch.equal(a.state(i), b.state(i)), (k, i)
    assert a.status() == 0 and b.status() == 0
    a.close()
    b.close()


def test_cut_grid_equals_single_grid_on_gpu(wiu):
    """The multi-block step of a cut periodic grid and the single-grid step
    of the uncut grid, both on the GPU."""
    import torch
    from test_gpu_parity import _dev, _host
    g, U, blocks, Ub = make("periodic4", "riemann", seed=5)
    sol = wiu.Solver(g.x, g.y, "5-2MP", g.bc, g.period)
    Ud = _dev(U)
    plan = plan_for(wiu, blocks, Ub, "5-2MP")
    plan.cfl_dt(0.5)
    dt = float(plan.get_dt()[0])
    sol.rk3_step(Ud, dt)
    plan.step(graph=True)
    assert plan.status() == 0 and sol.status() == 0
    ref = _host(Ud)
    out = W.assemble(blocks, [plan.state(b).cpu().numpy() for b in range(len(blocks))], g.shape)
    assert np.all(normwise(out - U, ref - U) <= 1e-11)
    plan.close()


@pytest.mark.parametrize("s", ["3-1MP", "5-2MP", "7-6MP"])
def test_free_stream_preserved_on_turned_blocks(wiu, s):
    import torch
    for name in ("periodic6", "bounded6"):
        kind, nx, ny, ic, jc, turns, _ = CONFIGS[name]
        g = (W.periodic_grid if kind == "periodic" else W.bounded_grid)(nx, ny, A=0.3, seed=2)
        U = W.uniform_flow(g)
        blocks, (Ub,) = W.cut_blocks(g, [U], icuts=ic, jcuts=jc, turns=turns)
        plan = plan_for(wiu, blocks, Ub, s)
        plan.cfl_dt(0.5)
        dt = plan.get_dt()
        plan.step(graph=False)
        assert plan.status() == 0
        # the increment over dt: the rate dU/dt, bounded as for one grid
        for b in range(len(blocks)):
            assert np.abs(plan.state(b).cpu().numpy() - Ub[b]).max() / dt[b] < 1e-11, (name, b)
        plan.close()
