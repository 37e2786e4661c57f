"""GPU parity of the wall and fixed-state side rules against the oracle
(residual within 1e-12 normwise, RK3 increments within 1e-11), plus the
mirror property on the GPU itself and the Shu-Osher run."""
import math
import sys

import numpy as np
import pytest

from paper_1810_11103_amd import workloads as W
from test_gpu_parity import _dev, _host, make_case, normwise
from test_oracle_boundaries import _box, _mirror_data

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wiu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1810_11103_amd import wenoiu
    return wenoiu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _riemann_with_sides(nx, ny, seed):
    g = W.bounded_grid(nx, ny, (0, 1, 0, 1), A=0.2, seed=seed)
    U = W.riemann_state(g)
    fixed = np.zeros((4, 4))
    fixed[0] = W.conservative(1.5, 0.8, 0.1, 1.5).ravel()
    fixed[3] = W.conservative(0.5, 0.0, -0.3, 0.4).ravel()
    return g, U, ("fixed", "wall", "wall", "fixed"), fixed


@pytest.mark.parametrize("s", ["3-1MP", "3-2MP", "5-1MP", "5-2MP", "7-2MP", "7-6MP"])
def test_rhs_parity_walls_and_fixed_sides(orc, wiu, s):
    say("rhs parity sides", s)
    g, U, sides, fixed = _riemann_with_sides(260, 90, 3)
    Mo = orc.metrics(s, g.x, g.y, g.bc, g.period)
    ref = orc.rhs(s, U, Mo, g.bc, sides=sides, fixed=fixed)
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period, sides=sides, fixed=fixed)
    out = _host(sol.rhs(_dev(U)))
    assert sol.status() == 0
    err = normwise(out, ref)
    assert np.all(err <= 1e-12), err


@pytest.mark.parametrize("s", ["5-2MP", "7-4MP"])
def test_rotated_wall_box_parity(orc, wiu, s):
    say("rotated wall box", s)
    x, y = _box(97, 83, theta=0.6)
    bc = ("transmissive", "transmissive")
    U = W.conservative(1.0 + 0.2 * np.cos(3 * x) * np.cos(2 * y), 0.3 * np.sin(2 * x), -0.2 * np.cos(x + y),
                       1.0 + 0.1 * np.sin(4 * x * y))
    sides = ("wall",) * 4
    Mo = orc.metrics(s, x, y, bc)
    ref = orc.rhs(s, U, Mo, bc, sides=sides)
    sol = wiu.Solver(x, y, s, bc, sides=sides)
    out = _host(sol.rhs(_dev(U)))
    assert sol.status() == 0
    assert np.all(normwise(out, ref) <= 1e-12)


def test_walls_equal_the_mirror_extended_problem_on_gpu(wiu):
    """The mirror property of the oracle tests, on the GPU (two different
    launches, so agreement is to round-off, not bitwise)."""
    s, N, ny = "5-2MP", 200, 96
    h = 1.0 / N
    jj, ii = np.meshgrid(np.arange(ny, dtype=float), np.arange(N + 1, dtype=float), indexing="ij")
    xw, yw = ii * h, jj / ny
    jj, ii = np.meshgrid(np.arange(ny, dtype=float), np.arange(2 * N, dtype=float), indexing="ij")
    xp, yp = -1.0 + ii * h, jj / ny
    solw = wiu.Solver(xw, yw, s, ("transmissive", "periodic"), (0.0, 1.0), sides=("wall", "wall", 0, 0))
    solp = wiu.Solver(xp, yp, s, ("periodic", "periodic"), (2.0, 1.0))
    Uw, Up = _dev(_mirror_data(xw, yw)), _dev(_mirror_data(xp, yp))
    idx = np.r_[np.arange(N, 2 * N), 0]
    for _ in range(5):
        solw.rk3_step(Uw, 1e-3)
        solp.rk3_step(Up, 1e-3)
    assert np.abs(_host(Uw) - _host(Up)[:, :, idx]).max() <= 1e-13
    assert solw.status() == 0 and solp.status() == 0


@pytest.mark.parametrize("s", ["3-2MP", "5-1MP", "7-6MP"])
def test_free_stream_with_walls_and_inflow_on_gpu(wiu, s):
    g = W.bounded_grid(512, 384, (0, 1.2, 0, 1), A=0.2, seed=6)
    U = W.uniform_flow(g, mach=2.0, angle=0.0)
    fixed = np.zeros((4, 4))
    fixed[0] = U[:, 0, 0]
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period, sides=("fixed", "transmissive", "wall", "wall"), fixed=fixed)
    d = _host(sol.rhs(_dev(U)))
    assert sol.status() == 0
    assert np.abs(d).max() < 1e-11


def test_shu_osher_steps_track_the_oracle(orc, wiu):
    """Sec. 6.2(2), 401 nodes, dt = 0.001: 200 steps on both sides."""
    s = "5-2MP"
    g = W.line_grid(401, -5.0, 5.0)
    U = W.shu_osher_state(g)
    fixed = np.zeros((4, 4))
    fixed[0] = U[:, 0, 0]
    sides = ("fixed", "transmissive", 0, 0)
    Mo = orc.metrics(s, g.x, g.y, g.bc, g.period)
    ref = orc.rk3_run(s, U, Mo, 1e-3, 200, g.bc, sides=sides, fixed=fixed)
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period, sides=sides, fixed=fixed)
    Ud = _dev(U)
    for _ in range(200):
        sol.rk3_step(Ud, 1e-3)
    assert sol.status() == 0
    err = normwise(_host(Ud) - U, ref - U)
    assert np.all(err <= 1e-10), err


def test_sides_are_validated(wiu):
    import torch
    g, U, sides, fixed = _riemann_with_sides(64, 48, 1)
    bad = np.array(fixed)
    bad[0, 0] = -1.0
    with pytest.raises(RuntimeError):
        wiu.Solver(g.x, g.y, "5-2MP", g.bc, g.period, sides=sides, fixed=bad).rhs(_dev(U))
    with pytest.raises(RuntimeError):
        wiu.Solver(g.x, g.y, "5-2MP", g.bc, g.period, sides=(3, 0, 0, 0)).rhs(_dev(U))
    sol = wiu.Solver(g.x, g.y, "5-2MP", g.bc, g.period, sides=sides, fixed=fixed)
    Ud = _dev(U)
    with pytest.raises(RuntimeError):
        sol.rhs_vjp(Ud, torch.ones_like(Ud))
