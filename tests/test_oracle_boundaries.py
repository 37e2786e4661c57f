"""Pins of the boundary rules beyond periodic and transmissive (the paper
states none; the library's): reflecting slip walls (mirror image about the
boundary node, momentum component along the boundary's metric direction
reversed) and fixed states (supersonic inflow), per side.

* A box with walls at both ends is the mirror-symmetric half of the periodic
  problem twice as long: the residual and several RK3 steps agree with that
  problem's to round-off on the shared nodes.
* On a rotated box the wall residual is the rotated residual (the wall
  normal comes from the metrics).
* Uniform flow parallel to walls, or entering through a fixed side equal to
  it, stays uniform (free-stream preservation with these rules).
* The Shu-Osher problem (Sec. 6.2(2); inflow on the left, transmissive on
  the right) converges under refinement against a finer solution."""
import math

import numpy as np
import pytest

from paper_1810_11103_amd import workloads as W

G = 4


def _box(nx, ny, L=1.0, H=1.0, theta=0.0):
    """Cartesian nodes x = i L/(nx-1), y = j H/(ny-1), rotated by theta."""
    jj, ii = np.meshgrid(np.arange(ny, dtype=float), np.arange(nx, dtype=float), indexing="ij")
    x, y = ii * L / (nx - 1), jj * H / (ny - 1)
    c, s = math.cos(theta), math.sin(theta)
    return np.ascontiguousarray(c * x - s * y), np.ascontiguousarray(s * x + c * y)


def _mirror_data(x, y):
    """rho, p, v even and u odd about x = 0 and x = 1 (period 2 in x),
    periodic in y with period 1."""
    rho = 1.0 + 0.2 * np.cos(np.pi * x) * (1.0 + 0.3 * np.sin(2 * np.pi * y))
    u = 0.4 * np.sin(np.pi * x) + 0.1 * np.sin(3 * np.pi * x)
    v = 0.2 * np.cos(np.pi * x) * np.cos(2 * np.pi * y)
    p = 1.0 + 0.15 * np.cos(2 * np.pi * x) + 0.05 * np.sin(2 * np.pi * y)
    return W.conservative(rho, u, v, p)


@pytest.mark.parametrize("s", ["3-1MP", "5-2MP", "7-4MP"])
def test_walls_equal_the_mirror_extended_periodic_problem(orc, s):
    N, ny = 40, 24
    h = 1.0 / N
    # wall problem: nodes x = 0..1 (N + 1), periodic in y
    jj, ii = np.meshgrid(np.arange(ny, dtype=float), np.arange(N + 1, dtype=float), indexing="ij")
    xw, yw = ii * h, jj / ny
    Uw = _mirror_data(xw, yw)
    bcw = ("transmissive", "periodic")
    Mw = orc.metrics(s, xw, yw, bcw, (0.0, 1.0))
    sides = ("wall", "wall", "transmissive", "transmissive")
    # periodic problem: nodes x = -1 .. 1 - h (2N), period 2
    jj, ii = np.meshgrid(np.arange(ny, dtype=float), np.arange(2 * N, dtype=float), indexing="ij")
    xp, yp = -1.0 + ii * h, jj / ny
    Up = _mirror_data(xp, yp)
    Mp = orc.metrics(s, xp, yp, ("periodic", "periodic"), (2.0, 1.0))
    idx = np.r_[np.arange(N, 2 * N), 0]  # periodic column of wall node i = 0..N
    dw = orc.rhs(s, Uw, Mw, bcw, sides=sides)
    dp = orc.rhs(s, Up, Mp, ("periodic", "periodic"))
    scale = np.abs(dp).max()
    assert np.abs(dw - dp[:, :, idx]).max() <= 1e-13 * scale
    for _ in range(3):
        Uw = orc.rk3_step(s, Uw, Mw, 2e-3, bcw, sides=sides)
        Up = orc.rk3_step(s, Up, Mp, 2e-3, ("periodic", "periodic"))
    assert np.abs(Uw - Up[:, :, idx]).max() <= 1e-13


def test_wall_normal_follows_the_metrics(orc):
    """Four walls on a unit box and on the same box rotated by 0.6 rad: the
    residuals agree with momentum rotated (scalars equal)."""
    s = "5-2MP"
    th = 0.6
    bc = ("transmissive", "transmissive")
    sides = ("wall",) * 4
    x0, y0 = _box(33, 29)
    x1, y1 = _box(33, 29, theta=th)
    rho = 1.0 + 0.2 * np.cos(np.pi * x0) * np.cos(np.pi * y0)
    u = 0.3 * np.sin(np.pi * x0) * np.cos(np.pi * y0)
    v = -0.2 * np.cos(np.pi * x0) * np.sin(np.pi * y0)
    p = 1.0 + 0.1 * np.cos(np.pi * x0 * 2)
    c, sn = math.cos(th), math.sin(th)
    U0 = W.conservative(rho, u, v, p)
    U1 = W.conservative(rho, c * u - sn * v, sn * u + c * v, p)
    d0 = orc.rhs(s, U0, orc.metrics(s, x0, y0, bc), bc, sides=sides)
    d1 = orc.rhs(s, U1, orc.metrics(s, x1, y1, bc), bc, sides=sides)
    scale = np.abs(d0).max()
    np.testing.assert_allclose(d1[0], d0[0], atol=1e-12 * scale)
    np.testing.assert_allclose(d1[3], d0[3], atol=1e-12 * scale)
    np.testing.assert_allclose(d1[1], c * d0[1] - sn * d0[2], atol=1e-12 * scale)
    np.testing.assert_allclose(d1[2], sn * d0[1] + c * d0[2], atol=1e-12 * scale)


@pytest.mark.parametrize("s", ["3-2MP", "5-1MP", "7-6MP"])
def test_free_stream_with_walls_and_inflow(orc, s):
    """Mach-2 flow along x on a randomized grid whose four boundary layers
    are uniform: walls top and bottom (parallel to the flow), the same state
    fixed on the left, transmissive on the right."""
    g = W.bounded_grid(48, 40, (0, 1.2, 0, 1), A=0.2, seed=6)
    U = W.uniform_flow(g, mach=2.0, angle=0.0)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    fixed = np.zeros((4, 4))
    fixed[0] = U[:, 0, 0]
    d = orc.rhs(s, U, M, g.bc, sides=("fixed", "transmissive", "wall", "wall"), fixed=fixed)
    assert np.abs(d).max() < 1e-11


def _shu_osher(orc, s, n, dt):
    g = W.line_grid(n, -5.0, 5.0)
    U = W.shu_osher_state(g)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    fixed = np.zeros((4, 4))
    fixed[0] = U[:, 0, 0]
    nsteps = int(round(1.8 / dt))
    U = orc.rk3_run(s, U, M, dt, nsteps, g.bc, sides=("fixed", "transmissive", "transmissive", "transmissive"),
                    fixed=fixed)
    return g, U


def test_shu_osher_converges_under_refinement(orc):
    """Sec. 6.2(2) with 201 and 401 nodes (the paper's dt = 0.001 at 401)
    against 801 nodes: positive, the main shock near x = 2.4, and the L1
    density difference to the finer solution falls with refinement."""
    s = "5-2MP"
    gf, Uf = _shu_osher(orc, s, 801, 0.0005)
    errs = []
    for n, dt, stride in ((201, 0.002, 4), (401, 0.001, 2)):
        g, U = _shu_osher(orc, s, n, dt)
        rho = W.primitive(U)[0][0]
        assert np.all(np.isfinite(U)) and rho.min() > 0 and W.primitive(U)[3].min() > 0
        errs.append(np.mean(np.abs(rho - W.primitive(Uf)[0][0][::stride])))
    assert errs[1] < 0.7 * errs[0], errs
    rho = W.primitive(U)[0][0]
    x = g.x[0]
    # the main shock: the largest density drop right of x = 1
    k = np.argmin(np.diff(rho) + 100 * (x[:-1] < 1.0))
    assert 2.2 < x[k] < 2.6, x[k]
