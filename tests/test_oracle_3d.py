"""Pins of the oracle's three-dimensional path (Sec. 2.1-2.4 in 3-D: Eq. 2.2,
symmetric conservative metrics Eq. 2.4, Jacobian Eq. 2.5, the characteristic
projection of Sec. 3.4 with five eigenvectors).

* z-independent data reduce to the 2-D scheme (pinned by the other test
  files): xi^ and eta^ and their midpoint values equal the 2-D metrics, the
  flux residual J^{-1} dU/dt equals the 2-D one, dU/dt of rho w and the
  variation along z vanish, and J^{-1} is Eq. 2.5: (2 J_2D + zeta^_z) / 3.
* Free-stream preservation on randomized periodic and bounded grids and on a
  smooth grid where all nine metrics vary (the property the symmetric
  conservative form exists for).
* Eigenvectors: L R = I and R diag(q_n - c, q_n, q_n, q_n, q_n + c) L is the
  flux Jacobian along n (central differences of E^).
* Conservation: sum J^{-1} dU/dt = 0 on periodic grids.
* Design order of the residual on an exact entropy wave over the smooth grid.
"""
import numpy as np
import pytest

import oracle as orc
from paper_1810_11103_amd import workloads as W

G = 4


def _flux_residual3(M3, r3):
    return M3[9, G:-G, G:-G, G:-G] * r3


@pytest.mark.parametrize("s", ["3-1MP", "3-2MP", "5-1MP", "5-2MP", "7-1MP", "7-4MP"])
@pytest.mark.parametrize("kind", ["periodic", "bounded"])
def test_z_independent_data_reduce_to_the_2d_scheme(s, kind):
    if kind == "periodic":
        g = W.periodic_grid(24, 20, box=(0.0, 2.4, 0.0, 2.0), A=0.3, seed=4)
        U = W.random_smooth_state(g, seed=2, amp=0.2)
    else:
        g = W.bounded_grid(22, 20, A=0.3, seed=4)
        U = W.riemann_state(g)
    M2 = orc.metrics(s, g.x, g.y, g.bc, g.period)
    r2 = orc.rhs(s, U, M2, g.bc)
    g3, U3 = W.extrude(g, 3, U)
    M3 = orc.metrics3(s, g3.x, g3.y, g3.z, g3.bc, g3.period)
    r3 = orc.rhs3(s, U3, M3, g3.bc)
    m = M3[:, G + 1]
    for p2, p3 in ((0, 0), (1, 1), (2, 3), (3, 4), (5, 10), (6, 11), (7, 13), (8, 14)):
        assert np.abs(M2[p2] - m[p3]).max() <= 1e-14 * np.abs(M2[p2]).max(), (p2, p3)
    assert np.all(m[[2, 5, 6, 7, 12, 15, 16, 17]] == 0.0)
    # Eq. 2.5 with z = zeta: (xi^ . r_xi + eta^ . r_eta + zeta^ . r_zeta) / 3
    assert np.abs(m[9] - (2.0 * M2[4] + m[8]) / 3.0).max() <= 1e-14 * np.abs(M2[4]).max()
    f2 = M2[4, G:-G, G:-G] * r2
    f3 = _flux_residual3(M3, r3)
    for q2, q3 in ((0, 0), (1, 1), (2, 2), (3, 4)):
        for k in range(3):
            assert np.abs(f3[q3, k] - f2[q2]).max() <= 1e-13 * np.abs(f2[q2]).max(), (q2, k)
    assert np.all(r3[3] == 0.0)


def test_cartesian_jacobian_equals_the_2d_one():
    g = W.periodic_grid(16, 12, box=(0.0, 1.6, 0.0, 1.2))
    M2 = orc.metrics("5-2MP", g.x, g.y, g.bc, g.period)
    g3, _ = W.extrude(g, 2)
    M3 = orc.metrics3("5-2MP", g3.x, g3.y, g3.z, g3.bc, g3.period)
    assert np.allclose(M3[9, G], M2[4], rtol=1e-14, atol=0.0)


@pytest.mark.parametrize("s", ["3-1MP", "5-2MP", "7-2MP", "7-6MP"])
def test_free_stream_preserved(s):
    for g in (W.wavy_grid3(20, 18, 16), W.periodic_grid3(18, 16, 14, A=0.3, seed=1),
              W.bounded_grid3(18, 16, 14, A=0.3, seed=1),
              W.mixed_grid3(18, 16, 14, ("periodic", "transmissive", "periodic"), A=0.3, seed=2),
              W.mixed_grid3(16, 18, 14, ("transmissive", "periodic", "transmissive"), A=0.3, seed=3)):
        U = W.uniform_flow3(g)
        M = orc.metrics3(s, g.x, g.y, g.z, g.bc, g.period)
        assert np.abs(orc.rhs3(s, U, M, g.bc)).max() < 1e-11


def test_eigenvectors_diagonalise_the_flux_jacobian():
    rng = np.random.default_rng(3)
    gam = 1.4
    for _ in range(6):
        Q = W.conservative3(1.0 + rng.random(), *(rng.standard_normal(3) * 0.5), 1.0 + rng.random())
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        L, R = orc.eigenvectors3(Q, gam, n)
        assert np.allclose(L @ R, np.eye(5), atol=1e-13)
        rho, u, v, w = Q[0], Q[1] / Q[0], Q[2] / Q[0], Q[3] / Q[0]
        p = (gam - 1) * (Q[4] - 0.5 * rho * (u * u + v * v + w * w))
        c = np.sqrt(gam * p / rho)
        qn = u * n[0] + v * n[1] + w * n[2]
        A = R @ np.diag([qn - c, qn, qn, qn, qn + c]) @ L
        h = 1e-6
        Jfd = np.zeros((5, 5))
        for b in range(5):
            e = np.zeros(5)
            e[b] = h * max(1.0, abs(Q[b]))
            Jfd[:, b] = (orc.flux_hat3(Q + e, gam, n) - orc.flux_hat3(Q - e, gam, n)) / (2 * e[b])
        assert np.allclose(A, Jfd, atol=1e-7)


def test_conservation_on_periodic_grids():
    g = W.periodic_grid3(16, 14, 12, A=0.3, seed=5)
    U = W.octant_state3(g)
    M = orc.metrics3("5-2MP", g.x, g.y, g.z, g.bc, g.period)
    f = _flux_residual3(M, orc.rhs3("5-2MP", U, M, g.bc))
    tot = f.sum(axis=(1, 2, 3))
    scale = np.abs(f).sum(axis=(1, 2, 3))
    assert np.all(np.abs(tot) < 1e-13 * scale), (tot, scale)


@pytest.mark.parametrize("s,order", [("3-2MP", 3.0), ("5-2MP", 5.0)])
def test_design_order_on_a_smooth_grid(s, order):
    """Residual against the exact dU/dt of an entropy wave (uniform velocity
    and pressure) on the smooth curvilinear grid, under refinement."""
    errs = []
    ns = (16, 24, 32)
    for n in ns:
        g = W.wavy_grid3(n, n, n)
        U = W.entropy_wave3(g)
        M = orc.metrics3(s, g.x, g.y, g.z, g.bc, g.period)
        r = orc.rhs3(s, U, M, g.bc)
        # d rho/dt = -amp (2 pi / L) (u + v + w) cos(2 pi (x + y + z) / L)
        k = 2 * np.pi / g.period[0]
        exact = -0.2 * k * (0.6 + 0.4 + 0.3) * np.cos(k * (g.x + g.y + g.z))
        errs.append(np.abs(r[0] - exact).max())
    p = np.log(errs[-2] / errs[-1]) / np.log(ns[-1] / ns[-2])
    assert p > order - 0.5, (errs, p)


def test_jacobian_by_eq_2_6():
    """Eq. 2.6 changes J^{-1} only: exact on a Cartesian grid, the other 18
    planes identical to Eq. 2.5's, and on a smooth grid the two forms of
    J^{-1} approach each other as the grid is refined (both approximate the
    same Jacobian, their difference at the operator's order)."""
    g = W.periodic_grid3(10, 10, 10, box=(0.0, 1.0, 0.0, 2.0, 0.0, 3.0))
    M6 = orc.metrics3("5-2MP", g.x, g.y, g.z, g.bc, g.period, jform=6)
    assert np.allclose(M6[9], 0.1 * 0.2 * 0.3, rtol=1e-14, atol=0.0)
    for g in (W.periodic_grid3(14, 12, 10, A=0.3, seed=1), W.bounded_grid3(14, 12, 12, A=0.3, seed=1)):
        M5 = orc.metrics3("5-2MP", g.x, g.y, g.z, g.bc, g.period, jform=5)
        M6 = orc.metrics3("5-2MP", g.x, g.y, g.z, g.bc, g.period, jform=6)
        assert np.array_equal(np.delete(M5, 9, axis=0), np.delete(M6, 9, axis=0))
    diffs = []
    for n in (12, 24):
        g = W.wavy_grid3(n, n, n)
        M5 = orc.metrics3("5-2MP", g.x, g.y, g.z, g.bc, g.period, jform=5)
        M6 = orc.metrics3("5-2MP", g.x, g.y, g.z, g.bc, g.period, jform=6)
        diffs.append(np.abs(M5[9] - M6[9]).max() / np.abs(M5[9]).max())
    assert np.log2(diffs[0] / diffs[1]) > 4.5, diffs


def _mirror_data3(x, y, z, axis):
    """rho, p and the two tangential velocities even, the normal velocity odd
    about both ends (0 and 1) of coordinate `axis`; periodic in the others."""
    c = (x, y, z)
    a = c[axis]
    b, e = c[(axis + 1) % 3], c[(axis + 2) % 3]
    rho = 1.0 + 0.2 * np.cos(np.pi * a) * (1.0 + 0.3 * np.sin(2 * np.pi * b) * np.cos(2 * np.pi * e))
    un = 0.4 * np.sin(np.pi * a) + 0.1 * np.sin(3 * np.pi * a)
    ub = 0.2 * np.cos(np.pi * a) * np.cos(2 * np.pi * b)
    ue = 0.15 * np.cos(2 * np.pi * a) * np.sin(2 * np.pi * e)
    p = 1.0 + 0.15 * np.cos(2 * np.pi * a) + 0.05 * np.sin(2 * np.pi * b)
    vel = [None] * 3
    vel[axis], vel[(axis + 1) % 3], vel[(axis + 2) % 3] = un, ub, ue
    return W.conservative3(rho, *vel, p)


def _box3(n, axis, two=False):
    """Nodes along `axis`: 0..1 (n+1 nodes) or, two=True, -1 .. 1-h (2n
    nodes); the other two axes periodic on [0, 1) with 10 and 8 nodes."""
    counts = [10, 8, 12]
    counts[axis] = 2 * n if two else n + 1
    kk, jj, ii = np.meshgrid(*[np.arange(counts[d], dtype=float) for d in (2, 1, 0)], indexing="ij")
    idx = (ii, jj, kk)
    crd = []
    for d in range(3):
        if d == axis:
            crd.append((-1.0 + idx[d] / n) if two else idx[d] / n)
        else:
            crd.append(idx[d] / counts[d])
    return [np.ascontiguousarray(v) for v in crd]


@pytest.mark.parametrize("s", ["3-1MP", "5-2MP"])
@pytest.mark.parametrize("axis", [0, 2])
def test_walls_equal_the_mirror_extended_periodic_problem_3d(s, axis):
    """Walls at both ends of one axis (Sec. 6 boundaries in 3-D; the library's
    rule, as in 2-D) give the residual and RK3 steps of the periodic problem
    twice as long with mirror-symmetric data, on the shared nodes."""
    N = 16
    xw, yw, zw = _box3(N, axis)
    bcw = ["periodic"] * 3
    bcw[axis] = "transmissive"
    per = [1.0, 1.0, 1.0]
    per[axis] = 0.0
    sides = ["transmissive"] * 6
    sides[2 * axis] = sides[2 * axis + 1] = "wall"
    Uw = _mirror_data3(xw, yw, zw, axis)
    Mw = orc.metrics3(s, xw, yw, zw, bcw, per)
    xp, yp, zp = _box3(N, axis, two=True)
    perp = [1.0, 1.0, 1.0]
    perp[axis] = 2.0
    Up = _mirror_data3(xp, yp, zp, axis)
    Mp = orc.metrics3(s, xp, yp, zp, ("periodic",) * 3, perp)
    idx = np.r_[np.arange(N, 2 * N), 0]
    take = lambda a: np.take(a, idx, axis=3 - axis)
    dw = orc.rhs3(s, Uw, Mw, bcw, sides=sides)
    dp = orc.rhs3(s, Up, Mp, ("periodic",) * 3)
    assert np.abs(dw - take(dp)).max() <= 1e-13 * np.abs(dp).max()
    for _ in range(3):
        Uw = orc.rk3_step3(s, Uw, Mw, 2e-3, bcw, sides=sides)
        Up = orc.rk3_step3(s, Up, Mp, 2e-3, ("periodic",) * 3)
    assert np.abs(Uw - take(Up)).max() <= 1e-13


@pytest.mark.parametrize("s", ["3-2MP", "5-2MP", "7-1MP"])
def test_free_stream_with_walls_and_inflow_3d(s):
    """Mach-2 flow along x on a randomized bounded grid with uniform boundary
    layers: walls on the y and z sides (parallel to the flow), the same state
    fixed on x low, transmissive on x high."""
    g = W.bounded_grid3(20, 16, 14, A=0.2, seed=6)
    U = W.uniform_flow3(g, mach=2.0, direction=(1.0, 0.0, 0.0))
    fixed = np.zeros((6, 5))
    fixed[0] = U[:, 0, 0, 0]
    M = orc.metrics3(s, g.x, g.y, g.z, g.bc, g.period)
    d = orc.rhs3(s, U, M, g.bc, sides=("fixed", "transmissive", "wall", "wall", "wall", "wall"), fixed=fixed)
    assert np.abs(d).max() < 1e-11


OPTION_CASES = [("5-2MP", dict(vars="conservative")), ("5-1MP", dict(vars="primitive")),
                ("3-2MP", dict(weights="z")), ("7-1MP", dict(weights="z", vars="primitive")),
                ("3-1MP", dict(alpha_h=0.8)), ("5-1MP", dict(alpha_h=1.3, vars="conservative")),
                ("5-2MP", dict(split="sw")), ("3-1MP", dict(split="vl")), ("7-2MP", dict(split="sw", weights="z")),
                ("5-1MP", dict(split="vl", vars="primitive"))]


@pytest.mark.parametrize("s,opts", OPTION_CASES)
def test_z_independent_data_reduce_to_the_2d_scheme_with_options(s, opts):
    """The scheme options of Secs. 2.4, 3.2-3.3 and 7 (interpolation
    variables, WENO-Z weights, the free alpha) in 3-D reduce to the 2-D
    oracle's for z-independent data (flux residual; the metrics with alpha)."""
    g = W.periodic_grid(24, 20, box=(0.0, 2.4, 0.0, 2.0), A=0.3, seed=4)
    U = W.random_smooth_state(g, seed=2, amp=0.2)
    ah = opts.get("alpha_h", 1.0)
    M2 = orc.metrics(s, g.x, g.y, g.bc, g.period, alpha_h=ah)
    r2 = orc.rhs(s, U, M2, g.bc, **opts)
    g3, U3 = W.extrude(g, 3, U)
    M3 = orc.metrics3(s, g3.x, g3.y, g3.z, g3.bc, g3.period, alpha_h=ah)
    r3 = orc.rhs3(s, U3, M3, g3.bc, **opts)
    m = M3[:, G + 1]
    for p2, p3 in ((0, 0), (1, 1), (2, 3), (3, 4), (5, 10), (6, 11), (7, 13), (8, 14)):
        assert np.abs(M2[p2] - m[p3]).max() <= 1e-14 * np.abs(M2[p2]).max(), (p2, p3)
    f2 = M2[4, G:-G, G:-G] * r2
    f3 = _flux_residual3(M3, r3)
    for q2, q3 in ((0, 0), (1, 1), (2, 2), (3, 4)):
        assert np.abs(f3[q3, 1] - f2[q2]).max() <= 1e-13 * np.abs(f2[q2]).max(), q2
    assert np.all(r3[3] == 0.0)


@pytest.mark.parametrize("s,opts", OPTION_CASES)
def test_free_stream_preserved_with_options(s, opts):
    for g in (W.wavy_grid3(16, 16, 14), W.bounded_grid3(16, 15, 14, A=0.3, seed=1)):
        U = W.uniform_flow3(g)
        M = orc.metrics3(s, g.x, g.y, g.z, g.bc, g.period, alpha_h=opts.get("alpha_h", 1.0))
        assert np.abs(orc.rhs3(s, U, M, g.bc, **opts)).max() < 1e-11


def test_3d_splits_sum_to_the_flux_and_van_leer_limits():
    """Both 3-D splits satisfy F+ + F- = E^(Q; k) (E^ is homogeneous of
    degree one); van Leer's F+ is E^ and F- zero for M >= 1 (mirrored for
    M <= -1); for random 3-D states and directions."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        vel = rng.standard_normal(3) * 0.8
        Q = W.conservative3(0.5 + rng.random(), *vel, 0.5 + rng.random())
        k = rng.standard_normal(3) * (0.5 + rng.random())
        E = orc.flux_hat3(Q, 1.4, k)
        for sp in ("sw", "vl"):
            tot = orc.midpoint_split3(sp, Q, k, 0) + orc.midpoint_split3(sp, Q, k, 1)
            assert np.allclose(tot, E, rtol=1e-13, atol=1e-13 * np.abs(E).max()), sp
    # supersonic along k
    Q = W.conservative3(1.0, 2.0, 0.3, -0.4, 0.5)
    k = np.array([1.0, 0.1, -0.2])
    assert np.allclose(orc.midpoint_split3("vl", Q, k, 0), orc.flux_hat3(Q, 1.4, k), rtol=1e-14)
    assert np.all(orc.midpoint_split3("vl", Q, k, 1) == 0.0)
    assert np.allclose(orc.midpoint_split3("vl", Q, -k, 1), orc.flux_hat3(Q, 1.4, -k), rtol=1e-14)
