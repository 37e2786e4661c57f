"""Pins of the oracle's 2-D Euler path (metrics, characteristic fluxes, rhs,
RK3) against what the paper and the mathematics fix: free-stream
preservation (Sec. 5.2, Table 4), telescoping conservation, mirror and
transpose symmetry, the exact Sod solution, the design order on the
isentropic vortex (Sec. 6.3(1)), and the third order of TVD-RK3."""
import os

import numpy as np
import pytest
from scipy.optimize import brentq

from paper_1810_11103_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SCHEMES = ["3-1MP", "3-2MP", "5-1MP", "5-2MP"]
GAMMA = 1.4


# ---------------------------------------------------------------------------
# pointwise pieces
# ---------------------------------------------------------------------------

def _textbook_flux(Q, kx, ky, g=GAMMA):
    rho, u, v, p = W.primitive(np.asarray(Q, dtype=float).reshape(4, 1, 1), g)
    rho, u, v, p = (float(a.ravel()[0]) for a in (rho, u, v, p))
    e = Q[3]
    E = np.array([rho * u, rho * u * u + p, rho * u * v, (e + p) * u])
    F = np.array([rho * v, rho * u * v, rho * v * v + p, (e + p) * v])
    return kx * E + ky * F


def test_flux_is_metric_combination_of_cartesian_fluxes(orc):
    """Eq. 2.2: E^ = xi_x^ E + xi_y^ F."""
    rng = np.random.default_rng(0)
    for _ in range(20):
        Q = W.conservative(rng.uniform(0.5, 2), rng.uniform(-1, 1), rng.uniform(-1, 1),
                           rng.uniform(0.5, 2)).ravel()
        kx, ky = rng.standard_normal(2)
        np.testing.assert_allclose(orc.flux_hat(Q, GAMMA, kx, ky), _textbook_flux(Q, kx, ky), rtol=1e-13,
                                   atol=1e-13)


def test_eigenvectors_diagonalise_the_flux_jacobian(orc):
    """Sec. 3.4: L R = I and A R = R diag(q_n - c, q_n, q_n, q_n + c) with A
    the Jacobian of the flux in the unit direction n (central differences)."""
    rng = np.random.default_rng(1)
    for _ in range(10):
        rho, u, v, p = rng.uniform(0.5, 2), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.5, 2)
        Q = W.conservative(rho, u, v, p).ravel()
        th = rng.uniform(0, 2 * np.pi)
        n = np.array([np.cos(th), np.sin(th)])
        L, R = orc.eigenvectors(Q, GAMMA, n[0], n[1])
        np.testing.assert_allclose(L @ R, np.eye(4), atol=1e-13)
        A = np.zeros((4, 4))
        for q in range(4):
            h = 1e-6 * max(1.0, abs(Q[q]))
            dq = np.zeros(4)
            dq[q] = h
            A[:, q] = (orc.flux_hat(Q + dq, GAMMA, *n) - orc.flux_hat(Q - dq, GAMMA, *n)) / (2 * h)
        c = np.sqrt(GAMMA * p / rho)
        qn = u * n[0] + v * n[1]
        lam = np.array([qn - c, qn, qn, qn + c])
        np.testing.assert_allclose(A @ R, R * lam[None, :], atol=2e-8)


def test_midpoint_flux_linear_weights_reduce_to_componentwise(orc):
    """On data with all indicators equal (a linear profile) the weights are
    the linear ones and characteristic interpolation equals componentwise
    interpolation of the conservative variables (R L = I)."""
    rng = np.random.default_rng(2)
    Q0 = W.conservative(1.0, 0.3, -0.2, 1.0).ravel()
    dQ = rng.standard_normal(4) * 0.01
    Qs = np.array([Q0 + m * dQ for m in range(-2, 4)])
    k0 = np.array([0.1, 0.02])
    k1 = np.array([0.11, 0.01])
    mk = np.array([0.105, 0.015])
    lam = 0.3
    for s in SCHEMES:
        Fp, Fm = orc.midpoint_flux(s, Qs, k0, k1, mk, lam)
        QL = Q0 + 0.5 * dQ  # linear data: every candidate is exact
        ref_p = 0.5 * (orc.flux_hat(QL, GAMMA, *mk) + lam * QL)
        ref_m = 0.5 * (orc.flux_hat(QL, GAMMA, *mk) - lam * QL)
        np.testing.assert_allclose(Fp, ref_p, atol=1e-13)
        np.testing.assert_allclose(Fm, ref_m, atol=1e-13)


# ---------------------------------------------------------------------------
# metrics
# ---------------------------------------------------------------------------

def _interior(M, G=4):
    return M[:, G:-G, G:-G]


@pytest.mark.parametrize("s", SCHEMES)
def test_metrics_exact_on_affine_grids(orc, s):
    """Sec. 2.2: on an affine grid every consistent operator returns the
    exact metrics (xi_x^ = y_eta, xi_y^ = -x_eta, eta_x^ = -y_xi, eta_y^ = x_xi)."""
    n = 24
    jj, ii = np.meshgrid(np.arange(n, dtype=float), np.arange(n, dtype=float), indexing="ij")
    a, b, c, d = 0.3, 0.05, -0.04, 0.25
    x = 1.0 + a * ii + b * jj
    y = -2.0 + c * ii + d * jj
    for bc, per in ((("transmissive", "transmissive"), (0, 0)),):
        M = _interior(orc.metrics(s, x, y, bc, per))
        np.testing.assert_allclose(M[0], d, atol=1e-14)
        np.testing.assert_allclose(M[1], -b, atol=1e-14)
        np.testing.assert_allclose(M[2], -c, atol=1e-14)
        np.testing.assert_allclose(M[3], a, atol=1e-14)
        np.testing.assert_allclose(M[4], a * d - b * c, atol=1e-14)
        np.testing.assert_allclose(M[5], d, atol=1e-14)
        np.testing.assert_allclose(M[8], a, atol=1e-14)


@pytest.mark.parametrize("s,order", [("3-1MP", 4), ("3-2MP", 4), ("5-1MP", 6), ("5-2MP", 6)])
def test_metrics_converge_on_smooth_grid(orc, s, order):
    """On a smooth periodic curvilinear grid the metrics converge to the
    analytic ones at the order of the scheme's central operator."""
    errs = []
    for n in (32, 64):
        g = W.sinusoidal_grid(n, n, amp=0.05)
        M = _interior(orc.metrics(s, g.x, g.y, g.bc, g.period))
        Lx, Ly = g.period
        s_, t_ = np.meshgrid(np.arange(n) / n, np.arange(n) / n)
        hx = hy = 1.0 / n
        x_xi = Lx * hx * np.ones_like(s_)
        x_eta = Lx * 0.05 * 2 * np.pi * np.cos(2 * np.pi * t_) * hy
        y_xi = Ly * 0.05 * 2 * np.pi * np.cos(2 * np.pi * s_) * hx
        y_eta = Ly * hy * np.ones_like(s_)
        jinv = x_xi * y_eta - x_eta * y_xi
        e = max(np.abs(M[0] - y_eta).max(), np.abs(M[1] + x_eta).max(), np.abs(M[2] + y_xi).max(),
                np.abs(M[3] - x_xi).max(), np.abs(M[4] - jinv).max() / hx)
        errs.append(e / hx)
    rate = np.log2(errs[0] / errs[1])
    assert rate > order - 0.3, (errs, rate)


def test_periodic_band_is_exact_copy_and_midpoints_interpolate(orc):
    g = W.periodic_grid(16, 12, A=0.2, seed=5)
    G = 4
    for s in SCHEMES:
        M = orc.metrics(s, g.x, g.y, g.bc, g.period)
        inner = M[:, G:-G, G:-G]
        # band columns/rows are bitwise copies of the wrapped interior
        np.testing.assert_array_equal(M[:, G:-G, :G], inner[:, :, -G:])
        np.testing.assert_array_equal(M[:, G:-G, -G:], inner[:, :, :G])
        np.testing.assert_array_equal(M[:, :G, G:-G], inner[:, -G:, :])
        # midpoint metric = interpolation of nodal metric along its own direction
        j, i = 3, 5
        gx = np.array([M[0, G + j, G + i + l] for l in range(-2, 4)])
        assert M[5, G + j, G + i] == pytest.approx(orc.interp_mid(gx), abs=1e-16)
        ge = np.array([M[3, G + j + l, G + i] for l in range(-2, 4)])
        assert M[8, G + j, G + i] == pytest.approx(orc.interp_mid(ge), abs=1e-16)


# ---------------------------------------------------------------------------
# free-stream preservation
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("s", SCHEMES)
@pytest.mark.parametrize("n", [64, 128])
def test_free_stream_preserved_on_randomized_periodic_grid(orc, s, n):
    """Sec. 5.2: uniform flow stays uniform to round-off on a randomized grid
    when the metrics use the scheme's own central operator."""
    g, U = W.fsp_problem(n, A=0.2)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    d = orc.rhs(s, U, M, g.bc)
    assert np.abs(d).max() < 1e-11


@pytest.mark.parametrize("s", SCHEMES)
def test_free_stream_preserved_on_bounded_randomized_grid(orc, s):
    g = W.bounded_grid(96, 80, (0, 1, 0, 1), A=0.2, seed=3)
    U = W.uniform_flow(g, mach=0.5, angle=0.3)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    assert np.abs(orc.rhs(s, U, M, g.bc)).max() < 1e-11


def test_negative_control_inconsistent_metrics_break_fsp(orc):
    """Building the metrics with another scheme's central operator violates
    the consistency requirement of Sec. 2.3 and leaves an O(h^q) residual."""
    g, U = W.fsp_problem(64, A=0.2)
    M = orc.metrics("3-1MP", g.x, g.y, g.bc, g.period)
    assert np.abs(orc.rhs("5-2MP", U, M, g.bc)).max() > 1e-6


def _read_table4():
    out = {}
    with open(os.path.join(GOLDEN, "table4_fsp.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            a, b = line.split()
            out[a] = float(b)
    return out


@pytest.mark.parametrize("s", SCHEMES)
def test_table4_fsp_randomized_81(orc, s):
    """Sec. 5.2, Table 4: Mach 0.5 uniform flow, 81 x 81 grid on [-8, 8]^2 with
    A = 0.45 and four uniform boundary layers, dt = 0.01 to t = 10.  The paper
    prints L2(v) ~ 2e-15; the oracle must stay at that round-off level."""
    ref = _read_table4()[s]
    g = W.bounded_grid(81, 81, (-8, 8, -8, 8), A=0.45, seed=81, layers=4)
    U = W.uniform_flow(g, mach=0.5, angle=0.0)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    Un = orc.rk3_run(s, U, M, 0.01, 1000, g.bc)
    v = Un[2] / Un[0]
    l2 = np.sqrt(np.mean(v ** 2))
    assert l2 < 10 * ref, (l2, ref)
    assert np.abs(Un - U).max() < 1e-12


# ---------------------------------------------------------------------------
# conservation and symmetry
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("s", SCHEMES)
def test_conservation_telescopes_on_periodic_grid(orc, s):
    """Eq. 3.2: with periodic boundaries the fluxes telescope, so
    sum_ij J^-1 dQ/dt = 0 to round-off."""
    g, U = W.vortex_problem(48, A=0.2)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    d = orc.rhs(s, U, M, g.bc)
    jinv = _interior(M)[4]
    tot = (d * jinv[None]).sum(axis=(1, 2))
    scale = (np.abs(d) * jinv[None]).sum(axis=(1, 2))
    assert np.all(np.abs(tot) < 1e-13 * scale), tot / scale


@pytest.mark.parametrize("s", SCHEMES)
def test_transpose_symmetry(orc, s):
    """Swapping x <-> y together with i <-> j and (rho u) <-> (rho v)
    transposes dQ/dt."""
    g, U = W.vortex_problem(32, A=0.2, seed=9)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    d = orc.rhs(s, U, M, g.bc)
    xt, yt = np.ascontiguousarray(g.y.T), np.ascontiguousarray(g.x.T)
    Ut = np.ascontiguousarray(np.stack([U[0].T, U[2].T, U[1].T, U[3].T]))
    Mt = orc.metrics(s, xt, yt, g.bc, g.period[::-1])
    dt_ = orc.rhs(s, Ut, Mt, g.bc)
    back = np.stack([dt_[0].T, dt_[2].T, dt_[1].T, dt_[3].T])
    scale = np.abs(d).max(axis=(1, 2), keepdims=True)
    assert np.all(np.abs(back - d) <= 1e-12 * scale)


@pytest.mark.parametrize("s", SCHEMES)
def test_mirror_symmetry(orc, s):
    """x -> -x with the i index reversed and u -> -u mirrors dQ/dt (the
    h^- half of the scheme is the mirror image of the h^+ half)."""
    g, U = W.vortex_problem(32, A=0.2, seed=4)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    d = orc.rhs(s, U, M, g.bc)
    xm = np.ascontiguousarray(-g.x[:, ::-1])
    ym = np.ascontiguousarray(g.y[:, ::-1])
    Um = np.ascontiguousarray(np.stack([U[0][:, ::-1], -U[1][:, ::-1], U[2][:, ::-1], U[3][:, ::-1]]))
    Mm = orc.metrics(s, xm, ym, g.bc, g.period)
    dm = orc.rhs(s, Um, Mm, g.bc)
    back = np.stack([dm[0][:, ::-1], -dm[1][:, ::-1], dm[2][:, ::-1], dm[3][:, ::-1]])
    scale = np.abs(d).max(axis=(1, 2), keepdims=True)
    assert np.all(np.abs(back - d) <= 1e-12 * scale)


def test_strip_equals_rows_of_a_cartesian_grid(orc):
    """On a Cartesian grid with data independent of y the eta sweep cancels
    exactly and every row equals the one-row (strip) computation."""
    n = 40
    s = "5-2MP"
    gs = W.strip_grid(n)
    Us = W.sod_state(gs)
    Ms = orc.metrics(s, gs.x, gs.y, gs.bc, gs.period)
    ds = orc.rhs(s, Us, Ms, gs.bc)
    h = 1.0 / n
    ny = 8
    x = np.repeat(gs.x, ny, axis=0)
    y = np.repeat((np.arange(ny) * h)[:, None], n, axis=1)
    U2 = np.ascontiguousarray(np.repeat(Us, ny, axis=1))
    M2 = orc.metrics(s, x, y, ("transmissive", "periodic"), (0.0, ny * h))
    d2 = orc.rhs(s, U2, M2, ("transmissive", "periodic"))
    for j in range(ny):
        np.testing.assert_allclose(d2[:, j, :], ds[:, 0, :], rtol=0, atol=1e-12 * np.abs(ds).max())


# ---------------------------------------------------------------------------
# Sod shock tube against the exact Riemann solution
# ---------------------------------------------------------------------------

def sod_exact(x, t, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), x0=0.5, g=GAMMA):
    """Exact solution of the 1-D Riemann problem (ideal gas): pressure
    function root for p*, then sampling of the self-similar waves."""
    rL, uL, pL = left
    rR, uR, pR = right
    cL, cR = np.sqrt(g * pL / rL), np.sqrt(g * pR / rR)

    def fk(p, r, pk, ck):
        if p > pk:
            A, B = 2 / ((g + 1) * r), (g - 1) / (g + 1) * pk
            return (p - pk) * np.sqrt(A / (p + B))
        return 2 * ck / (g - 1) * ((p / pk) ** ((g - 1) / (2 * g)) - 1)

    ps = brentq(lambda p: fk(p, rL, pL, cL) + fk(p, rR, pR, cR) + uR - uL, 1e-8, 10.0, xtol=1e-14)
    us = 0.5 * (uL + uR) + 0.5 * (fk(ps, rR, pR, cR) - fk(ps, rL, pL, cL))
    out = np.zeros((3, x.size))
    for k, xi in enumerate((x - x0) / t):
        if xi < us:  # left of contact
            if ps > pL:
                rs = rL * ((ps / pL + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pL + 1))
                S = uL - cL * np.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
                out[:, k] = (rL, uL, pL) if xi < S else (rs, us, ps)
            else:
                rs = rL * (ps / pL) ** (1 / g)
                cs = cL * (ps / pL) ** ((g - 1) / (2 * g))
                if xi < uL - cL:
                    out[:, k] = (rL, uL, pL)
                elif xi > us - cs:
                    out[:, k] = (rs, us, ps)
                else:
                    u = 2 / (g + 1) * (cL + (g - 1) / 2 * uL + xi)
                    c = 2 / (g + 1) * (cL + (g - 1) / 2 * (uL - xi))
                    r = rL * (c / cL) ** (2 / (g - 1))
                    out[:, k] = (r, u, pL * (c / cL) ** (2 * g / (g - 1)))
        else:
            if ps > pR:
                rs = rR * ((ps / pR + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pR + 1))
                S = uR + cR * np.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
                out[:, k] = (rs, us, ps) if xi < S else (rR, uR, pR)
            else:
                rs = rR * (ps / pR) ** (1 / g)
                cs = cR * (ps / pR) ** ((g - 1) / (2 * g))
                if xi > uR + cR:
                    out[:, k] = (rR, uR, pR)
                elif xi < us + cs:
                    out[:, k] = (rs, us, ps)
                else:
                    u = 2 / (g + 1) * (-cR + (g - 1) / 2 * uR + xi)
                    c = 2 / (g + 1) * (cR - (g - 1) / 2 * (uR - xi))
                    r = rR * (c / cR) ** (2 / (g - 1))
                    out[:, k] = (r, u, pR * (c / cR) ** (2 * g / (g - 1)))
    return out, ps, us


def test_exact_sod_solver_textbook_values():
    _, ps, us = sod_exact(np.array([0.5]), 0.2)
    assert ps == pytest.approx(0.30313, abs=1e-5)
    assert us == pytest.approx(0.92745, abs=1e-5)


def run_sod(orc, s, n, tend=0.2, cfl=0.5):
    g = W.strip_grid(n)
    U = W.sod_state(g)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    t = 0.0
    while t < tend - 1e-14:
        dt = orc.cfl_dt(U, M, cfl)
        dt = min(dt, tend - t)
        U = orc.rk3_step(s, U, M, dt, g.bc)
        t += dt
    return g, U


@pytest.mark.parametrize("s", SCHEMES)
def test_sod_matches_exact_riemann_solution(orc, s):
    """Sec. 6.2(1) (with the [0,1], 200-point, t = 0.2 setup): positivity and
    L1 density error <= 1e-2 against the exact solution."""
    g, U = run_sod(orc, s, 200)
    rho, u, v, p = W.primitive(U)
    assert np.all(np.isfinite(U)) and rho.min() > 0 and p.min() > 0
    ex, _, _ = sod_exact(g.x[0], 0.2)
    l1 = np.mean(np.abs(rho[0] - ex[0]))
    assert l1 < 1e-2, l1


@pytest.mark.slow
def test_sod_converges_under_refinement(orc):
    errs = []
    for n in (200, 400, 800):
        g, U = run_sod(orc, "5-2MP", n)
        ex, _, _ = sod_exact(g.x[0], 0.2)
        errs.append(np.mean(np.abs(W.primitive(U)[0][0] - ex[0])))
    assert errs[0] > errs[1] > errs[2], errs


# ---------------------------------------------------------------------------
# design order on the isentropic vortex (Sec. 6.3(1))
# ---------------------------------------------------------------------------

def _vortex_exact_rate(g):
    """dQ/dt of the translating vortex, -(u0 d/dx + v0 d/dy) Q0, by complex
    step differentiation of the initial state."""
    h = 1e-30
    c = np.sqrt(GAMMA)
    u0, v0 = 0.5 * c * np.cos(np.pi / 4), 0.5 * c * np.sin(np.pi / 4)
    dx = (W.vortex_state(g.x + 1j * h, g.y + 0j).imag) / h
    dy = (W.vortex_state(g.x + 0j, g.y + 1j * h).imag) / h
    return -(u0 * dx + v0 * dy)


@pytest.mark.parametrize("s,order", [("3-1MP", 3), ("3-2MP", 3), ("5-1MP", 5), ("5-2MP", 5)])
def test_design_order_on_vortex(orc, s, order):
    """The residual's truncation error on a smooth curvilinear grid decays at
    the design order (measured within r <= 4 of the vortex centre)."""
    errs = []
    for n in (48, 96):
        g = W.sinusoidal_grid(n, n, amp=0.03)
        U = W.vortex_state(g.x, g.y)
        M = orc.metrics(s, g.x, g.y, g.bc, g.period)
        d = orc.rhs(s, U, M, g.bc)
        ex = _vortex_exact_rate(g)
        r = np.hypot(g.x - 5, g.y - 5)
        errs.append(np.abs(d - ex)[:, r <= 4].max())
    rate = np.log2(errs[0] / errs[1])
    assert rate > order - 0.5, (errs, rate)


def test_rk3_is_third_order_in_time(orc):
    """TVD-RK3: halving dt divides the time-integration error by ~8."""
    g, U0 = W.vortex_problem(32, A=0.0)
    M = orc.metrics("5-2MP", g.x, g.y, g.bc, g.period)
    T = 0.4
    sols = []
    for nsteps in (16, 32, 64, 128):
        sols.append(orc.rk3_run("5-2MP", U0, M, T / nsteps, nsteps, g.bc))
    e = [np.abs(sols[k] - sols[k + 1]).max() for k in range(3)]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    # the rate approaches 3 from above as dt -> 0 (3.29, 3.14 here)
    assert np.all(np.abs(rates - 3) < 0.35) and rates[-1] < rates[0], rates


def test_line_eigenvalues_are_line_maxima(orc):
    """Sec. 2.3: one Lax-Friedrichs eigenvalue per grid line, alpha times the
    maximum of |U^| + c|k^| over that line."""
    g, U = W.vortex_problem(24, A=0.2)
    M = orc.metrics("5-2MP", g.x, g.y, g.bc, g.period)
    _, lx, le = orc.rhs("5-2MP", U, M, g.bc, return_lambda=True)
    rho, u, v, p = W.primitive(U)
    c = np.sqrt(GAMMA * p / rho)
    Mi = _interior(M)
    sx = np.abs(Mi[0] * u + Mi[1] * v) + c * np.hypot(Mi[0], Mi[1])
    se = np.abs(Mi[2] * u + Mi[3] * v) + c * np.hypot(Mi[2], Mi[3])
    np.testing.assert_allclose(lx, 1.1 * sx.max(axis=1), rtol=1e-14)
    np.testing.assert_allclose(le, 1.1 * se.max(axis=0), rtol=1e-14)
