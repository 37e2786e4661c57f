"""Pins of the oracle's scheme options beyond the paper's tested
configuration:

* the free parameter alpha of the one-midpoint families (Eq. 3.5 for
  3-1MP, Eq. 3.17 for 5-1MP, Appendix (1) for 7-1MP), which the paper
  prints but tests only at alpha = 1, with the central operator that Eq. 2.7
  then defines for the metrics;
* the variables the midpoint values are interpolated in (Sec. 2.4):
  characteristic (the paper's choice, Sec. 3.4), conservative or primitive.

The accuracy relations printed after Eqs. 3.5 and 3.17 and the special
members Eq. 3.6 (alpha = 8/9) and Eq. 3.18 (alpha = 32/25) fix the general
forms; Table 1's linear interpolation fixes the component-wise variants.
"""
import math
from math import factorial

import numpy as np
import pytest

from paper_1810_11103_amd import workloads as W
from test_oracle_euler import _vortex_exact_rate, sod_exact

ONE_MP = ["3-1MP", "5-1MP", "7-1MP"]
VARS = ["characteristic", "conservative", "primitive"]


def _hplus_coeffs(orc, s, a):
    """(node coefficients c[m], m = -3..3; midpoint coefficients d[m], m = -3..2)
    of h^+_{i+1/2} from unit vectors."""
    c = np.array([orc.hplus(s, np.eye(7)[k], np.zeros(6), alpha_h=a) for k in range(7)])
    d = np.array([orc.hplus(s, np.zeros(7), np.eye(6)[k], alpha_h=a) for k in range(6)])
    return c, d


def _moment(orc, s, a, n):
    """Coefficient of dx^n f^(n)(x_{i+1/2}) in the Taylor expansion of h^+:
    sum_m c_m (m - 1/2)^n / n! over nodes plus the midpoints' terms."""
    c, d = _hplus_coeffs(orc, s, a)
    nodes = np.arange(-3, 4) - 0.5
    mids = np.arange(-3, 3, dtype=float)
    return (np.dot(c, nodes ** n) + np.dot(d, mids ** n)) / factorial(n)


# ---------------------------------------------------------------------------
# free alpha
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("s", ONE_MP)
def test_general_form_is_affine_and_reduces_to_the_printed_scheme(orc, s):
    """h^+(alpha) is affine in alpha and its midpoint of alpha = 0 and 2 is the
    printed alpha = 1 scheme (Eqs. 3.4, 3.16, Appendix (1))."""
    rng = np.random.default_rng(3)
    for _ in range(10):
        f, F = rng.standard_normal(7), rng.standard_normal(6)
        h0, h1, h2 = (orc.hplus(s, f, F, alpha_h=a) for a in (0.0 + 1e-300, 1.0, 2.0))
        assert 0.5 * (h0 + h2) == pytest.approx(h1, abs=1e-14)


def test_eq_3_6_is_the_member_alpha_8_9(orc):
    c, d = _hplus_coeffs(orc, "3-1MP", 8.0 / 9.0)
    np.testing.assert_allclose(c, [0, 0, -1 / 18, 1 / 6, 0, 0, 0], atol=1e-15)
    np.testing.assert_allclose(d, [0, 0, 0, 8 / 9, 0, 0], atol=1e-15)


def test_eq_3_18_is_the_member_alpha_32_25(orc):
    """Eq. 3.18 drops f_{j+2}; its coefficients must sum to one, which fixes
    the garbled f_j coefficient as -7/60 (the printed 7189/24000 does not)."""
    c, d = _hplus_coeffs(orc, "5-1MP", 32.0 / 25.0)
    np.testing.assert_allclose(c, [0, 1 / 300, -1 / 60, -7 / 60, -3 / 20, 0, 0], atol=1e-15)
    np.testing.assert_allclose(d, [0, 0, 0, 32 / 25, 0, 0], atol=1e-15)
    printed = 32 / 25 + 1 / 300 - 1 / 60 + 7189 / 24000 - 3 / 20
    assert abs(printed - 1.0) > 0.1


@pytest.mark.parametrize("a", [0.5, 8.0 / 9.0, 1.0, 1.3])
def test_accuracy_relation_of_eq_3_5(orc, a):
    """Printed after Eq. 3.5: h = f - dx^2 f''/24 + k3 dx^3 f''' + (3a/128 -
    37/1152) dx^4 f'''' + ...  The printed k3 = (a/16 - 1/12) carries the sign
    slip already recorded for a = 1 (Eq. 3.4 and Tables 2-3 agree with the
    expansion): the expansion gives -(a/16 - 1/12)."""
    s = "3-1MP"
    assert _moment(orc, s, a, 0) == pytest.approx(1.0, abs=1e-14)
    assert _moment(orc, s, a, 1) == pytest.approx(0.0, abs=1e-14)
    assert _moment(orc, s, a, 2) == pytest.approx(-1 / 24, abs=1e-14)
    assert _moment(orc, s, a, 3) == pytest.approx(-(a / 16 - 1 / 12), abs=1e-14)
    assert _moment(orc, s, a, 4) == pytest.approx(3 * a / 128 - 37 / 1152, abs=1e-14)


@pytest.mark.parametrize("a", [0.5, 1.0, 32.0 / 25.0, 1.7])
def test_accuracy_relation_of_eq_3_17(orc, a):
    """Printed after Eq. 3.17: f - dx^2/24 f'' + 7/5760 dx^4 f'''' +
    (45a - 64)/3840 dx^5 f^(5) - (675a - 983)/138240 dx^6 f^(6) + ..."""
    s = "5-1MP"
    expect = {0: 1.0, 1: 0.0, 2: -1 / 24, 3: 0.0, 4: 7 / 5760, 5: (45 * a - 64) / 3840,
              6: -(675 * a - 983) / 138240}
    for n, v in expect.items():
        assert _moment(orc, s, a, n) == pytest.approx(v, abs=1e-14), n


@pytest.mark.parametrize("a", [0.6, 1.0, 1.4])
def test_appendix_one_midpoint_general_form_is_seventh_order(orc, a):
    """Appendix (1), any alpha: the expansion matches Eq. 3.3 through dx^6
    (-1/24, 7/5760, -31/967680 on the even terms, odd terms zero)."""
    s = "7-1MP"
    expect = {0: 1.0, 1: 0.0, 2: -1 / 24, 3: 0.0, 4: 7 / 5760, 5: 0.0, 6: -31 / 967680}
    for n, v in expect.items():
        assert _moment(orc, s, a, n) == pytest.approx(v, abs=1e-14), n
    assert abs(_moment(orc, s, a, 7)) > 1e-9


@pytest.mark.parametrize("s,order", [("3-1MP", 4), ("5-1MP", 6), ("7-1MP", 8)])
def test_eq_2_7_operator(orc, s, order):
    """The Eq. 2.7 construction reproduces the printed central operators at
    alpha = 1 (Eqs. 3.7, 3.19, Appendix (1)); at other alpha it is still
    antisymmetric and exact to its order on polynomials."""
    rng = np.random.default_rng(8)
    for _ in range(10):
        g, gm = rng.standard_normal(9), rng.standard_normal(8)
        assert orc.delta_c_eq27(s, g, gm, alpha_h=1.0) == pytest.approx(orc.delta_c(s, g, gm), abs=1e-14)
    for a in (0.7, 1.25):
        for n in range(order + 2):
            g = np.arange(-4, 5, dtype=float) ** n
            gm = (np.arange(-4, 4) + 0.5) ** n
            d = orc.delta_c(s, g, gm, alpha_h=a)
            exact = 1.0 if n == 1 else 0.0
            if n <= order:
                assert d == pytest.approx(exact, abs=1e-9), (a, n)
        # antisymmetry: a symmetric sequence has zero derivative at 0
        g = np.abs(np.arange(-4, 5, dtype=float)) ** 1.5
        gm = np.abs(np.arange(-4, 4) + 0.5) ** 1.5
        assert abs(orc.delta_c(s, g, gm, alpha_h=a)) < 1e-13


@pytest.mark.parametrize("s", ONE_MP)
def test_free_alpha_keeps_free_stream_preservation(orc, s):
    """Sec. 2.3: the metrics must use the central operator of the scheme
    actually run; with alpha != 1 that is the Eq. 2.7 operator, and FSP holds."""
    g, U = W.fsp_problem(40, A=0.2)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period, alpha_h=0.8)
    assert np.abs(orc.rhs(s, U, M, g.bc, alpha_h=0.8)).max() < 1e-11


def test_free_alpha_changes_the_3_1mp_metrics(orc):
    """For 3-1MP the alpha term of Eq. 3.5 is alpha (F - P3 f), P3 the
    three-point interpolation (-1, 6, 3)/8; with its mirror it averages to the
    four-point central interpolation, not the six-point one of the metrics, so
    the central operator depends on alpha: alpha = 1 metrics under an
    alpha = 0.8 scheme leave O(1e-3) residuals on the jittered grid."""
    s = "3-1MP"
    g, U = W.fsp_problem(40, A=0.2)
    M1 = orc.metrics(s, g.x, g.y, g.bc, g.period)
    assert np.abs(orc.rhs(s, U, M1, g.bc, alpha_h=0.8)).max() > 1e-6


@pytest.mark.parametrize("s", ["5-1MP", "7-1MP"])
def test_free_alpha_leaves_5_and_7_1mp_metrics_unchanged(orc, s):
    """For 5-1MP (7-1MP) the alpha term is alpha (F - P f) with P the five-
    (seven-) point one-sided interpolation; averaged with its mirror that is
    the six- (eight-) point central interpolation the metrics use, so the
    Eq. 2.7 operator, and the metrics, do not depend on alpha."""
    g = W.periodic_grid(24, 20, A=0.2, seed=5)
    M1 = orc.metrics(s, g.x, g.y, g.bc, g.period)
    for a in (0.5, 1.7):
        Ma = orc.metrics(s, g.x, g.y, g.bc, g.period, alpha_h=a)
        assert np.abs(Ma - M1).max() <= 1e-13 * np.abs(M1).max()


@pytest.mark.parametrize("s,order", [("3-1MP", 3), ("5-1MP", 5), ("7-1MP", 7)])
def test_free_alpha_keeps_design_order(orc, s, order):
    """Sec. 5.1's advection test with alpha = 0.8."""
    dtpow = {3: 1.0, 5: 1.25, 7: 1.75}[order]
    e = [orc.adv1d_run(s, N, dtpow=dtpow, alpha_h=0.8)[0] for N in (40, 80)]
    assert math.log2(e[0] / e[1]) > order - 0.4, e


def test_free_alpha_rejected_for_other_schemes(orc):
    g, U = W.fsp_problem(16, A=0.2)
    with pytest.raises(ValueError):
        orc.metrics("5-2MP", g.x, g.y, g.bc, g.period, alpha_h=0.9)


# ---------------------------------------------------------------------------
# interpolation variables
# ---------------------------------------------------------------------------

def _midpoint_state(orc, s, Qs, vars, eps=1e-40, ppm=1):
    """Q^L and Q^R at k+1/2, read off the split fluxes: F(lam = 2) - F(lam = 0)
    = +-Q (F^+- = (E^ +- lam Q)/2)."""
    k = np.array([0.7, 0.2])
    args = dict(eps=eps, ppm=ppm, vars=vars)
    p0, m0 = orc.midpoint_flux(s, Qs, k, k, k, 0.0, **args)
    p2, m2 = orc.midpoint_flux(s, Qs, k, k, k, 2.0, **args)
    return p2 - p0, m0 - m2


def _random_states(rng, n):
    rho = rng.uniform(0.5, 2.0, n)
    u, v = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    p = rng.uniform(0.5, 2.0, n)
    return np.ascontiguousarray(W.conservative(rho, u, v, p).T)


LINEAR_R3 = np.array([3, -20, 90, 60, -5]) / 128.0  # Table 1 candidates with weights C


@pytest.mark.parametrize("vars", ["conservative", "primitive"])
def test_linear_weights_give_table_1_interpolation_of_the_variables(orc, vars):
    """With linear weights (huge eps, no mapping) the component-wise variants
    interpolate each conservative / primitive variable with Table 1's
    five-point combination (3, -20, 90, 60, -5)/128 (mirrored for the right
    value)."""
    rng = np.random.default_rng(4)
    for _ in range(5):
        Qs = _random_states(rng, 8)  # Q_{k-3..k+4}
        QL, QR = _midpoint_state(orc, "5-2MP", Qs, vars, eps=1e30, ppm=0)
        V = Qs if vars == "conservative" else np.stack(W.primitive(Qs.T), axis=1)
        vl = LINEAR_R3 @ V[1:6]
        vr = LINEAR_R3 @ V[2:7][::-1]
        got_l = QL if vars == "conservative" else np.array(W.primitive(QL))
        got_r = QR if vars == "conservative" else np.array(W.primitive(QR))
        np.testing.assert_allclose(got_l, vl, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(got_r, vr, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("s", ["3-1MP", "5-2MP", "7-4MP"])
def test_characteristic_equals_conservative_with_linear_weights(orc, s):
    """A linear interpolation commutes with the projection (R L = I), so with
    linear weights the characteristic and conservative variants coincide."""
    g, U = W.vortex_problem(40, A=0.2)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    a = orc.rhs(s, U, M, g.bc, eps=1e30, ppm=0, vars="characteristic")
    b = orc.rhs(s, U, M, g.bc, eps=1e30, ppm=0, vars="conservative")
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
    c = orc.rhs(s, U, M, g.bc, eps=1e30, ppm=0, vars="primitive")
    assert np.abs(c - a).max() > 1e-8 * np.abs(a).max()


@pytest.mark.parametrize("vars", VARS)
def test_contact_keeps_pressure_and_velocity(orc, vars):
    """An entropy wave (rho varies; u, v, p uniform): every variant
    reconstructs the uniform velocity and pressure at the midpoint."""
    rng = np.random.default_rng(6)
    rho = rng.uniform(0.3, 3.0, 8)
    Qs = np.ascontiguousarray(W.conservative(rho, np.full(8, 0.4), np.full(8, -0.3), np.full(8, 0.9)).T)
    for Q in _midpoint_state(orc, "5-2MP", Qs, vars):
        r, u, v, p = W.primitive(Q)
        assert u == pytest.approx(0.4, abs=1e-14) and v == pytest.approx(-0.3, abs=1e-14)
        assert p == pytest.approx(0.9, abs=1e-13)


@pytest.mark.parametrize("vars", ["conservative", "primitive"])
@pytest.mark.parametrize("s", ["3-2MP", "5-1MP", "7-6MP"])
def test_component_variants_preserve_free_stream(orc, s, vars):
    g, U = W.fsp_problem(40, A=0.2)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    assert np.abs(orc.rhs(s, U, M, g.bc, vars=vars)).max() < 1e-11
    g = W.bounded_grid(36, 28, (0, 1, 0, 1), A=0.2, seed=2)
    U = W.uniform_flow(g)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    assert np.abs(orc.rhs(s, U, M, g.bc, vars=vars)).max() < 1e-11


@pytest.mark.parametrize("vars", ["conservative", "primitive"])
def test_component_variants_conserve(orc, vars):
    s = "5-2MP"
    g, U = W.vortex_problem(40, A=0.2)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    d = orc.rhs(s, U, M, g.bc, vars=vars)
    jinv = M[4][4:-4, 4:-4]
    tot = (d * jinv[None]).sum(axis=(1, 2))
    scale = (np.abs(d) * jinv[None]).sum(axis=(1, 2))
    assert np.all(np.abs(tot) < 1e-13 * scale)


@pytest.mark.parametrize("vars", ["conservative", "primitive"])
@pytest.mark.parametrize("s,order", [("3-1MP", 3), ("5-2MP", 5)])
def test_component_variants_keep_design_order_on_vortex(orc, s, order, vars):
    errs = []
    for n in (48, 96):
        g = W.sinusoidal_grid(n, n, amp=0.03)
        U = W.vortex_state(g.x, g.y)
        M = orc.metrics(s, g.x, g.y, g.bc, g.period)
        d = orc.rhs(s, U, M, g.bc, vars=vars)
        ex = _vortex_exact_rate(g)
        r = np.hypot(g.x - 5, g.y - 5)
        # root-mean-square over r <= 4: the maximum is dominated by a few
        # nodes where the weights switch and converges irregularly
        errs.append(np.sqrt(np.mean((d - ex)[:, r <= 4] ** 2)))
    assert np.log2(errs[0] / errs[1]) > order - 0.5, errs


@pytest.mark.parametrize("vars", ["conservative", "primitive"])
def test_component_variants_capture_sod(orc, vars):
    """Sod at 200 points, t = 0.2 (Sec. 6.2(1) setup): positive, L1 density
    error below 1e-2 against the exact solution."""
    s = "5-2MP"
    g = W.strip_grid(200)
    U = W.sod_state(g)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    t = 0.0
    while t < 0.2 - 1e-14:
        dt = min(orc.cfl_dt(U, M, 0.5), 0.2 - t)
        U = orc.rk3_step(s, U, M, dt, g.bc, vars=vars)
        t += dt
    rho, u, v, p = W.primitive(U)
    assert np.all(np.isfinite(U)) and rho.min() > 0 and p.min() > 0
    ex, _, _ = sod_exact(g.x[0], 0.2)
    assert np.mean(np.abs(rho[0] - ex[0])) < 1e-2


# ---------------------------------------------------------------------------
# WENO-Z weights (Sec. 7 names them; reading: alpha_k = C_k (1 + (tau /
# (eps + IS_k))^2), tau = |IS_0 - IS_2| (r = 3), |IS_0 - IS_1| (r = 2),
# |IS_0 + 3 IS_1 - 3 IS_2 - IS_3| (r = 4), no mapping)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("r,order", [(3, 5), (4, 7)])
def test_weno_z_design_order_including_a_critical_point(orc, r, order):
    """Smooth data with f'(x_k) = 0 at the interpolation node: the Z weights
    (no mapping) keep the design order."""
    f = lambda x: np.cos(2.0 * x) + 0.1 * x ** 3  # f'(0) = 0
    n = 2 * r - 1
    def err(h, **kw):
        v = f(h * np.arange(-(r - 1), r))
        return abs(orc.weno(r, v[:n], **kw) - f(0.5 * h))
    ez = [err(h, weights="z") for h in (0.2, 0.1, 0.05)]
    assert math.log2(ez[1] / ez[2]) > order - 0.6, ez


@pytest.mark.parametrize("r", [2, 3, 4])
def test_weno_z_picks_the_smooth_stencil_at_a_jump(orc, r):
    """Data with a unit jump after k+1: the interpolated value at k+1/2 stays
    within 1e-6 of the smooth side's value (the crossing stencils' weights
    vanish), and uniform data is reproduced."""
    n = {2: 4, 3: 5, 4: 7}[r]
    k = {2: 2, 3: 2, 4: 3}[r]
    v = np.where(np.arange(n) > k + 1, 1.0, 0.0)
    v = v + 0.01 * np.arange(n)  # a gentle slope on both sides
    lin = 0.01 * (k + 0.5)
    assert abs(orc.weno(r, v, weights="z") - lin) < 1e-6
    assert orc.weno(r, np.full(n, 0.7), weights="z") == pytest.approx(0.7, abs=1e-15)


@pytest.mark.parametrize("s,order", [("3-2MP", 3), ("5-1MP", 5), ("7-2MP", 7)])
def test_weno_z_advection_order(orc, s, order):
    dtpow = {3: 1.0, 5: 1.25, 7: 1.75}[order]
    e = [orc.adv1d_run(s, N, dtpow=dtpow, weights="z")[0] for N in (40, 80)]
    assert math.log2(e[0] / e[1]) > order - 0.5, e


@pytest.mark.parametrize("s", ["3-1MP", "5-2MP", "7-4MP"])
def test_weno_z_preserves_free_stream(orc, s):
    g, U = W.fsp_problem(40, A=0.2)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    assert np.abs(orc.rhs(s, U, M, g.bc, weights="z")).max() < 1e-11


# ---------------------------------------------------------------------------
# midpoint flux splittings (Sec. 7 names Steger-Warming and van Leer for the
# midpoint flux; the nodal fluxes keep the Lax-Friedrichs split)
# ---------------------------------------------------------------------------

def _split_pair(orc, Q, k, split):
    """(F+, F-) of one state Q at the midpoint metric k (all window states
    equal Q, so the interpolated states are Q itself)."""
    Qs = np.ascontiguousarray(np.tile(Q, (8, 1)))
    return orc.midpoint_flux("5-2MP", Qs, k, k, k, 0.0, split=split)


def _states(rng, n):
    for _ in range(n):
        rho, p = rng.uniform(0.3, 3.0), rng.uniform(0.2, 3.0)
        c = math.sqrt(1.4 * p / rho)
        m = rng.uniform(-2.5, 2.5)  # normal Mach numbers across both sonic points
        th = rng.uniform(0, 2 * math.pi)
        yield W.conservative(rho, m * c * math.cos(th), m * c * math.sin(th), p).ravel()


@pytest.mark.parametrize("split", ["sw", "vl"])
def test_split_parts_sum_to_the_flux(orc, split):
    """F+ + F- = E^(Q; k): Steger-Warming by the degree-one homogeneity of
    E^, van Leer by construction."""
    rng = np.random.default_rng(12)
    for Q in _states(rng, 200):
        k = rng.uniform(-1.5, 1.5, 2)
        Fp, Fm = _split_pair(orc, Q, k, split)
        E = orc.flux_hat(Q, 1.4, k[0], k[1])
        np.testing.assert_allclose(Fp + Fm, E, rtol=1e-12, atol=1e-12 * np.abs(E).max())


def test_steger_warming_matches_the_one_dimensional_textbook_form(orc):
    """Along k = (kx, 0) with v = 0 the split is the classical 1-D
    Steger-Warming flux (scaled by |kx|): f+- = rho/(2 gamma) [2(gamma-1) l2 +
    l1 + l3, 2(gamma-1) l2 u + l1 (u-c) + l3 (u+c), (gamma-1) l2 u^2 +
    l1 (u-c)^2/2 + l3 (u+c)^2/2 + (3-gamma)(l1 + l3) c^2 / (2(gamma-1))] with
    l = (u-c, u, u+c) split into positive and negative parts."""
    g = 1.4
    rng = np.random.default_rng(2)
    for _ in range(50):
        rho, p, u = rng.uniform(0.3, 3), rng.uniform(0.2, 3), rng.uniform(-3, 3)
        kx = rng.uniform(0.2, 2.0)
        c = math.sqrt(g * p / rho)
        Q = W.conservative(rho, u, 0.0, p).ravel()
        Fp, Fm = _split_pair(orc, Q, np.array([kx, 0.0]), "sw")
        for F, sgn in ((Fp, 1), (Fm, -1)):
            l1, l2, l3 = [0.5 * (x + sgn * abs(x)) for x in (u - c, u, u + c)]
            f = rho / (2 * g) * np.array([
                2 * (g - 1) * l2 + l1 + l3,
                2 * (g - 1) * l2 * u + l1 * (u - c) + l3 * (u + c),
                0.0,
                (g - 1) * l2 * u * u + 0.5 * l1 * (u - c) ** 2 + 0.5 * l3 * (u + c) ** 2
                + (3 - g) * (l1 + l3) * c * c / (2 * (g - 1))])
            np.testing.assert_allclose(F, kx * f, rtol=1e-12, atol=1e-13)


def test_van_leer_limits_and_smoothness(orc):
    """van Leer along n: F+ = E^ for M >= 1 and 0 for M <= -1, continuous at
    M = +-1, with a double root at M = -1 (F+ = O((M+1)^2))."""
    g = 1.4
    rho, p = 1.3, 0.9
    c = math.sqrt(g * p / rho)
    k = np.array([0.6, 0.8])
    def fp(M):
        Q = W.conservative(rho, M * c * 0.6, M * c * 0.8, p).ravel()
        return _split_pair(orc, Q, k, "vl")[0], Q
    for M in (1.0, 1.5):
        F, Q = fp(M)
        np.testing.assert_allclose(F, orc.flux_hat(Q, g, k[0], k[1]), rtol=1e-13)
    F, Q = fp(1.0 - 1e-9)
    np.testing.assert_allclose(F, orc.flux_hat(Q, g, k[0], k[1]), rtol=1e-7)
    assert np.abs(fp(-1.0)[0]).max() == 0.0
    a, b = np.abs(fp(-1 + 1e-3)[0]).max(), np.abs(fp(-1 + 2e-3)[0]).max()
    assert 3.5 < b / a < 4.5


@pytest.mark.parametrize("split", ["sw", "vl"])
@pytest.mark.parametrize("s", ["3-1MP", "5-2MP", "7-6MP"])
def test_splittings_preserve_free_stream(orc, s, split):
    """Sec. 7's claim: another midpoint splitting leaves FSP intact."""
    g, U = W.fsp_problem(40, A=0.2)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    assert np.abs(orc.rhs(s, U, M, g.bc, split=split)).max() < 1e-11


@pytest.mark.parametrize("split", ["sw", "vl"])
def test_splittings_keep_design_order_and_capture_sod(orc, split):
    s = "5-2MP"
    errs = []
    for n in (48, 96):
        g = W.sinusoidal_grid(n, n, amp=0.03)
        U = W.vortex_state(g.x, g.y)
        M = orc.metrics(s, g.x, g.y, g.bc, g.period)
        d = orc.rhs(s, U, M, g.bc, split=split)
        ex = _vortex_exact_rate(g)
        r = np.hypot(g.x - 5, g.y - 5)
        errs.append(np.sqrt(np.mean((d - ex)[:, r <= 4] ** 2)))
    assert np.log2(errs[0] / errs[1]) > 4.5, errs
    g = W.strip_grid(200)
    U = W.sod_state(g)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    t = 0.0
    while t < 0.2 - 1e-14:
        dt = min(orc.cfl_dt(U, M, 0.5), 0.2 - t)
        U = orc.rk3_step(s, U, M, dt, g.bc, split=split)
        t += dt
    rho, u, v, p = W.primitive(U)
    assert np.all(np.isfinite(U)) and rho.min() > 0 and p.min() > 0
    ex, _, _ = sod_exact(g.x[0], 0.2)
    assert np.mean(np.abs(rho[0] - ex[0])) < 1e-2
