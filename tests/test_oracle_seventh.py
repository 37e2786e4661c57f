"""Pins of the oracle's seventh-order WENOIU family (Appendix): the four
schemes with one, two, four and six midpoints, their eighth-order central
operators, the r = 4 WENO interpolation of Table A1 with the fourth-order
mapping, and the 2-D residual built from them.

The Appendix prints two garbled coefficients.  The central-scheme
decomposition (Eq. 2.7), which ties every h to its separately printed
delta^{c,(1)}, fixes them: 7-2MP's f_j coefficient is -93 (printed -92) and
7-6MP's node term is 3840 f_j (printed 3840 f_{j-1}).  The tests show the
printed forms violate Eq. 2.7 and consistency while the corrected ones
satisfy them.
"""
import math
import os
import sys

import numpy as np
import pytest

from paper_1810_11103_amd import workloads as W

sys.path.insert(0, os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle"))
import derive_weno_is  # noqa: E402

SEVENTH = ["7-1MP", "7-2MP", "7-4MP", "7-6MP"]


def _hp(orc, s, fn, Fn, i):
    """h^+_{i+1/2} from nodal fn(m) and midpoint Fn(m) = f_{m+1/2}."""
    f = np.array([fn(i + m) for m in range(-3, 4)])
    F = np.array([Fn(i + m) for m in range(-3, 3)])
    return orc.hplus(s, f, F)


def _hm(orc, s, fn, Fn, i):
    """h^-_{i+1/2}: h^+ mirrored about i+1/2 (node i+m <-> i+1-m, midpoint
    i+1/2+m <-> i+1/2-m)."""
    f = np.array([fn(i + 1 - m) for m in range(-3, 4)])
    F = np.array([Fn(i - m) for m in range(-3, 3)])
    return orc.hplus(s, f, F)


# the printed (garbled) variants, as corrections to the oracle's h^+
def _printed_extra(s, fn, Fn, i):
    if s == "7-2MP":
        return fn(i) / 1260.0                      # -92 f_j instead of -93 f_j
    if s == "7-6MP":
        return 3840.0 / 26880.0 * (fn(i - 1) - fn(i))  # 3840 f_{j-1} instead of 3840 f_j
    return 0.0


@pytest.mark.parametrize("s", SEVENTH)
def test_central_scheme_decomposition(orc, s):
    """Eq. 2.7 for the Appendix schemes: (D+ + D-)/2 equals the printed
    eighth-order delta^{c,(1)}, with the two corrections."""
    rng = np.random.default_rng(17)
    for _ in range(20):
        nodes = rng.standard_normal(9)   # m = -4..4
        mids = rng.standard_normal(8)    # m + 1/2, m = -4..3
        fn = lambda m: nodes[m + 4]
        Fn = lambda m: mids[m + 4]
        dp = _hp(orc, s, fn, Fn, 0) - _hp(orc, s, fn, Fn, -1)
        dm = _hm(orc, s, fn, Fn, 0) - _hm(orc, s, fn, Fn, -1)
        assert 0.5 * (dp + dm) == pytest.approx(orc.delta_c(s, nodes, mids), abs=1e-13)


@pytest.mark.parametrize("s", ["7-2MP", "7-6MP"])
def test_printed_coefficients_break_the_order(orc, s):
    """The coefficients as printed lose the design order: D+ of a quadratic
    (exact nodal and midpoint values) is no longer exact, while the corrected
    h gives it to round-off.  7-2MP as printed is not even consistent (h of a
    constant differs from it) -- the evidence for the reading."""
    if s == "7-2MP":
        one = lambda m: 1.0
        assert abs(_hp(orc, s, one, one, 0) + _printed_extra(s, one, one, 0) - 1.0) > 1e-4
    fn = lambda m: float(m) ** 2
    Fn = lambda m: (m + 0.5) ** 2
    hp = lambda i: _hp(orc, s, fn, Fn, i) + _printed_extra(s, fn, Fn, i)
    assert abs(hp(0) - hp(-1)) > 1e-4
    assert abs(_hp(orc, s, fn, Fn, 0) - _hp(orc, s, fn, Fn, -1)) < 1e-12


@pytest.mark.parametrize("s", SEVENTH)
def test_upwind_biased_order_seven(orc, s):
    """D+ f_0 = h_{1/2} - h_{-1/2} is exact for polynomials of degree <= 7 when
    the midpoint values are exact (seventh order), and not for degree 8."""
    for n in range(0, 9):
        fn = lambda m: float(m) ** n
        Fn = lambda m: (m + 0.5) ** n
        dp = _hp(orc, s, fn, Fn, 0) - _hp(orc, s, fn, Fn, -1)
        exact = 1.0 if n == 1 else 0.0
        if n <= 7:
            assert dp == pytest.approx(exact, abs=1e-9), (n, dp)
        else:
            assert abs(dp - exact) > 1e-6, n


@pytest.mark.parametrize("s", SEVENTH)
def test_delta_c_order_eight(orc, s):
    """delta^{c,(1)} is exact for polynomials of degree <= 8, not 9."""
    for n in range(0, 10):
        nodes = np.array([float(m) ** n for m in range(-4, 5)])
        mids = np.array([(m + 0.5) ** n for m in range(-4, 4)])
        exact = 1.0 if n == 1 else 0.0
        d = orc.delta_c(s, nodes, mids)
        if n <= 8:
            assert d == pytest.approx(exact, abs=1e-7), (n, d)
        else:
            assert abs(d - exact) > 1e-3, n


def test_table_A1_candidates_and_linear_weights(orc):
    """Each candidate of Table A1 interpolates cubics exactly at x_{j+1/2};
    with the linear weights (the limit of large eps, no mapping) they combine
    into the seven-point interpolation, exact for degree <= 6."""
    x = np.arange(-3, 4, dtype=float)   # nodes j-3..j+3 at 0 = x_j
    for n in range(0, 8):
        v = x ** n
        lin = orc.weno(4, v, eps=1e30, ppm=0)
        if n <= 6:
            assert lin == pytest.approx(0.5 ** n, abs=1e-12), n
        else:
            assert abs(lin - 0.5 ** n) > 1e-6
    # a cubic: every candidate is exact, so any weights give the exact value
    v = 0.3 * x ** 3 - x ** 2 + 2.0 * x - 0.7
    exact = 0.3 * 0.125 - 0.25 + 1.0 - 0.7
    assert orc.weno(4, v) == pytest.approx(exact, abs=1e-13)


def test_r4_indicators_match_their_derivation(orc):
    """The oracle's r = 4 indicators equal the exact Jiang-Shu quadratic forms,
    and the same derivation reproduces the r = 3 indicators of Eq. 3.22."""
    rng = np.random.default_rng(5)
    Q4 = derive_weno_is.indicators(4)
    Q3 = derive_weno_is.indicators(3)
    for _ in range(10):
        v = rng.standard_normal(7)
        for k in range(4):
            w = v[k:k + 4]
            ref = float(sum(float(Q4[k][a][b]) * w[a] * w[b] for a in range(4) for b in range(4)))
            assert orc.smoothness4(k, *w) == pytest.approx(ref, rel=1e-12, abs=1e-12)
        for k in range(3):
            w = v[k:k + 3]
            ref = float(sum(float(Q3[k][a][b]) * w[a] * w[b] for a in range(3) for b in range(3)))
            assert orc.smoothness(k, *w) == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_r4_indicators_share_their_leading_term(orc):
    """For smooth data every r = 4 indicator is (f' h)^2 (1 + O(h^2)), which is
    what makes the nonlinear weights approach the linear ones."""
    f = lambda x: np.sin(1.3 * x + 0.4)
    fp = lambda x: 1.3 * np.cos(1.3 * x + 0.4)
    prev = None
    for h in (0.1, 0.05, 0.025):
        v = f(h * np.arange(-3, 4))
        r = np.array([orc.smoothness4(k, *v[k:k + 4]) for k in range(4)]) / (fp(0.0) * h) ** 2
        dev = np.abs(r - 1.0).max()
        if prev is not None:
            assert dev < prev / 3.0
        prev = dev
    assert prev < 1e-2


def test_ppm4_identities(orc):
    """Fourth-order mapping (Appendix): g(0) = 0, g(C) = C, g(1) = 1 and
    g', g'', g''' vanish at C (flat to fourth order)."""
    for C in (1.0 / 64, 21.0 / 64, 35.0 / 64, 7.0 / 64):
        assert orc.ppm(4, 0.0, C) == pytest.approx(0.0, abs=1e-15)
        assert orc.ppm(4, C, C) == pytest.approx(C, abs=1e-15)
        assert orc.ppm(4, 1.0, C) == pytest.approx(1.0, abs=1e-14)
        h = 1e-3
        for sgn in (-1.0, 1.0):
            assert abs(orc.ppm(4, C + sgn * h, C) - C) < 10 * h ** 4 / min(C, 1 - C) ** 3
        ws = np.linspace(0.0, 1.0, 201)
        g = np.array([orc.ppm(4, w, C) for w in ws])
        assert np.all(np.diff(g) >= -1e-15)


def test_weno7_design_order_on_smooth_data(orc):
    """With the mapping, the nonlinear r = 4 interpolation converges at
    seventh order to the midpoint value of smooth data (no critical point)."""
    f = lambda x: np.exp(0.7 * x) + 0.3 * np.sin(2.0 * x)
    errs = []
    for h in (0.2, 0.1, 0.05):
        v = f(h * np.arange(-3, 4))
        errs.append(abs(orc.weno(4, v) - f(0.5 * h)))
    assert errs[0] / errs[1] > 80 and errs[1] / errs[2] > 90, errs


@pytest.mark.parametrize("s", SEVENTH)
def test_linear_advection_converges_at_seventh_order(orc, s):
    """Sec. 5.1's problem (no printed table for these schemes): u_t + u_x = 0
    on [-1, 1), t = 2, RK4 with dt = dx^{7/4}; the L2 error falls like dx^7."""
    e = [orc.adv1d_run(s, N, dtpow=1.75)[0] for N in (20, 40, 80)]
    orders = [math.log2(e[0] / e[1]), math.log2(e[1] / e[2])]
    assert orders[1] > 6.3, (e, orders)


@pytest.mark.parametrize("s", SEVENTH)
def test_free_stream_preservation(orc, s):
    """Sec. 5.2 with the seventh-order metrics: uniform flow on randomized
    periodic and bounded grids keeps dU/dt at round-off."""
    g, U = W.fsp_problem(40, A=0.2)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    assert np.abs(orc.rhs(s, U, M, g.bc)).max() < 1e-11
    g = W.bounded_grid(36, 28, (0, 1, 0, 1), A=0.2, seed=2)
    U = W.uniform_flow(g)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    assert np.abs(orc.rhs(s, U, M, g.bc)).max() < 1e-10


@pytest.mark.parametrize("s", SEVENTH)
def test_conservation_telescopes(orc, s):
    """Eq. 3.2: periodic fluxes telescope, sum_ij J^-1 dQ/dt = 0 to round-off."""
    g, U = W.vortex_problem(40, A=0.2)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    d = orc.rhs(s, U, M, g.bc)
    jinv = M[4][4:-4, 4:-4]
    tot = (d * jinv[None]).sum(axis=(1, 2))
    scale = (np.abs(d) * jinv[None]).sum(axis=(1, 2))
    assert np.all(np.abs(tot) < 1e-13 * scale)


def test_eight_point_midpoint_interpolation(orc):
    """The seventh-order schemes' metric interpolation is the central
    Lagrange one on g_{i-3..i+4}: exact for degree <= 7, not 8."""
    x = np.arange(-3, 5, dtype=float)
    for n in range(0, 9):
        v = orc.interp_mid(x ** n)
        if n <= 7:
            assert v == pytest.approx(0.5 ** n, abs=1e-12), n
        else:
            assert abs(v - 0.5 ** n) > 1e-3


@pytest.mark.parametrize("s", SEVENTH)
def test_metrics_converge_at_eighth_order(orc, s):
    """Sec. 2.3 with the Appendix operators: the metrics of a smooth periodic
    curvilinear grid converge at the order of delta^{c,(1)}, eight."""
    errs = []
    for n in (24, 48):
        g = W.sinusoidal_grid(n, n, amp=0.05)
        M = orc.metrics(s, g.x, g.y, g.bc, g.period)[:, 4:-4, 4:-4]
        Lx, Ly = g.period
        s_, t_ = np.meshgrid(np.arange(n) / n, np.arange(n) / n)
        h = 1.0 / n
        x_eta = Lx * 0.05 * 2 * np.pi * np.cos(2 * np.pi * t_) * h
        y_xi = Ly * 0.05 * 2 * np.pi * np.cos(2 * np.pi * s_) * h
        e = max(np.abs(M[1] + x_eta).max(), np.abs(M[2] + y_xi).max())
        errs.append(e / h)
    assert math.log2(errs[0] / errs[1]) > 7.5, errs


@pytest.mark.parametrize("s", SEVENTH)
def test_residual_converges_at_seventh_order(orc, s):
    """The 2-D residual of a smooth periodic state on a smooth curvilinear
    grid converges at seventh order: the difference between resolutions n and
    2n, sampled at the coarse nodes, falls by about 2^7 per doubling."""
    ds = []
    for n in (32, 64, 128):
        g = W.sinusoidal_grid(n, n, amp=0.05)
        U = W.random_smooth_state(g, seed=1, amp=0.05)
        M = orc.metrics(s, g.x, g.y, g.bc, g.period)
        ds.append(orc.rhs(s, U, M, g.bc))
    e1 = np.abs(ds[1][:, ::2, ::2] - ds[0]).max()
    e2 = np.abs(ds[2][:, ::2, ::2] - ds[1]).max()
    assert math.log2(e1 / e2) > 6.5, (e1, e2)
