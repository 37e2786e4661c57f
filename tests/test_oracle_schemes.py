"""Pins of the oracle's scheme components against what the paper prints.

Each test compares an oracle routine with an artefact of the paper other than
the formula the routine was typed from (Table 2, the printed accuracy
relations, the central-scheme decomposition, Table 3), or with a property the
mathematics fixes (polynomial exactness, mapping-function identities).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SCHEMES = ["3-1MP", "3-2MP", "5-1MP", "5-2MP"]


def _h_coeffs(orc, s):
    """Coefficients of h^+_{i+1/2} on nodes i-3..i+3 and midpoints
    i-3/2..i+3/2, probed with unit impulses (h^+ is linear in its inputs)."""
    a = np.zeros(7)
    b = np.zeros(4)
    for m in range(7):
        f = np.zeros(7)
        f[m] = 1.0
        a[m] = orc.hplus(s, f, np.zeros(4))
    for m in range(4):
        F = np.zeros(4)
        F[m] = 1.0
        b[m] = orc.hplus(s, np.zeros(7), F)
    return a, b


def _read_table2():
    rows = {}
    with open(os.path.join(GOLDEN, "table2_spectral.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            s, part, expr = line.split(None, 2)
            rows[(s, part)] = expr.strip()
    return rows


@pytest.mark.parametrize("s", SCHEMES)
def test_table2_modified_wavenumber(orc, s):
    """Sec. 4.1, Eq. 4.2 and Table 2: Re/Im of the modified wavenumber of
    D+ f_j = h_{j+1/2} - h_{j-1/2} match the printed closed forms (alpha = 1)."""
    a, b = _h_coeffs(orc, s)
    k = np.linspace(0.0, np.pi, 97)
    node_m = np.arange(-3, 4)
    mid_m = np.arange(-2, 2) + 0.5
    A = (a[None, :] * np.exp(1j * np.outer(k, node_m))).sum(1) + \
        (b[None, :] * np.exp(1j * np.outer(k, mid_m))).sum(1)
    kp = -1j * A * (1.0 - np.exp(-1j * k))
    rows = _read_table2()
    env = {"sin": np.sin, "cos": np.cos, "k": k, "a": 1.0}
    disp = eval(rows[(s, "dispersion")], {}, env)
    diss = eval(rows[(s, "dissipation")], {}, env)
    np.testing.assert_allclose(kp.real, disp, atol=1e-14)
    np.testing.assert_allclose(kp.imag, diss, atol=1e-14)
    # upwind: no amplification of any wave
    assert np.all(kp.imag <= 1e-15)


def _read_accuracy():
    out = {}
    with open(os.path.join(GOLDEN, "accuracy_relations.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            out[parts[0]] = [Fraction(p) for p in parts[1:]]
    return out


# The dx^3 term of the accuracy relation printed for the family Eq. 3.5 reads
# (alpha/16 - 1/12); expanding Eq. 3.5 (and its alpha = 1 member Eq. 3.4)
# gives (1/12 - alpha/16), i.e. +1/48 at alpha = 1.  Table 2's 3-1MP closed
# forms and the Table 3 errors agree with Eq. 3.4 itself, so the printed sign
# of that one term is taken as a typesetting slip.
PRINT_ERRATA = {("3-1MP", 3): Fraction(1, 48)}


@pytest.mark.parametrize("s", SCHEMES)
def test_printed_accuracy_relations(orc, s):
    """Secs. 3.2-3.3: h_{j+1/2} applied to f = x^n / n! (origin at x_{j+1/2},
    unit spacing) gives the printed Taylor coefficient c_n."""
    c = _read_accuracy()[s]
    for n, cn in enumerate(c):
        cn = PRINT_ERRATA.get((s, n), cn)
        f = np.array([(m - 0.5) ** n / math.factorial(n) for m in range(-3, 4)])
        # midpoints f_{i-3/2}, f_{i-1/2}, f_{i+1/2}, f_{i+3/2} sit at x = -2, -1, 0, 1
        F = np.array([(m) ** n / math.factorial(n) for m in (-2, -1, 0, 1)])
        h = orc.hplus(s, f, F)
        assert h == pytest.approx(float(cn), abs=1e-15), (n, h, cn)


def _mirror_D(orc, s, fn, Fm_):
    """D+ and D- at node 0 for nodal values fn(m) and midpoint values Fm_(m)
    = f_{m+1/2}.  D- uses h^- = h^+ mirrored about i+1/2."""
    def hp(i):
        f = np.array([fn(i + m) for m in range(-3, 4)])
        F = np.array([Fm_(i + m) for m in (-2, -1, 0, 1)])
        return orc.hplus(s, f, F)

    def hm(i):  # node i+m <-> i+1-m, midpoint i+1/2+m <-> i+1/2-m
        f = np.array([fn(i + 1 - m) for m in range(-3, 4)])
        F = np.array([Fm_(i - m) for m in (-2, -1, 0, 1)])
        return orc.hplus(s, f, F)
    return hp(0) - hp(-1), hm(0) - hm(-1)


@pytest.mark.parametrize("s", SCHEMES)
def test_central_scheme_decomposition(orc, s):
    """Eq. 2.7: (D+ + D-)/2 built from h^+ (Eqs. 3.4/3.8/3.16/3.20) equals the
    separately printed delta^{c,(1)} (Eqs. 3.7/3.9/3.19/3.21)."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        nodes = rng.standard_normal(9)   # m = -4..4
        mids = rng.standard_normal(8)    # m + 1/2 for m = -4..3
        fn = lambda m: nodes[m + 4]
        Fm_ = lambda m: mids[m + 4]
        dp, dm = _mirror_D(orc, s, fn, Fm_)
        dc = orc.delta_c(s, nodes, mids)
        assert 0.5 * (dp + dm) == pytest.approx(dc, abs=1e-13)


@pytest.mark.parametrize("s,order", [("3-1MP", 4), ("3-2MP", 4), ("5-1MP", 6), ("5-2MP", 6)])
def test_delta_c_order(orc, s, order):
    """delta^{c,(1)} is exact for polynomials of degree <= its order (Sec. 3)."""
    for n in range(order + 1):
        nodes = np.array([float(m) ** n for m in range(-4, 5)])
        mids = np.array([(m + 0.5) ** n for m in range(-4, 4)])
        exact = float(n) * 0.0 ** (n - 1) if n > 0 else 0.0
        assert orc.delta_c(s, nodes, mids) == pytest.approx(exact, abs=1e-12), n
    n = order + 1
    nodes = np.array([float(m) ** n for m in range(-4, 5)])
    mids = np.array([(m + 0.5) ** n for m in range(-4, 4)])
    assert abs(orc.delta_c(s, nodes, mids)) > 1e-6


def test_midpoint_interpolation_exact_to_degree5(orc):
    for n in range(6):
        g = np.array([float(m) ** n for m in range(-2, 4)])
        assert orc.interp_mid(g) == pytest.approx(0.5 ** n, abs=1e-13)
    g = np.array([float(m) ** 6 for m in range(-2, 4)])
    assert abs(orc.interp_mid(g) - 0.5 ** 6) > 1e-3


@pytest.mark.parametrize("s,order", [("3-1MP", 4), ("3-2MP", 4), ("5-1MP", 6), ("5-2MP", 6)])
def test_metric_operator_is_scheme_central_operator(orc, s, order):
    """The combined metric operator (delta^{c,(1)} with interpolated midpoints)
    differentiates polynomials of degree <= order exactly at the node, for
    relative data r_m = g_{i+m} - g_i."""
    x0 = 0.37
    for n in range(1, order + 1):
        g = lambda t: (x0 + t) ** n
        r = np.array([g(m) - g(0) for m in range(-8, 9)])
        assert orc.metric_derivative(s, r) == pytest.approx(n * x0 ** (n - 1), rel=1e-12, abs=1e-12)


def test_is_sum_of_squares_matches_printed_eq_3_22(orc):
    """Eq. 3.22 as printed (expanded quadratic forms) equals the oracle's
    indicators."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        u = rng.standard_normal(5)  # u_{j-2..j+2}
        a, b, c, d, e = u
        is0 = (4 * a * a - 19 * a * b + 25 * b * b + 11 * a * c - 31 * b * c + 10 * c * c) / 3
        is1 = (4 * b * b - 13 * b * c + 13 * c * c + 5 * b * d - 13 * c * d + 4 * d * d) / 3
        is2 = (10 * c * c - 31 * c * d + 25 * d * d + 11 * c * e - 19 * d * e + 4 * e * e) / 3
        assert orc.smoothness(0, a, b, c) == pytest.approx(is0, rel=1e-12, abs=1e-12)
        assert orc.smoothness(1, b, c, d) == pytest.approx(is1, rel=1e-12, abs=1e-12)
        assert orc.smoothness(2, c, d, e) == pytest.approx(is2, rel=1e-12, abs=1e-12)


def test_is_taylor_expansion(orc):
    """Sec. 3.3(3): IS_k = u'^2 dx^2 + (a u' u''' + 13/12 u''^2) dx^4 + O(dx^5)
    with a = -2/3, 1/3, -2/3 (expansion about x_j)."""
    u1, u2, u3 = 0.7, -1.3, 2.1
    f = lambda x: u1 * x + u2 * x * x / 2 + u3 * x ** 3 / 6
    for k, a in zip(range(3), (-2 / 3, 1 / 3, -2 / 3)):
        est = []
        for h in (1e-2, 5e-3):
            pts = [f(h * m) for m in (range(-2, 1), range(-1, 2), range(0, 3))[k]]
            IS = orc.smoothness(k, *pts)
            est.append((IS - u1 * u1 * h * h) / h ** 4)
        target = a * u1 * u3 + 13 / 12 * u2 * u2
        # the remainder is O(dx^5): one Richardson step removes it
        assert 2 * est[1] - est[0] == pytest.approx(target, rel=2e-3), (k, est, target)


@pytest.mark.parametrize("order,C", [(2, 0.25), (2, 0.75), (3, 1 / 16), (3, 10 / 16), (3, 5 / 16)])
def test_ppm_mapping_properties(orc, order, C):
    """Eqs. 3.15 and 3.23: g(0) = 0, g(C) = C, g(1) = 1, g'(C) = 0, monotone."""
    g = lambda w: orc.ppm(order, w, C)
    assert g(0.0) == pytest.approx(0.0, abs=1e-15)
    assert g(C) == pytest.approx(C, abs=1e-15)
    assert g(1.0) == pytest.approx(1.0, abs=1e-14)
    h = 1e-5
    assert (g(C + h) - g(C - h)) / (2 * h) == pytest.approx(0.0, abs=1e-4)
    ws = np.linspace(0, 1, 201)
    vals = np.array([g(w) for w in ws])
    assert np.all(np.diff(vals) >= -1e-15)


@pytest.mark.parametrize("r,order", [(3, 5), (2, 3)])
def test_weno_interpolation_converges_at_design_order(orc, r, order):
    """Table 1 candidates and linear weights: on smooth data (including a
    critical point) the mapped WENO value converges to the midpoint value at
    the design order; the linear combination is the Lagrange interpolant
    (3, -20, 90, 60, -5)/128 (r = 3) or (-1, 6, 3)/8 (r = 2)."""
    f = lambda x: np.sin(1.3 * x + 0.4)
    errs = []
    for h in (0.1, 0.05, 0.025):
        x0 = 0.12 - np.pi / 2  # near the critical point of sin(1.3 x + 0.4)
        v = np.array([f(x0 + h * m) for m in range(-2, 3 if r == 3 else 2)])
        w = orc.weno(r, v)
        errs.append(abs(w - f(x0 + 0.5 * h)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > order - 0.4), rates
    # linear limit
    v = np.array([f(0.3 + 0.01 * m) for m in range(-2, 3 if r == 3 else 2)])
    lag = (np.dot([3, -20, 90, 60, -5], v) / 128) if r == 3 else (np.dot([-1, 6, 3], v[1:]) / 8)
    assert orc.weno(r, v) == pytest.approx(lag, abs=1e-12)


def _read_table3():
    rows = []
    with open(os.path.join(GOLDEN, "table3_linear_advection.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([float(t) for t in line.split()])
    return np.array(rows)


@pytest.mark.parametrize("col,s", list(enumerate(SCHEMES)))
def test_table3_linear_advection(orc, col, s):
    """Sec. 5.1, Table 3: errors of the whole scalar WENOIU operator (WENO +
    PPM + h^+) with RK4 at dt = dx^{5/4}.  With the upwind split the oracle
    reproduces every printed error to within 3 % for N >= 40 (7 % at N = 20,
    15 % at N = 10 where two digits are printed) and the printed orders to
    0.05."""
    tab = _read_table3()
    errs = []
    for row in tab:
        N = int(row[0])
        l2, li = orc.adv1d_run(s, N, split=0)
        errs.append((l2, li))
        p2, pi = row[1 + 2 * col], row[2 + 2 * col]
        tol = 0.03 if N >= 40 else (0.07 if N == 20 else 0.15)
        assert l2 == pytest.approx(p2, rel=tol), (N, l2, p2)
        assert li == pytest.approx(pi, rel=tol), (N, li, pi)
    errs = np.array(errs)
    ours = np.log2(errs[:-1] / errs[1:])
    paper = np.log2(tab[:-1, 1 + 2 * col:3 + 2 * col] / tab[1:, 1 + 2 * col:3 + 2 * col])
    np.testing.assert_allclose(ours[3:], paper[3:], atol=0.05)


def test_lf_split_scalar_converges(orc):
    """With the Lax-Friedrichs split (which also exercises h^- and the
    right-biased interpolation) the scalar operator keeps the design order."""
    for s, order in (("3-1MP", 3), ("5-2MP", 5)):
        e = [orc.adv1d_run(s, N, split=1)[0] for N in (80, 160, 320)]
        rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
        assert np.all(np.abs(rates - order) < 0.2), rates


def test_scalar_operator_mirror_symmetry(orc):
    """h^- is h^+ mirrored about i+1/2 and uses the right-biased
    interpolation: the operator built from f^- = u alone (split weights
    (0, 1)) equals minus the mirror image of the operator built from f^+ = u
    alone applied to the mirrored data."""
    rng = np.random.default_rng(11)
    n = 64
    u = np.sin(2 * np.pi * np.arange(n) / n) + 0.3 * rng.standard_normal(n)
    dx = 2.0 / n
    for s in SCHEMES:
        dm = orc.adv1d_rhs(s, u, dx, split=1, alpha=-1.0)       # f+ = 0, f- = u
        dp = orc.adv1d_rhs(s, u[::-1].copy(), dx, split=0)      # f+ = u, f- = 0
        np.testing.assert_allclose(dm, -dp[::-1], rtol=0, atol=1e-12)
