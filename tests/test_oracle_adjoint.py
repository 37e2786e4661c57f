"""Pins of the oracle's tangent (dual numbers) and adjoint (tape) of the
residual and of one TVD-RK3 step, metrics held fixed: the dot-product
identity <J v, w> = <v, J^T w> between the two independent modes, and
central finite differences along smooth directions."""
import numpy as np
import pytest

from paper_1810_11103_amd import workloads as W

SCHEMES = ["3-1MP", "3-2MP", "5-1MP", "5-2MP"]


def _case(kind):
    if kind == "vortex":
        g, U = W.vortex_problem(20, A=0.2)
    else:
        g = W.bounded_grid(22, 18, (0, 1, 0, 1), A=0.2, seed=3)
        U = W.riemann_state(g)
    return g, U


def _bump(g, cx, cy, w=1.0):
    r2 = (g.x - cx) ** 2 + (g.y - cy) ** 2
    b = np.exp(-r2 / w)
    return np.stack([b, 0.5 * b, -0.3 * b, 0.8 * b])


@pytest.mark.parametrize("s", SCHEMES)
@pytest.mark.parametrize("kind", ["vortex", "riemann"])
def test_rhs_dot_product_identity(orc, s, kind):
    g, U = _case(kind)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    rng = np.random.default_rng(1)
    V = rng.standard_normal(U.shape)
    Wt = rng.standard_normal(U.shape)
    val, tan = orc.rhs_jvp(s, U, V, M, g.bc)
    assert np.array_equal(val, orc.rhs(s, U, M, g.bc))
    ub = orc.rhs_vjp(s, U, M, Wt, g.bc)
    a, b = (tan * Wt).sum(), (V * ub).sum()
    assert abs(a - b) <= 1e-12 * max(np.abs(tan * Wt).sum(), 1e-300)


@pytest.mark.parametrize("s", ["3-1MP", "5-2MP"])
def test_rk3_step_dot_product_identity(orc, s):
    g, U = _case("vortex")
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    rng = np.random.default_rng(2)
    V = rng.standard_normal(U.shape)
    Wt = rng.standard_normal(U.shape)
    dt = 0.5 * orc.cfl_dt(U, M, 0.5)
    val, tan = orc.rk3_step_jvp(s, U, V, M, dt, g.bc)
    assert np.array_equal(val, orc.rk3_step(s, U, M, dt, g.bc))
    ub = orc.rk3_step_vjp(s, U, M, dt, Wt, g.bc)
    a, b = (tan * Wt).sum(), (V * ub).sum()
    assert abs(a - b) <= 1e-12 * np.abs(tan * Wt).sum()


@pytest.mark.parametrize("s", SCHEMES)
def test_rhs_tangent_matches_central_differences(orc, s):
    """Along a smooth direction inside the vortex core the central difference
    converges to the tangent at second order (h^2 ratio 100 per decade)."""
    g, U = _case("vortex")
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    V = _bump(g, 5.0, 5.5)
    _, tan = orc.rhs_jvp(s, U, V, M, g.bc)
    errs = []
    for h in (1e-4, 1e-5):
        fd = (orc.rhs(s, U + h * V, M, g.bc) - orc.rhs(s, U - h * V, M, g.bc)) / (2 * h)
        errs.append(np.abs(fd - tan).max() / np.abs(tan).max())
    assert errs[1] < 1e-6
    assert errs[0] / errs[1] > 30
