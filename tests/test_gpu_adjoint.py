"""The hand-written GPU adjoint against the oracle's tape adjoint and its
dual-number tangent (dot-product identity), on the same seeded inputs.
Bar: normwise 1e-10 per component for the VJP, 1e-11 relative for the
dot-product identity.

Conditioning: with epsilon = 1e-40 the derivative of the WENO weights is
discontinuous at uniform data, so on nearly flat data (the far field of an
isolated vortex, say) last-bit differences of the forward quantities change
the adjoint at O(1): perturbing U by 1e-15 moves the oracle's own adjoint by
1e-1 there.  The parity inputs are therefore either exactly flat away from
discontinuities (both sides then see exactly zero indicators, since the
characteristic deviations of equal states are exactly zero) or carry a smooth
perturbation everywhere (there 1e-15 input noise moves the adjoint by ~5e-12)."""
import sys

import numpy as np
import pytest

from paper_1810_11103_amd import workloads as W

pytestmark = pytest.mark.gpu
SCHEMES = ["3-1MP", "3-2MP", "5-1MP", "5-2MP"]


@pytest.fixture(scope="module")
def wiu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1810_11103_amd import wenoiu
    return wenoiu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64).cuda()


def _case(kind):
    if kind == "vortex":
        g, U = W.vortex_problem(24, A=0.2, seed=3)
        U = U + 0.02 * W.random_smooth_state(g, seed=6, amp=1.0)
    elif kind == "vortex_ragged":
        g = W.periodic_grid(150, 20, (0, 10, 0, 10), A=0.2, seed=4)
        U = W.vortex_periodic_state(g) + 0.02 * W.random_smooth_state(g, seed=7, amp=1.0)
    elif kind == "riemann":
        g = W.bounded_grid(140, 70, (0, 1, 0, 1), A=0.2, seed=5)
        U = W.riemann_state(g)
    else:
        g = W.strip_grid(40)
        U = W.sod_state(g)
    return g, U


def normwise(a, b):
    return np.array([np.abs(a[c] - b[c]).max() / max(np.abs(b[c]).max(), 1e-300) for c in range(4)])


@pytest.mark.parametrize("s", SCHEMES)
@pytest.mark.parametrize("kind", ["vortex", "vortex_ragged", "riemann", "strip"])
def test_rhs_vjp_matches_oracle(orc, wiu, s, kind):
    say("rhs vjp", s, kind)
    g, U = _case(kind)
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    rng = np.random.default_rng(11)
    Gb = rng.standard_normal(U.shape)
    ref = orc.rhs_vjp(s, U, M, Gb, g.bc)
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period)
    out = sol.rhs_vjp(_dev(U), _dev(Gb)).cpu().numpy()
    assert sol.status() == 0
    err = normwise(out, ref)
    assert np.all(err <= 1e-10), err


@pytest.mark.parametrize("s", ["3-1MP", "5-2MP"])
def test_rhs_vjp_dot_product_with_oracle_tangent(orc, wiu, s):
    g, U = _case("riemann")
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    rng = np.random.default_rng(12)
    V = rng.standard_normal(U.shape)
    Wt = rng.standard_normal(U.shape)
    _, tan = orc.rhs_jvp(s, U, V, M, g.bc)
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period)
    ub = sol.rhs_vjp(_dev(U), _dev(Wt)).cpu().numpy()
    a, b = (tan * Wt).sum(), (V * ub).sum()
    assert abs(a - b) <= 1e-11 * np.abs(tan * Wt).sum()


def test_rhs_vjp_is_deterministic(wiu):
    g, U = _case("riemann")
    sol = wiu.Solver(g.x, g.y, "5-2MP", g.bc, g.period)
    rng = np.random.default_rng(3)
    Gb = _dev(rng.standard_normal(U.shape))
    Ud = _dev(U)
    a = sol.rhs_vjp(Ud, Gb).cpu().numpy()
    b = sol.rhs_vjp(Ud, Gb).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("s", ["3-2MP", "5-2MP"])
@pytest.mark.parametrize("stored", [False, True, "record"])
def test_rk3_step_vjp_matches_oracle(orc, wiu, s, stored):
    import torch
    say("rk3 vjp", s, stored)
    g, U = _case("vortex_ragged")
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    dt = 0.5 * orc.cfl_dt(U, M, 0.5)
    rng = np.random.default_rng(13)
    Wt = rng.standard_normal(U.shape)
    ref = orc.rk3_step_vjp(s, U, M, dt, Wt, g.bc)
    sol = wiu.Solver(g.x, g.y, s, g.bc, g.period)
    sol.dt.fill_(dt)
    Ud = _dev(U)
    if stored:
        U1, U2 = torch.empty_like(Ud), torch.empty_like(Ud)
        rec = sol.step_record() if stored == "record" else None
        Uf = Ud.clone()
        sol.rk3_step_stages(Uf, U1, U2, rec=rec)
        # the stage-storing step is the ordinary step
        Uo = Ud.clone()
        sol.rk3_step(Uo)
        assert torch.equal(Uf, Uo)
        out = sol.rk3_step_vjp(Ud, _dev(Wt), U1, U2, rec=rec).cpu().numpy()
        if rec is not None:  # the recorded maxima are the ones the adjoint would recompute
            assert np.array_equal(out, sol.rk3_step_vjp(Ud, _dev(Wt), U1, U2).cpu().numpy())
    else:
        out = sol.rk3_step_vjp(Ud, _dev(Wt)).cpu().numpy()
    assert sol.status() == 0
    err = normwise(out, ref)
    assert np.all(err <= 1e-10), err
