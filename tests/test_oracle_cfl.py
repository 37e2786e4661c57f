"""Pins of the oracle's CFL time step (the reading of the configurations'
"CFL 0.5" for a method the paper runs at fixed dt):

    dt = CFL / max_nodes [ (|U^| + c|xi^|) + (|V^| + c|eta^|) ] / J^{-1}

in 2-D, and the sum over the three directions in 3-D, with hatted metrics.

On an affine grid x = x0 + A (i, j)^T every central metric operator is exact
(it differentiates linear functions exactly), so xi^, eta^ and J^{-1} are
the constants of the cofactor matrix of A and the time step has a closed
form computed here from A alone, never from the oracle's metrics.  Three
kinds of slip fail these tests:
* taking the maximum of each direction separately and adding the maxima
  (the hot-spot states put the xi and eta maxima on different nodes);
* leaving J^{-1} out of one direction (J^{-1} is far from 1 here);
* using |k^| = 1, or c instead of c|k^| (the grids are sheared and
  anisotropic, so |xi^| != |eta^| != 1).
The GPU's time step is checked against the same closed forms.
"""
import numpy as np
import pytest

import oracle as orc
from paper_1810_11103_amd import workloads as W

GAM = 1.4

# sheared, rotated, anisotropic affine maps (columns: d/di, d/dj)
A2 = [np.array([[0.031, 0.011], [-0.007, 0.017]]),
      np.array([[0.5, -0.2], [0.35, 0.9]]) * 1e-2,
      np.array([[2.0e-3, 0.0], [0.0, 7.0e-3]])]


def _affine_grid(A, nx, ny, origin=(0.3, -0.2)):
    jj, ii = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    x = origin[0] + A[0, 0] * ii + A[0, 1] * jj
    y = origin[1] + A[1, 0] * ii + A[1, 1] * jj
    return W.Grid(np.ascontiguousarray(x), np.ascontiguousarray(y), ("transmissive", "transmissive"))


def _hat2(A):
    """Hatted metrics of the affine map: xi^ = (y_eta, -x_eta), eta^ =
    (-y_xi, x_xi), J^{-1} = det A."""
    (x_xi, x_eta), (y_xi, y_eta) = A
    return np.array([y_eta, -x_eta]), np.array([-y_xi, x_xi]), x_xi * y_eta - x_eta * y_xi


def _speed(rho, u, v, p, k):
    c = np.sqrt(GAM * p / rho)
    return abs(k[0] * u + k[1] * v) + c * np.hypot(k[0], k[1])


def _node_sum2(A, prim):
    xi, eta, J = _hat2(A)
    return (_speed(*prim, xi) + _speed(*prim, eta)) / J


@pytest.mark.parametrize("s", ["3-1MP", "5-2MP", "7-4MP"])
@pytest.mark.parametrize("a", range(len(A2)))
def test_uniform_flow_on_affine_grid(s, a):
    A = A2[a]
    g = _affine_grid(A, 23, 19)
    prim = (1.3, 0.4, -0.25, 0.9)
    U = np.stack(W.conservative(*[np.full(g.shape, v) for v in prim]))
    M = orc.metrics(s, g.x, g.y, g.bc, g.period)
    expect = 0.5 / _node_sum2(A, prim)
    assert orc.cfl_dt(U, M, 0.5) == pytest.approx(expect, rel=1e-13)


def _hot_spot_state2(shape):
    """Uniform background, one node with a fast x-velocity and another with a
    fast y-velocity: the two directions' maxima sit on different nodes."""
    base = (1.0, 0.1, 0.05, 1.0)
    hx = (1.0, 3.0, 0.0, 1.0)
    hy = (0.8, 0.0, 2.5, 0.7)
    prim = [np.full(shape, v) for v in base]
    for q, v in zip(prim, hx):
        q[5, 7] = v
    for q, v in zip(prim, hy):
        q[11, 3] = v
    return np.stack(W.conservative(*prim)), (base, hx, hy)


@pytest.mark.parametrize("a", range(len(A2)))
def test_maximum_of_node_sums_not_sum_of_maxima(a):
    A = A2[a]
    g = _affine_grid(A, 17, 16)
    U, states = _hot_spot_state2(g.shape)
    M = orc.metrics("5-2MP", g.x, g.y, g.bc, g.period)
    xi, eta, J = _hat2(A)
    sums = [_node_sum2(A, s) for s in states]
    expect = 0.5 / max(sums)
    got = orc.cfl_dt(U, M, 0.5)
    assert got == pytest.approx(expect, rel=1e-13)
    # the slips this test exists to catch give other values
    sum_of_max = max(_speed(*s, xi) for s in states) / J + max(_speed(*s, eta) for s in states) / J
    assert abs(0.5 / sum_of_max - expect) > 1e-3 * expect
    no_j_eta = max((_speed(*s, xi) / J + _speed(*s, eta)) for s in states)
    assert abs(0.5 / no_j_eta - expect) > 1e-3 * expect


def test_cfl_dt_scales_with_cfl_number_and_state_speed():
    A = A2[0]
    g = _affine_grid(A, 16, 16)
    U, _ = _hot_spot_state2(g.shape)
    M = orc.metrics("5-2MP", g.x, g.y, g.bc, g.period)
    d1 = orc.cfl_dt(U, M, 0.5)
    assert orc.cfl_dt(U, M, 0.25) == pytest.approx(0.5 * d1, rel=1e-15)
    # doubling every velocity and the sound speed (p x 4) halves dt
    U2 = U.copy()
    rho, u, v, p = W.primitive(U)
    U2[:] = np.stack(W.conservative(rho, 2 * u, 2 * v, 4 * p))
    assert orc.cfl_dt(U2, M, 0.5) == pytest.approx(0.5 * d1, rel=1e-13)


# ---- three dimensions -------------------------------------------------------

A3 = [np.array([[0.021, 0.004, -0.003], [0.002, 0.013, 0.005], [-0.004, 0.001, 0.031]]),
      np.diag([3.0e-3, 5.0e-3, 11.0e-3])]


def _affine_grid3(A, nx, ny, nz):
    ii, jj, kk = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64),
                             np.arange(nz, dtype=np.float64), indexing="ij")
    ii, jj, kk = (np.ascontiguousarray(np.transpose(t, (2, 1, 0))) for t in (ii, jj, kk))
    c = [np.ascontiguousarray(0.1 * r + A[r, 0] * ii + A[r, 1] * jj + A[r, 2] * kk) for r in range(3)]
    return W.Grid3(c[0], c[1], c[2], ("transmissive",) * 3, (0.0, 0.0, 0.0))


def _node_sum3(A, prim):
    """sum over directions of (|k^ . u| + c |k^|) / J^{-1}, with k^ the rows of
    J^{-1} A^{-1} (the cofactor metrics of the affine map) and J^{-1} = det A."""
    rho, u, v, w, p = prim
    J = np.linalg.det(A)
    K = J * np.linalg.inv(A)
    c = np.sqrt(GAM * p / rho)
    vel = np.array([u, v, w])
    return sum(abs(K[d] @ vel) + c * np.linalg.norm(K[d]) for d in range(3)) / J


def _state3(shape, prims, spots):
    fields = [np.full(shape, v) for v in prims[0]]
    for (k, j, i), pr in zip(spots, prims[1:]):
        for f, v in zip(fields, pr):
            f[k, j, i] = v
    return np.stack(W.conservative3(*fields))


@pytest.mark.parametrize("a", range(len(A3)))
def test_uniform_flow_on_affine_grid_3d(a):
    A = A3[a]
    g = _affine_grid3(A, 14, 13, 12)
    prim = (1.2, 0.3, -0.2, 0.15, 0.8)
    U = _state3(g.shape, [prim], [])
    M = orc.metrics3("5-2MP", g.x, g.y, g.z, g.bc, g.period)
    assert orc.cfl_dt3(U, M, 0.5) == pytest.approx(0.5 / _node_sum3(A, prim), rel=1e-13)


@pytest.mark.parametrize("a", range(len(A3)))
def test_maximum_of_node_sums_3d(a):
    A = A3[a]
    g = _affine_grid3(A, 14, 13, 12)
    prims = [(1.0, 0.1, 0.05, -0.05, 1.0), (1.0, 3.0, 0.0, 0.0, 1.0), (0.9, 0.0, 2.6, 0.0, 0.8),
             (1.1, 0.0, 0.0, 2.2, 1.2)]
    U = _state3(g.shape, prims, [(6, 5, 7), (3, 9, 4), (8, 2, 10)])
    M = orc.metrics3("5-2MP", g.x, g.y, g.z, g.bc, g.period)
    sums = [_node_sum3(A, pr) for pr in prims]
    expect = 0.5 / max(sums)
    assert orc.cfl_dt3(U, M, 0.5) == pytest.approx(expect, rel=1e-13)
    J = np.linalg.det(A)
    K = J * np.linalg.inv(A)

    def dir_speed(pr, d):
        rho, u, v, w, p = pr
        return (abs(K[d] @ np.array([u, v, w])) + np.sqrt(GAM * p / rho) * np.linalg.norm(K[d])) / J
    sum_of_max = sum(max(dir_speed(pr, d) for pr in prims) for d in range(3))
    assert abs(0.5 / sum_of_max - expect) > 1e-3 * expect


# ---- the GPU time step against the same closed forms -------------------------

@pytest.mark.gpu
@pytest.mark.parametrize("a", range(len(A2)))
def test_gpu_cfl_dt_closed_form(a):
    import torch
    from paper_1810_11103_amd import wenoiu
    A = A2[a]
    g = _affine_grid(A, 40, 36)
    U, states = _hot_spot_state2(g.shape)
    sol = wenoiu.Solver(g.x, g.y, "5-2MP", g.bc, g.period)
    sol.cfl_dt(torch.as_tensor(U).cuda().contiguous(), 0.5)
    expect = 0.5 / max(_node_sum2(A, s) for s in states)
    assert float(sol.dt.item()) == pytest.approx(expect, rel=1e-13)
    assert sol.status() == 0


@pytest.mark.gpu
@pytest.mark.parametrize("a", range(len(A3)))
def test_gpu_cfl_dt_closed_form_3d(a):
    import torch
    from paper_1810_11103_amd import wenoiu
    A = A3[a]
    g = _affine_grid3(A, 20, 18, 16)
    prims = [(1.0, 0.1, 0.05, -0.05, 1.0), (1.0, 3.0, 0.0, 0.0, 1.0), (0.9, 0.0, 2.6, 0.0, 0.8),
             (1.1, 0.0, 0.0, 2.2, 1.2)]
    U = _state3(g.shape, prims, [(6, 5, 7), (3, 9, 4), (8, 2, 10)])
    sol = wenoiu.Solver3(g.x, g.y, g.z, "5-2MP", g.bc, g.period)
    dt = sol.cfl_dt(torch.as_tensor(U).cuda().contiguous(), 0.5)
    expect = 0.5 / max(_node_sum3(A, pr) for pr in prims)
    assert float(torch.as_tensor(dt).reshape(-1)[0].item()) == pytest.approx(expect, rel=1e-13)
    assert sol.status() == 0
