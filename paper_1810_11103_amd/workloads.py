"""Seeded synthetic grids and initial states (inputs only).

This module builds the inputs shared by the HIP path, the tests and the
benchmark: node coordinates of uniform and randomized curvilinear grids and
conservative initial states of the paper's test problems.  It contains none of
the method's arithmetic (no metrics, fluxes, interpolation or time stepping).

Conventions: arrays are float64, row-major, the xi index i fastest.
Coordinates have shape (ny, nx); states have shape (4, ny, nx) holding
(rho, rho u, rho v, e) with e = p/(gamma-1) + rho (u^2 + v^2)/2 (Sec. 2.1).
"""
from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4


@dataclass
class Grid:
    x: np.ndarray
    y: np.ndarray
    bc: tuple = ("periodic", "periodic")
    period: tuple = (0.0, 0.0)
    spacing: tuple = (1.0, 1.0)
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.x.shape


def conservative(rho, u, v, p, gamma=GAMMA):
    dt = np.result_type(rho, u, v, p, np.float64)  # complex inputs stay complex
    rho, u, v, p = np.broadcast_arrays(*(np.asarray(a, dtype=dt) for a in (rho, u, v, p)))
    e = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, e]))


def primitive(U, gamma=GAMMA):
    rho = U[0]
    u = U[1] / rho
    v = U[2] / rho
    p = (gamma - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


# ---------------------------------------------------------------------------
# Grids (Sec. 6.1)
# ---------------------------------------------------------------------------

def _jitter(nx, ny, A, rng, mask):
    """Sec. 6.1(1): each node is displaced by 2A(Rand(0,1) - 0.5) spacings in
    x or in y, the direction chosen by a fair coin Rand(0|1)."""
    r = rng.random((ny, nx))
    coin = rng.integers(0, 2, size=(ny, nx))
    d = 2.0 * A * (r - 0.5) * mask
    return d * coin, d * (1 - coin)


def periodic_grid(nx, ny, box=(0.0, 10.0, 0.0, 10.0), A=0.0, seed=0):
    """Periodic grid of nx x ny distinct nodes on [x0, x1) x [y0, y1): node
    (i, j) sits at (x0 + i hx, y0 + j hy), hx = (x1-x0)/nx, displaced at every
    node when A > 0 (the images across the period are the same nodes)."""
    x0, x1, y0, y1 = box
    hx, hy = (x1 - x0) / nx, (y1 - y0) / ny
    jj, ii = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    dx = dy = 0.0
    if A > 0:
        rng = np.random.default_rng(seed)
        dx, dy = _jitter(nx, ny, A, rng, np.ones((ny, nx)))
    x = x0 + (ii + dx) * hx
    y = y0 + (jj + dy) * hy
    return Grid(np.ascontiguousarray(x), np.ascontiguousarray(y), ("periodic", "periodic"),
                (x1 - x0, y1 - y0), (hx, hy), {"A": A, "seed": seed})


def bounded_grid(nx, ny, box=(0.0, 1.0, 0.0, 1.0), A=0.0, seed=0, layers=4):
    """Non-periodic grid with nodes from x0 to x1 inclusive, displaced by A
    spacings except in `layers` uniform node layers along every boundary
    (Sec. 6.1(1) and (3); the 'or' of Sec. 6.1(1) is read as 'and')."""
    x0, x1, y0, y1 = box
    hx, hy = (x1 - x0) / (nx - 1), (y1 - y0) / (ny - 1)
    jj, ii = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    dx = dy = 0.0
    if A > 0:
        rng = np.random.default_rng(seed)
        iv = np.arange(nx)
        jv = np.arange(ny)
        mi = (iv >= layers) & (iv < nx - layers)
        mj = (jv >= layers) & (jv < ny - layers)
        mask = (mj[:, None] & mi[None, :]).astype(np.float64)
        dx, dy = _jitter(nx, ny, A, rng, mask)
    x = x0 + (ii + dx) * hx
    y = y0 + (jj + dy) * hy
    return Grid(np.ascontiguousarray(x), np.ascontiguousarray(y), ("transmissive", "transmissive"),
                (0.0, 0.0), (hx, hy), {"A": A, "seed": seed, "layers": layers})


def strip_grid(n, x0=0.0, x1=1.0):
    """One-row grid for 1-D problems: cell centres x_i = x0 + (i + 1/2) h,
    transmissive in x, periodic in y with period h (so every eta line is a
    single repeated node)."""
    h = (x1 - x0) / n
    x = (x0 + (np.arange(n, dtype=np.float64) + 0.5) * h)[None, :]
    y = np.zeros((1, n))
    return Grid(np.ascontiguousarray(x), y, ("transmissive", "periodic"), (0.0, h), (h, h), {})


def line_grid(n, x0=0.0, x1=1.0):
    """One-row node grid for 1-D problems with boundary nodes on x0 and x1:
    x_i = x0 + i h, i = 0..n-1, h = (x1 - x0)/(n - 1); non-periodic in x,
    periodic in y with period h."""
    h = (x1 - x0) / (n - 1)
    x = (x0 + np.arange(n, dtype=np.float64) * h)[None, :]
    y = np.zeros((1, n))
    return Grid(np.ascontiguousarray(x), y, ("transmissive", "periodic"), (0.0, h), (h, h), {})


def sinusoidal_grid(nx, ny, box=(0.0, 10.0, 0.0, 10.0), amp=0.1):
    """Smooth periodic curvilinear grid: x = x0 + L_x[s + a sin(2 pi t)],
    y = y0 + L_y[t + a sin(2 pi s)] with s = i/nx, t = j/ny."""
    x0, x1, y0, y1 = box
    Lx, Ly = x1 - x0, y1 - y0
    jj, ii = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    s, t = ii / nx, jj / ny
    x = x0 + Lx * (s + amp * np.sin(2 * np.pi * t))
    y = y0 + Ly * (t + amp * np.sin(2 * np.pi * s))
    return Grid(np.ascontiguousarray(x), np.ascontiguousarray(y), ("periodic", "periodic"), (Lx, Ly),
                (Lx / nx, Ly / ny), {"amp": amp})


# ---------------------------------------------------------------------------
# Initial states
# ---------------------------------------------------------------------------

def uniform_flow(grid, mach=0.5, angle=np.pi / 4, rho=1.0, p=1.0, gamma=GAMMA):
    c = np.sqrt(gamma * p / rho)
    u = mach * c * np.cos(angle)
    v = mach * c * np.sin(angle)
    shape = grid.x.shape
    return conservative(np.full(shape, rho), np.full(shape, u), np.full(shape, v), np.full(shape, p), gamma)


def vortex_state(x, y, center=(5.0, 5.0), strength=5.0 / (2 * np.pi), alpha=0.5, rc=1.0, mach=0.5,
                 angle=np.pi / 4, gamma=GAMMA):
    """Isentropic vortex of Sec. 6.3(1): (du, dv) = eps r e^{alpha(1-r^2)}
    (sin t, -cos t), dT = -(gamma-1) eps^2 / (4 alpha gamma) e^{2 alpha (1-r^2)},
    on a mean flow rho = p = T = 1 of the given Mach number.  The defaults give
    the classic strength-5 vortex (alpha = 1/2, eps = 5/(2 pi))."""
    c = np.sqrt(gamma)
    u0 = mach * c * np.cos(angle)
    v0 = mach * c * np.sin(angle)
    dx = (x - center[0]) / rc
    dy = (y - center[1]) / rc
    r2 = dx * dx + dy * dy
    f = strength * np.exp(alpha * (1.0 - r2))
    # r sin(theta) = dy, r cos(theta) = dx
    u = u0 + f * dy
    v = v0 - f * dx
    T = 1.0 - (gamma - 1.0) * strength ** 2 / (4.0 * alpha * gamma) * np.exp(2.0 * alpha * (1.0 - r2))
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    return conservative(rho, u, v, p, gamma)


def vortex_periodic_state(grid, t=0.0, **kw):
    """Vortex translated by the mean flow for time t on the periodic box (the
    exact solution of the Euler equations), summing the nearest images."""
    mach = kw.get("mach", 0.5)
    angle = kw.get("angle", np.pi / 4)
    gamma = kw.get("gamma", GAMMA)
    center = kw.get("center", (5.0, 5.0))
    Lx, Ly = grid.period
    c = np.sqrt(gamma)
    cx = center[0] + mach * c * np.cos(angle) * t
    cy = center[1] + mach * c * np.sin(angle) * t
    x0 = grid.x.min() if Lx == 0 else 0.0
    # place the centre inside the box and measure distances to the nearest image
    bx = 0.0 if Lx == 0 else (cx - np.floor((cx - 0.0) / Lx) * Lx)
    by = 0.0 if Ly == 0 else (cy - np.floor((cy - 0.0) / Ly) * Ly)
    dx = grid.x - bx
    dy = grid.y - by
    if Lx:
        dx = dx - Lx * np.round(dx / Lx)
    if Ly:
        dy = dy - Ly * np.round(dy / Ly)
    del x0
    kw2 = {k: v for k, v in kw.items() if k not in ("center",)}
    return vortex_state(dx, dy, center=(0.0, 0.0), **kw2)


# Four-quadrant Riemann problem of Sec. 6.3(3): (rho, u, v, p) per quadrant.
RIEMANN_QUADRANTS = {
    "ne": (1.0, 0.0, -0.3, 1.0),
    "nw": (2.0, 0.0, 0.3, 1.0),
    "sw": (1.0625, 0.0, 0.8145, 0.4),
    "se": (0.5313, 0.0, 0.4276, 0.4),
}


def riemann_state(grid, gamma=GAMMA, split=(0.5, 0.5)):
    x, y = grid.x, grid.y
    east = x >= split[0]
    north = y >= split[1]
    out = []
    for k in range(4):
        a = np.where(north & east, RIEMANN_QUADRANTS["ne"][k],
            np.where(north & ~east, RIEMANN_QUADRANTS["nw"][k],
            np.where(~north & ~east, RIEMANN_QUADRANTS["sw"][k], RIEMANN_QUADRANTS["se"][k])))
        out.append(a)
    return conservative(*out, gamma=gamma)


def sod_state(grid, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), x0=0.5, gamma=GAMMA):
    x = grid.x
    L = x < x0
    rho = np.where(L, left[0], right[0])
    u = np.where(L, left[1], right[1])
    p = np.where(L, left[2], right[2])
    return conservative(rho, u, np.zeros_like(u), p, gamma)


def shu_osher_state(grid, gamma=GAMMA):
    """Shu-Osher problem (Sec. 6.2(2)) on [-5, 5]: (rho, u, p) = (3.857143,
    2.629369, 10.3333) for x < -4, (1 + 0.2 sin 5x, 0, 1) otherwise."""
    x = grid.x
    left = x < -4.0
    rho = np.where(left, 3.857143, 1.0 + 0.2 * np.sin(5.0 * x))
    u = np.where(left, 2.629369, 0.0)
    p = np.where(left, 10.3333, 1.0)
    return conservative(rho, u, np.zeros_like(x), p, gamma)


def riemann_problem(n=2048, A=0.2, seed=2048, layers=4):
    """2-D Riemann throughput workload on [0,1]^2 (randomized when A > 0)."""
    g = bounded_grid(n, n, (0.0, 1.0, 0.0, 1.0), A=A, seed=seed, layers=layers)
    return g, riemann_state(g)


def fsp_problem(n, A=0.2, seed=None, box=(0.0, 10.0, 0.0, 10.0)):
    seed = 1810 + n if seed is None else seed
    g = periodic_grid(n, n, box, A=A, seed=seed)
    return g, uniform_flow(g)


def vortex_problem(n, A=0.2, seed=None, box=(0.0, 10.0, 0.0, 10.0), **kw):
    seed = 1810 + n if seed is None else seed
    g = periodic_grid(n, n, box, A=A, seed=seed)
    return g, vortex_periodic_state(g, **kw)


def random_smooth_state(grid, seed=0, amp=0.05):
    """Smooth random perturbation of a uniform state (for parity tests)."""
    rng = np.random.default_rng(seed)
    Lx = grid.period[0] or (grid.x.max() - grid.x.min())
    Ly = grid.period[1] or (grid.y.max() - grid.y.min())
    x, y = grid.x, grid.y
    fields = []
    for _ in range(4):
        f = np.zeros_like(x)
        for _k in range(3):
            kx, ky = rng.integers(1, 4, size=2)
            ph = rng.random() * 2 * np.pi
            f += np.sin(2 * np.pi * (kx * x / Lx + ky * y / Ly) + ph)
        fields.append(f)
    rho = 1.0 + amp * fields[0]
    u = 0.3 + amp * fields[1]
    v = -0.2 + amp * fields[2]
    p = 1.0 + amp * fields[3]
    return conservative(rho, u, v, p)


def batched_blocks(nblocks=64, seed=64, h=1.0 / 512, A=0.2, nmin=64, nmax=1024, speed=4.0, amp=0.05):
    """Batched multi-block workload: `nblocks` independent periodic
    randomized blocks with n_x ~ U{nmin..nmax}, aspect a ~ logU(1/4, 4),
    n_y = clip(round(n_x a), nmin, nmax), spacing h; each carries a uniform
    flow rho = 1, p = 1/gamma (c = 1) at `speed` in a random direction plus an
    entropy wave rho += amp sum_3 sin(2 pi (k x/L_x + l y/L_y) + phi).
    Returns a list of (Grid, U)."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(nblocks):
        nx = int(rng.integers(nmin, nmax + 1))
        a = float(np.exp(rng.uniform(np.log(0.25), np.log(4.0))))
        ny = int(np.clip(round(nx * a), nmin, nmax))
        g = periodic_grid(nx, ny, (0.0, nx * h, 0.0, ny * h), A=A, seed=seed * 1000 + b)
        th = rng.uniform(0.0, 2 * np.pi)
        Lx, Ly = g.period
        rho = np.ones_like(g.x)
        for _ in range(3):
            k, l = rng.integers(1, 4, size=2)
            ph = rng.uniform(0.0, 2 * np.pi)
            rho = rho + amp * np.sin(2 * np.pi * (k * g.x / Lx + l * g.y / Ly) + ph)
        U = conservative(rho, speed * np.cos(th), speed * np.sin(th), 1.0 / GAMMA)
        out.append((g, U))
    return out


# ---- multi-block grids cut from one structured grid --------------------------

SIDE_KINDS = {"transmissive": 0, "wall": 1, "fixed": 2, "interface": 3}


@dataclass
class MBlock:
    """One block of a multi-block grid.  Sides are x lo, x hi, y lo, y hi;
    side kinds index SIDE_KINDS; an "interface" side continues into side
    nbr_side[s] of block nbr[s], whose coordinates are read shifted by
    shift[s] (non-zero across a periodic seam only).  `src` maps each node
    (j, i) of the block to the flat index of the node it came from in the
    grid it was cut from (for reassembly)."""
    x: np.ndarray
    y: np.ndarray
    sides: list
    nbr: list
    nbr_side: list
    shift: np.ndarray
    fixed: np.ndarray
    src: np.ndarray
    bc: tuple = ("transmissive", "transmissive")
    period: tuple = (0.0, 0.0)

    @property
    def shape(self):
        return self.x.shape


def cut_blocks(grid, fields=(), icuts=(), jcuts=(), turns=None, sides=("transmissive",) * 4, fixed=None):
    """Cut `grid` into (len(icuts)+1) x (len(jcuts)+1) rectangular blocks at
    the given node indices and turn the index frame of block b by
    90 * turns[b] degrees (a rotation, so every block stays right-handed).
    Periodic directions of the grid become interfaces with a shift of one
    period; its other sides take `sides` (x lo, x hi, y lo, y hi) and the
    fixed states `fixed` [4][4].  `fields` are arrays [..., ny, nx] cut and
    turned with the blocks.  Returns (blocks, [per-field lists of block
    arrays])."""
    ny, nx = grid.x.shape
    ia = [0, *icuts, nx]
    jc = [0, *jcuts, ny]
    P, Q = len(ia) - 1, len(jc) - 1
    nb = P * Q
    turns = [0] * nb if turns is None else list(turns)
    per = (grid.bc[0] == "periodic", grid.bc[1] == "periodic")
    Lx, Ly = grid.period
    fixed = np.zeros((4, 4)) if fixed is None else np.asarray(fixed, dtype=np.float64).reshape(4, 4)
    flat = np.arange(nx * ny).reshape(ny, nx)
    bid = lambda p, q: q * P + p
    pieces, conn = [], []
    for q in range(Q):
        for p in range(P):
            sl = (slice(jc[q], jc[q + 1]), slice(ia[p], ia[p + 1]))
            pieces.append(sl)
            c = []
            # (kind, neighbour, its side, shift) for sides 0..3 of the unturned piece
            for s, (dp, dq, other) in enumerate([(-1, 0, 1), (1, 0, 0), (0, -1, 3), (0, 1, 2)]):
                pp, qq = p + dp, q + dq
                sh = np.zeros(2)
                inside = 0 <= pp < P and 0 <= qq < Q
                if not inside and per[0 if s < 2 else 1]:
                    if s < 2:
                        sh[0] = -Lx if pp < 0 else Lx
                    else:
                        sh[1] = -Ly if qq < 0 else Ly
                    pp, qq, inside = pp % P, qq % Q, True
                if inside:
                    c.append((3, bid(pp, qq), other, sh))
                else:
                    k = sides[s]
                    c.append((SIDE_KINDS[k] if isinstance(k, str) else int(k), -1, 0, sh))
            conn.append(c)

    def side_nodes(a):  # flat indices on sides 0..3 of a [ny][nx] index array
        return [set(a[:, 0].ravel()), set(a[:, -1].ravel()), set(a[0, :].ravel()), set(a[-1, :].ravel())]

    # side renaming under each block's turn
    newside = []
    for b, sl in enumerate(pieces):
        idx = flat[sl]
        before = side_nodes(idx)
        after = side_nodes(np.rot90(idx, turns[b]))
        newside.append([after.index(before[s]) for s in range(4)])
    blocks = []
    for b, sl in enumerate(pieces):
        k = turns[b]
        src = np.ascontiguousarray(np.rot90(flat[sl], k))
        kinds, nbr, nsd = [0] * 4, [-1] * 4, [0] * 4
        shift = np.zeros((4, 2))
        fx = np.zeros((4, 4))
        for s in range(4):
            kind, n2, s2, sh = conn[b][s]
            t = newside[b][s]
            kinds[t] = kind
            if kind == 3:
                nbr[t], nsd[t] = n2, newside[n2][s2]
                shift[t] = sh
            else:
                fx[t] = fixed[s]
        blocks.append(MBlock(x=np.ascontiguousarray(np.rot90(grid.x[sl], k)),
                             y=np.ascontiguousarray(np.rot90(grid.y[sl], k)),
                             sides=kinds, nbr=nbr, nbr_side=nsd, shift=shift, fixed=fx, src=src))
    out = []
    for f in fields:
        f = np.asarray(f)
        out.append([np.ascontiguousarray(np.rot90(f[(..., *sl)], turns[b], axes=(-2, -1)))
                    for b, sl in enumerate(pieces)])
    return blocks, out


def assemble(blocks, arrays, shape):
    """Inverse of cut_blocks for block arrays [..., ny_b, nx_b]: the array
    [..., ny, nx] of the original grid."""
    ny, nx = shape
    lead = np.asarray(arrays[0]).shape[:-2]
    out = np.full(lead + (ny * nx,), np.nan)
    for blk, a in zip(blocks, arrays):
        a = np.asarray(a)
        out[..., blk.src.ravel()] = a.reshape(lead + (-1,))
    return out.reshape(lead + (ny, nx))


# ---- three-dimensional grids and states --------------------------------------

@dataclass
class Grid3:
    x: np.ndarray  # [nz][ny][nx]
    y: np.ndarray
    z: np.ndarray
    bc: tuple = ("periodic", "periodic", "periodic")
    period: tuple = (0.0, 0.0, 0.0)
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.x.shape


def _mesh3(nx, ny, nz):
    kk, jj, ii = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                             np.arange(nx, dtype=np.float64), indexing="ij")
    return ii, jj, kk


def _jitter3(shape, A, rng, mask):
    """The 3-D counterpart of Sec. 6.1(1): each node displaced by
    2A(Rand(0,1) - 0.5) spacings along one axis drawn uniformly."""
    r = rng.random(shape)
    axis = rng.integers(0, 3, size=shape)
    d = 2.0 * A * (r - 0.5) * mask
    return d * (axis == 0), d * (axis == 1), d * (axis == 2)


def periodic_grid3(nx, ny, nz, box=(0.0, 1.0, 0.0, 1.0, 0.0, 1.0), A=0.0, seed=0):
    """Periodic grid of nx x ny x nz distinct nodes, randomized at every node
    when A > 0."""
    x0, x1, y0, y1, z0, z1 = box
    h = ((x1 - x0) / nx, (y1 - y0) / ny, (z1 - z0) / nz)
    ii, jj, kk = _mesh3(nx, ny, nz)
    d = (0.0, 0.0, 0.0)
    if A > 0:
        d = _jitter3(ii.shape, A, np.random.default_rng(seed), np.ones(ii.shape))
    c = lambda a: np.ascontiguousarray(a)
    return Grid3(c(x0 + (ii + d[0]) * h[0]), c(y0 + (jj + d[1]) * h[1]), c(z0 + (kk + d[2]) * h[2]),
                 ("periodic",) * 3, (x1 - x0, y1 - y0, z1 - z0), {"A": A, "seed": seed})


def bounded_grid3(nx, ny, nz, box=(0.0, 1.0, 0.0, 1.0, 0.0, 1.0), A=0.0, seed=0, layers=4):
    """Non-periodic grid (nodes on both ends), randomized except in `layers`
    uniform layers along every boundary."""
    x0, x1, y0, y1, z0, z1 = box
    h = ((x1 - x0) / (nx - 1), (y1 - y0) / (ny - 1), (z1 - z0) / (nz - 1))
    ii, jj, kk = _mesh3(nx, ny, nz)
    d = (0.0, 0.0, 0.0)
    if A > 0:
        inner = lambda v, n: (v >= layers) & (v < n - layers)
        mask = (inner(ii, nx) & inner(jj, ny) & inner(kk, nz)).astype(np.float64)
        d = _jitter3(ii.shape, A, np.random.default_rng(seed), mask)
    c = lambda a: np.ascontiguousarray(a)
    return Grid3(c(x0 + (ii + d[0]) * h[0]), c(y0 + (jj + d[1]) * h[1]), c(z0 + (kk + d[2]) * h[2]),
                 ("transmissive",) * 3, (0.0, 0.0, 0.0), {"A": A, "seed": seed, "layers": layers})


def mixed_grid3(nx, ny, nz, bc=("periodic", "transmissive", "periodic"), box=(0.0, 1.0, 0.0, 1.0, 0.0, 1.0),
                A=0.0, seed=0, layers=4):
    """Grid with some directions periodic (distinct nodes, spacing L/n) and
    the others bounded (nodes on both ends, spacing L/(n-1), `layers`
    uniform node layers along those boundaries), randomized as in
    periodic_grid3 elsewhere."""
    n = (nx, ny, nz)
    per = [b == "periodic" for b in bc]
    lo, hi = box[0::2], box[1::2]
    h = [(hi[a] - lo[a]) / (n[a] if per[a] else n[a] - 1) for a in range(3)]
    idx = _mesh3(nx, ny, nz)
    d = (0.0, 0.0, 0.0)
    if A > 0:
        mask = np.ones(idx[0].shape, dtype=bool)
        for a in range(3):
            if not per[a]:
                mask &= (idx[a] >= layers) & (idx[a] < n[a] - layers)
        d = _jitter3(idx[0].shape, A, np.random.default_rng(seed), mask.astype(np.float64))
    c = [np.ascontiguousarray(lo[a] + (idx[a] + d[a]) * h[a]) for a in range(3)]
    return Grid3(c[0], c[1], c[2], tuple(bc), tuple((hi[a] - lo[a]) if per[a] else 0.0 for a in range(3)),
                 {"A": A, "seed": seed})


def wavy_grid3(nx, ny, nz, L=1.0, amp=0.04):
    """Smooth periodic curvilinear grid on [0, L)^3: every coordinate is
    displaced by amp L sin(2 pi a) sin(2 pi b) of the two other index
    coordinates (a, b in [0, 1)), so all nine metrics vary."""
    ii, jj, kk = _mesh3(nx, ny, nz)
    a, b, c = ii / nx, jj / ny, kk / nz
    s = lambda u: np.sin(2 * np.pi * u)
    x = L * a + amp * L * s(b) * s(c)
    y = L * b + amp * L * s(c) * s(a)
    z = L * c + amp * L * s(a) * s(b)
    f = np.ascontiguousarray
    return Grid3(f(x), f(y), f(z), ("periodic",) * 3, (L, L, L), {"amp": amp})


def extrude(grid, nz, U=None):
    """A 2-D grid (and state [4][ny][nx]) made z-independent in 3-D: z = k
    (period nz), w = 0; returns (Grid3, state [5][nz][ny][nx] or None)."""
    ny, nx = grid.x.shape
    rep = lambda a: np.ascontiguousarray(np.broadcast_to(a, (nz, ny, nx)))
    z = np.ascontiguousarray(np.broadcast_to(np.arange(nz, dtype=np.float64)[:, None, None], (nz, ny, nx)))
    g3 = Grid3(rep(grid.x), rep(grid.y), z, (grid.bc[0], grid.bc[1], "periodic"),
               (grid.period[0], grid.period[1], float(nz)))
    if U is None:
        return g3, None
    U3 = np.zeros((5, nz, ny, nx))
    U3[0], U3[1], U3[2], U3[4] = rep(U[0]), rep(U[1]), rep(U[2]), rep(U[3])
    return g3, U3


def conservative3(rho, u, v, w, p, gamma=GAMMA):
    rho = np.asarray(rho, dtype=np.float64)
    e = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.ascontiguousarray(np.stack([rho, rho * u * np.ones_like(rho), rho * v * np.ones_like(rho),
                                          rho * w * np.ones_like(rho), e * np.ones_like(rho)]))


def uniform_flow3(grid, mach=0.5, direction=(1.0, 0.7, 0.4), rho=1.0, p=1.0, gamma=GAMMA):
    n = np.asarray(direction, dtype=np.float64)
    n = n / np.linalg.norm(n)
    c = np.sqrt(gamma * p / rho)
    r = np.full(grid.x.shape, rho)
    return conservative3(r, mach * c * n[0], mach * c * n[1], mach * c * n[2], p, gamma)


def entropy_wave3(grid, t=0.0, vel=(0.6, 0.4, 0.3), amp=0.2, gamma=GAMMA):
    """rho = 1 + amp sin(2 pi (x + y + z - (u + v + w) t) / L) with uniform
    velocity and pressure 1: an exact solution of the Euler equations on a
    periodic cube of side L."""
    L = grid.period[0]
    u, v, w = vel
    rho = 1.0 + amp * np.sin(2 * np.pi * (grid.x + grid.y + grid.z - (u + v + w) * t) / L)
    return conservative3(rho, u, v, w, 1.0, gamma)


def octant_state3(grid, gamma=GAMMA):
    """Discontinuous state: eight octants about the centre of the box with
    different densities, velocities and pressures (a 3-D Riemann problem)."""
    xm = 0.5 * (grid.x.min() + grid.x.max())
    ym = 0.5 * (grid.y.min() + grid.y.max())
    zm = 0.5 * (grid.z.min() + grid.z.max())
    o = (grid.x > xm).astype(int) + 2 * (grid.y > ym).astype(int) + 4 * (grid.z > zm).astype(int)
    rho = np.array([1.0, 0.5323, 0.5323, 0.138, 0.8, 1.2, 0.7, 1.5])[o]
    u = np.array([0.0, 1.206, 0.0, 1.206, 0.1, -0.2, 0.3, 0.0])[o]
    v = np.array([0.0, 0.0, 1.206, 1.206, -0.1, 0.2, 0.0, 0.3])[o]
    w = np.array([0.0, 0.2, -0.2, 0.0, 0.4, 0.0, -0.3, 0.1])[o]
    p = np.array([1.0, 0.3, 0.3, 0.029, 0.9, 1.4, 0.6, 1.1])[o]
    return conservative3(rho, u, v, w, p, gamma)


def smooth_state3(grid, seed=0, amp=0.15, gamma=GAMMA):
    """Smooth random state: density, pressure and the three velocities each
    a constant plus three sinusoids of the coordinates (wavelengths of the
    box size) with random phases, amplitudes up to `amp`."""
    rng = np.random.default_rng(seed)
    L = [max(float(c.max() - c.min()), 1e-12) for c in (grid.x, grid.y, grid.z)]

    def field(base):
        f = np.full(grid.x.shape, base)
        for _ in range(3):
            k = rng.integers(1, 3, size=3)
            ph = rng.uniform(0.0, 2 * np.pi)
            f = f + amp * rng.uniform(0.3, 1.0) * np.sin(
                2 * np.pi * (k[0] * grid.x / L[0] + k[1] * grid.y / L[1] + k[2] * grid.z / L[2]) + ph)
        return f

    return conservative3(field(1.0), field(0.3), field(-0.2), field(0.1), field(1.0), gamma)
