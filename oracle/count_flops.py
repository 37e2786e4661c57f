"""Algorithmic operation counts of one rhs evaluation -- TEST INFRASTRUCTURE
(run by hand; its printed table is what the benchmark's roofline uses).

The oracle is instantiated with an operation-counting scalar (add, sub,
mul, div and sqrt count one each; metric-only work is not counted).  A
sweep of one direction costs A per cell plus B per grid line (the line's
wave-speed maximum and the boundary stencils), so on lines of n nodes it is
A + B / n per cell.  A and B come from two line lengths on the Riemann
state; the count depends on the data only through the two branches of each
weight mapping (a few hundredths of an operation per cell).

What is counted is the method's own work as the oracle performs it: each
side projects only the window entries its interpolation reads, less the
reference node itself (its deviation, and so its projection, is zero), each
deviation Q_m - Q_ref is formed once per side, and sums of products start
from their first term (no additions of zero).  The dense eigenvector
products still include the structural zeros of L and R.

Usage: python oracle/count_flops.py
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
from paper_1810_11103_amd import workloads as W  # noqa: E402


def per_direction(scheme, vars):
    counts = []
    for n in (96, 192):
        g, U = W.riemann_problem(n, A=0.2, seed=n)
        M = oracle.metrics(scheme, g.x, g.y, g.bc, g.period)
        cx, ce, comb = oracle.count_rhs_flops(scheme, U, M, g.bc, vars=vars)
        counts.append((n, 0.5 * (cx + ce) / n, comb / (n * n)))
    (n1, c1, comb), (n2, c2, _) = counts
    A = (c2 - c1) / (n2 - n1)
    B = c1 - A * n1
    return A, B, comb


def per_item3(scheme, n=48, lines=24, seed=3):
    """3-D direction pass, per item: nodal split flux (per node -4 .. n+3),
    midpoint split fluxes (per midpoint -4 .. n+2), combination and
    difference (per interior node); averaged over `lines` sampled lines of
    each direction of an octant Riemann state on a randomized periodic
    n^3 grid (the counts vary slightly with the data through the mappings'
    branches)."""
    g = W.periodic_grid3(n, n, n, A=0.2, seed=seed)
    U = W.octant_state3(g)
    M = oracle.metrics3(scheme, g.x, g.y, g.z, g.bc, g.period)
    G = oracle.G
    rng = np.random.default_rng(seed)
    tot = np.zeros(4)
    cnt = 0
    for d in range(3):
        for _ in range(lines):
            a, b = rng.integers(0, n, size=2)
            # line along axis d (array axes are z, y, x)
            ax = 2 - d
            idx = [slice(None)] * 3
            others = [x for x in (0, 1, 2) if x != ax]
            idx[others[0]], idx[others[1]] = a, b
            Q = U[(slice(None), *idx)]
            Mi = [slice(None)] * 3
            Mi[others[0]], Mi[others[1]] = a + G, b + G
            K = np.concatenate([M[3 * d:3 * d + 3][(slice(None), *Mi)], M[10 + 3 * d:13 + 3 * d][(slice(None), *Mi)]])
            tot += oracle.count_line_flops3(scheme, Q, K)
            cnt += 1
    tot /= cnt
    return tot[1] / (n + 8), tot[2] / (n + 7), tot[3] / n, tot[0] / n


if __name__ == "__main__":
    print("3-D, per item: scheme  nodal  midpoint  difference  line-maximum")
    for s in oracle.SCHEMES:
        fn, fm, fd, fx = per_item3(s)
        print(f"{s}  {fn:7.1f}  {fm:8.1f}  {fd:6.1f}  {fx:5.1f}")
    print("scheme  vars  A (per cell per direction)  B (per line)  final combination per cell")
    for s in oracle.SCHEMES:
        for v in ("characteristic", "conservative", "primitive"):
            A, B, comb = per_direction(s, v)
            print(f"{s}  {v:14s}  {A:8.1f}  {B:8.1f}  {comb:4.1f}")
