"""Algorithmic operation counts of one rhs evaluation -- TEST INFRASTRUCTURE
(run by hand; its printed table is what the benchmark's roofline uses).

The oracle is instantiated with an operation-counting scalar (add, sub,
mul, div and sqrt count one each; metric-only work is not counted).  A
sweep of one direction costs A per cell plus B per grid line (the line's
wave-speed maximum and the boundary stencils), so on lines of n nodes it is
A + B / n per cell.  A and B come from two line lengths on a smooth periodic
state; the count does not depend on the data (no data-dependent branches in
the counted arithmetic).

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


if __name__ == "__main__":
    print("scheme  vars  A (per cell per direction)  B (per line)  final combination per cell")
    for s in oracle.SCHEMES:
        for v in ("characteristic", "conservative", "primitive"):
            A, B, comb = per_direction(s, v)
            print(f"{s}  {v:14s}  {A:8.1f}  {B:8.1f}  {comb:4.1f}")
