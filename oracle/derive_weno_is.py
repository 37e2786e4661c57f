"""Smoothness indicators of WENO interpolation as exact quadratic forms --
TEST INFRASTRUCTURE ONLY (it writes no file; the oracle carries the r = 4
coefficients as constants and the test suite re-derives and compares them).

The paper prints the r = 3 indicators (Eqs. 3.14, 3.22) and only the
candidate coefficients and linear weights for r = 4 (Table A1).  The r = 3
indicators are the Jiang-Shu ones, applied to nodal values with the node
index in place of the cell index; the r = 4 indicators used for the
seventh-order schemes follow the same definition:

    IS_k = sum_{l=1}^{r-1} int_{-1/2}^{1/2} (d^l p_k / dx^l)^2 dx,

where p_k is the polynomial of degree r-1 whose averages over the unit cells
centred on the stencil points {k-r+1, ..., k} (relative to the node j at 0)
equal the stencil values.  Everything is done in rational arithmetic.
"""
from fractions import Fraction as Fr


def _solve(A, b):
    """Exact Gauss-Jordan solve of A X = B (A square, B a list of columns)."""
    n = len(A)
    M = [row[:] + [bb[i] for bb in b] for i, row in enumerate(A)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [v / piv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [vr - f * vc for vr, vc in zip(M[r], M[c])]
    return [[M[i][n + j] for i in range(n)] for j in range(len(b))]


def _cell_avg_row(c, r):
    """Averages of x^0..x^{r-1} over [c - 1/2, c + 1/2]."""
    lo, hi = Fr(2 * c - 1, 2), Fr(2 * c + 1, 2)
    return [(hi ** (n + 1) - lo ** (n + 1)) / (n + 1) for n in range(r)]


def indicator_matrix(r, k):
    """Symmetric matrix Q (r x r, Fractions) with IS_k = v^T Q v for the
    stencil values v = (v_{k-r+1}, ..., v_k) around node 0, k = 0..r-1
    counted from the leftmost stencil (cells k-r+1 .. k relative to the
    stencil's last point at k - r + 1 + r - 1)."""
    cells = [k - (r - 1) + m for m in range(r)]
    A = [_cell_avg_row(c, r) for c in cells]
    # columns of A^{-1}: polynomial coefficients of the cardinal functions
    I = [[Fr(int(i == j)) for i in range(r)] for j in range(r)]
    card = _solve(A, I)  # card[m] = coefficients a_0..a_{r-1} of cardinal m
    Q = [[Fr(0)] * r for _ in range(r)]
    for l in range(1, r):
        # derivative of order l of each cardinal polynomial
        der = []
        for m in range(r):
            a = card[m]
            d = [Fr(0)] * r
            for n in range(l, r):
                f = Fr(1)
                for t in range(n - l + 1, n + 1):
                    f *= t
                d[n - l] = a[n] * f
            der.append(d)
        # integral over [-1/2, 1/2] of products of polynomials
        def integ(p, q):
            s = Fr(0)
            for i, pi in enumerate(p):
                if pi == 0:
                    continue
                for j, qj in enumerate(q):
                    if qj == 0:
                        continue
                    n = i + j
                    s += pi * qj * (Fr(1, 2) ** (n + 1) - Fr(-1, 2) ** (n + 1)) / (n + 1)
            return s
        for a in range(r):
            for b in range(r):
                Q[a][b] += integ(der[a], der[b])
    return Q


def indicators(r):
    """The r matrices, stencil k covering nodes (k - r + 1 .. k) + (r - 1) - ...
    i.e. for the left-biased value at j+1/2 from v_{j-r+1..j+r-1}: stencil k
    holds v_{j-r+1+k .. j+k}."""
    # stencil k of the interpolation holds nodes j-r+1+k .. j+k; relative to
    # the cell j (at 0) those are cells (k - r + 1) .. k
    return [indicator_matrix(r, k) for k in range(r)]


if __name__ == "__main__":
    for r in (2, 3, 4):
        print(f"r = {r}")
        for k, Q in enumerate(indicators(r)):
            print("  k =", k, [[str(v) for v in row] for row in Q])
