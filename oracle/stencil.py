"""Finite-difference weights of the central-difference constraints.

The paper's central-difference rows (Eq. 5) tie a derivative variable to a
difference of neighbouring solution values; in practice a 5-point central
window is used, with one-sided (forward/backward) windows at the edges of
the grid (the sentence following Eq. 5).

For a window of offsets o_0..o_4 (in grid steps, relative to the point the
row belongs to) and derivative order q, the weights w_k are the unique
solution of the moment system

    sum_k w_k * o_k**p / p!  =  [p == q],      p = 0..4,

so that sum_k w_k u(i + o_k) = s**q * u^(q)(i) + O(s**5) for smooth u.
The system is solved here in exact rational arithmetic (Gauss-Jordan over
``fractions.Fraction``), then converted to float64.

Oracle module: test infrastructure only.
"""

from fractions import Fraction
from math import factorial

WINDOW = 5  # points per central-difference window


def window_offsets(i, n, periodic):
    """Offsets (relative to point ``i``) of the 5-point window on an axis of
    ``n`` points.  Periodic axes always use the centred window -2..2 (indices
    wrap); non-periodic axes use the centred window where it fits and the
    window shifted inward at the edges (first window 0..4, last -4..0)."""
    if n < WINDOW:
        raise ValueError("an axis needs at least 5 points for 5-point windows")
    if periodic:
        return tuple(range(-2, 3))
    start = min(max(i - 2, 0), n - WINDOW)
    return tuple(start - i + k for k in range(WINDOW))


def _solve_exact(M, rhs):
    """Gauss-Jordan elimination over Fractions (M square, nonsingular)."""
    n = len(M)
    a = [list(map(Fraction, row)) + [Fraction(r)] for row, r in zip(M, rhs)]
    for col in range(n):
        piv = next(r for r in range(col, n) if a[r][col] != 0)
        a[col], a[piv] = a[piv], a[col]
        pv = a[col][col]
        a[col] = [x / pv for x in a[col]]
        for r in range(n):
            if r != col and a[r][col] != 0:
                f = a[r][col]
                a[r] = [x - f * y for x, y in zip(a[r], a[col])]
    return [a[r][n] for r in range(n)]


def fd_weights_exact(offsets, order):
    """Exact rational weights for derivative ``order`` on the given offsets."""
    m = len(offsets)
    M = [[Fraction(o) ** p / factorial(p) for o in offsets] for p in range(m)]
    rhs = [1 if p == order else 0 for p in range(m)]
    return tuple(_solve_exact(M, rhs))


def fd_weights(offsets, order):
    """Float64 weights for derivative ``order`` on ``offsets``."""
    return tuple(float(w) for w in fd_weights_exact(offsets, order))
