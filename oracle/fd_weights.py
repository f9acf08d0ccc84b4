"""Centred second-derivative weights, derived from their moment conditions.

The paper gives no weights for the space orders it benchmarks (2, 4, 8;
Section 6.1).  The oracle derives them independently of the GPU path: the
symmetric weights c_{-k} = c_k of order 2r are the unique solution of

    sum_{k=-r..r} c_k k^(2j) = 2 [j == 1],    j = 0..r,

solved here in exact rational arithmetic.  Test infrastructure only.
"""
from __future__ import annotations

import math
from fractions import Fraction


def _solve(a, b):
    """Gaussian elimination over Fractions (square, nonsingular)."""
    n = len(a)
    m = [list(row) + [rhs] for row, rhs in zip(a, b)]
    for col in range(n):
        piv = next(r for r in range(col, n) if m[r][col] != 0)
        m[col], m[piv] = m[piv], m[col]
        for r in range(n):
            if r != col and m[r][col] != 0:
                f = m[r][col] / m[col][col]
                m[r] = [x - f * y for x, y in zip(m[r], m[col])]
    return [m[i][n] / m[i][i] for i in range(n)]


def fd_weights(space_order: int) -> list:
    """[c_0, c_1, ..., c_r] as Fractions for space order 2r."""
    if space_order < 2 or space_order % 2:
        raise ValueError("space order must be even and >= 2")
    r = space_order // 2
    # unknowns c_1..c_r:  sum_k c_k k^(2j) = [j == 1], j = 1..r
    a = [[Fraction(k) ** (2 * j) for k in range(1, r + 1)] for j in range(1, r + 1)]
    b = [Fraction(1 if j == 1 else 0) for j in range(1, r + 1)]
    ck = _solve(a, b)
    c0 = -2 * sum(ck)
    return [c0] + ck


def fd_weights_float(space_order: int) -> list:
    return [float(x) for x in fd_weights(space_order)]


def symbol(c, theta: float) -> float:
    """S(theta) = -(c_0 + 2 sum_k c_k cos(k theta)): minus the operator's
    eigenvalue on the Fourier mode exp(i theta x), per axis, h = 1."""
    return -(float(c[0]) + 2.0 * sum(float(c[k]) * math.cos(k * theta) for k in range(1, len(c))))
