"""Centred second-derivative weights of the star stencil.

The paper benchmarks space orders 2, 4 and 8 (Section 6.1) without printing
the weights; these are the standard centred weights of order 2r for the
second derivative (c_0 .. c_r, with c_{-k} = c_k), as tabulated by Fornberg
(Math. Comp. 51, 1988).
"""
from __future__ import annotations

from fractions import Fraction

_TABLE = {
    2: (Fraction(-2), Fraction(1)),
    4: (Fraction(-5, 2), Fraction(4, 3), Fraction(-1, 12)),
    6: (Fraction(-49, 18), Fraction(3, 2), Fraction(-3, 20), Fraction(1, 90)),
    8: (Fraction(-205, 72), Fraction(8, 5), Fraction(-1, 5), Fraction(8, 315), Fraction(-1, 560)),
}


def second_derivative_weights(space_order: int) -> list:
    """[c_0, ..., c_r] as floats for the given even space order (2..8)."""
    if space_order not in _TABLE:
        raise ValueError("space order must be 2, 4, 6 or 8")
    return [float(c) for c in _TABLE[space_order]]


def heat_weights(space_order: int, alpha: float) -> list:
    """Weights of the explicit heat update u + alpha * L u (alpha = a dt / h^2)."""
    return [alpha * c for c in second_derivative_weights(space_order)]


def damping_profile(n: int, width: int, gmax: float):
    """Per-axis absorbing-layer profile of n points: g = gmax * ((width - d) /
    width)^2 at distance d < width (in points) from the nearer end, else 0."""
    import numpy as np
    d = np.minimum(np.arange(n), np.arange(n)[::-1]).astype(np.float64)
    return np.where(d < width, gmax * ((width - d) / max(width, 1)) ** 2, 0.0)

