"""B-spline bases (Sec. 3.1, Definition of p-open knot vectors and the recursion).

Pinned by: the piecewise formulas of the paper's Figure 1 (p = 0, 1, 2 on the
knot vector with interior knots 1/3, 2/3), partition of unity, and the
dimension count k = #knots - p - 1.
"""
from __future__ import annotations

import numpy as np


def refinement_knots(p: int, m: int) -> np.ndarray:
    """Xi_{p,m}: p+1 zeros, the interior knots j/2^m, p+1 ones (Sec. 3.3)."""
    n = 2 ** m
    return np.array([0.0] * (p + 1) + [j / n for j in range(1, n)] + [1.0] * (p + 1))


def _degree0(knots: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Indicator functions of [xi_j, xi_{j+1}); the last non-empty interval is
    closed on the right so that the basis is defined at x = 1."""
    nk = len(knots)
    b = np.zeros((len(x), nk - 1))
    last = max(j for j in range(nk - 1) if knots[j] < knots[j + 1])
    for j in range(nk - 1):
        if knots[j] < knots[j + 1]:
            inside = (knots[j] <= x) & (x < knots[j + 1])
            if j == last:
                inside |= x == knots[j + 1]
            b[:, j] = inside
    return b


def _inv(den: np.ndarray) -> np.ndarray:
    # the recursion uses the convention 0/0 = 0 for repeated knots
    safe = np.where(den == 0.0, 1.0, den)
    return np.where(den == 0.0, 0.0, 1.0 / safe)


def basis(knots: np.ndarray, p: int, x) -> np.ndarray:
    """All k = len(knots)-p-1 basis functions b_j^p at the points x: (len(x), k).

    b_j^d = (x - xi_j)/(xi_{j+d} - xi_j) b_j^{d-1}
          + (xi_{j+d+1} - x)/(xi_{j+d+1} - xi_{j+1}) b_{j+1}^{d-1}
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    kn = np.asarray(knots, dtype=np.float64)
    b = _degree0(kn, x)
    xc = x[:, None]
    for d in range(1, p + 1):
        nb = b.shape[1] - 1
        lo = kn[:nb]                # xi_j
        hi = kn[d:d + nb]           # xi_{j+d}
        lo1 = kn[1:1 + nb]          # xi_{j+1}
        hi1 = kn[d + 1:d + 1 + nb]  # xi_{j+d+1}
        b = ((xc - lo) * _inv(hi - lo)) * b[:, :nb] + ((hi1 - xc) * _inv(hi1 - lo1)) * b[:, 1:nb + 1]
    return b


def basis_and_derivative(knots: np.ndarray, p: int, x):
    """(values, first derivatives) of all basis functions at x.

    The derivative follows from differentiating the recursion:
    b_j^p' = p/(xi_{j+p}-xi_j) b_j^{p-1} - p/(xi_{j+p+1}-xi_{j+1}) b_{j+1}^{p-1}.
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    kn = np.asarray(knots, dtype=np.float64)
    val = basis(kn, p, x)
    if p == 0:
        return val, np.zeros_like(val)
    low = basis(kn, p - 1, x)
    k = val.shape[1]
    c0 = p * _inv(kn[p:p + k] - kn[:k])
    c1 = p * _inv(kn[p + 1:p + 1 + k] - kn[1:1 + k])
    der = c0 * low[:, :k] - c1 * low[:, 1:k + 1]
    return val, der
