"""Pins of oracle.bspline: the worked example of Sec. 3.1, Figure 1."""
import json
import os

import numpy as np
import sympy as sp

from oracle import bspline

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig1_bsplines.json")


def test_figure1_piecewise_formulas():
    data = json.load(open(GOLD))
    x = sp.Symbol("x")
    for case in data["cases"]:
        kn = np.array(case["knots"], float)
        p = case["p"]
        seen = set()
        for j, lo, hi, expr in case["pieces"]:
            f = sp.lambdify(x, sp.sympify(expr, rational=True), "numpy")
            t = lo + (hi - lo) * np.linspace(0.05, 0.95, 11)
            val = bspline.basis(kn, p, t)[:, j]
            np.testing.assert_allclose(val, np.broadcast_to(f(t), t.shape), atol=1e-14)
            seen.add((j, lo))
        # every function not listed on an interval vanishes there
        inner = sorted(set(kn))
        for a, b in zip(inner[:-1], inner[1:]):
            t = a + (b - a) * np.linspace(0.05, 0.95, 7)
            val = bspline.basis(kn, p, t)
            for j in range(val.shape[1]):
                if not any(abs(lo - a) < 1e-12 and jj == j for jj, lo in seen):
                    assert np.all(np.abs(val[:, j]) < 1e-15)


def test_partition_of_unity_and_count():
    for p in range(4):
        for m in range(4):
            kn = bspline.refinement_knots(p, m)
            t = np.linspace(0, 1, 101)
            b, db = bspline.basis_and_derivative(kn, p, t)
            assert b.shape[1] == 2 ** m + p
            np.testing.assert_allclose(b.sum(1), 1.0, atol=1e-14)
            np.testing.assert_allclose(db.sum(1), 0.0, atol=1e-11)


def test_derivative_matches_finite_difference():
    kn = bspline.refinement_knots(3, 2)
    t = np.linspace(0.01, 0.99, 37)
    _, d = bspline.basis_and_derivative(kn, 3, t)
    eps = 1e-6
    fd = (bspline.basis(kn, 3, t + eps) - bspline.basis(kn, 3, t - eps)) / (2 * eps)
    np.testing.assert_allclose(d, fd, atol=1e-7)
