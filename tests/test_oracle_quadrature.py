"""Pins of oracle.quadrature: the Duffy-type singular rules against closed forms
of flat configurations (kernel 1/|x-y|, kappa = 0).

* identical unit square:  4 ln(1+sqrt 2) - 4/3 (sqrt 2 - 1)   (closed form)
* rectangle a x b self-interaction by a polar-coordinate brute force whose
  inner radial integral is exact (a polynomial in r); it reproduces the square's
  closed form, and rectangle decompositions give the edge and vertex values:
      I_edge   = (I(2,1) - 2 I_sq) / 2,     I_vertex = I_sq - 2 I_edge.
"""
import numpy as np
import pytest

from oracle import quadrature as qd

I_SQ = 4 * np.log(1 + np.sqrt(2)) - 4.0 / 3.0 * (np.sqrt(2) - 1)


def rect_self(a, b, n=60):
    x, w = np.polynomial.legendre.leggauss(n)
    tot = 0.0
    tc = np.arctan2(b, a)
    for lo, hi, side in ((0, tc, "a"), (tc, np.pi / 2, "b")):
        th = lo + (hi - lo) * (x + 1) / 2
        wt = w * (hi - lo) / 2
        R = a / np.cos(th) if side == "a" else b / np.sin(th)
        s, c = np.sin(th), np.cos(th)
        tot += np.sum(wt * (a * b * R - (a * s + b * c) * R ** 2 / 2 + s * c * R ** 3 / 3))
    return 4 * tot


def test_brute_force_reference_reproduces_closed_form():
    assert abs(rect_self(1, 1) - I_SQ) < 1e-14
    assert abs(rect_self(2, 2) - 8 * I_SQ) < 1e-13


@pytest.mark.parametrize("rule", [qd.identical, qd.edge, qd.vertex])
def test_weights_sum_to_one(rule):
    assert abs(rule(5)[2].sum() - 1.0) < 1e-13


def _flat(rule, ymap, n):
    xs, ys, w = rule(n)
    Y = ymap(ys)
    r = np.linalg.norm(xs - Y, axis=1)
    return np.sum(w / r)


def test_identical_flat_square():
    val = _flat(qd.identical, lambda y: y, 10)
    assert abs(val - I_SQ) < 1e-12


def test_edge_flat_squares():
    i_edge = (rect_self(2, 1) - 2 * I_SQ) / 2
    val = _flat(qd.edge, lambda y: np.stack([y[:, 0], -y[:, 1]], 1), 10)
    assert abs(val - i_edge) < 1e-12


def test_vertex_flat_squares():
    i_edge = (rect_self(2, 1) - 2 * I_SQ) / 2
    i_vertex = I_SQ - 2 * i_edge
    val = _flat(qd.vertex, lambda y: -y, 10)
    assert abs(val - i_vertex) < 1e-12


def test_square_symmetries():
    for code in range(8):
        corners = qd.d4_apply(code, np.array([[0, 0], [1, 0], [0, 1], [1, 1]], float))
        assert sorted(map(tuple, corners.tolist())) == [(0, 0), (0, 1), (1, 0), (1, 1)]
    assert qd.d4_find({(0, 0): (1, 1), (1, 0): (1, 0)}) >= 0
