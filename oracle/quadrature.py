"""Quadrature rules for the Galerkin double integrals over element pairs.

The paper leaves quadrature to its references (Sec. 4.4 refers to DHP16 /
DHK+18).  The reading taken here: regular element pairs use tensor
Gauss-Legendre rules; pairs that share an element, an edge or a vertex use
Duffy-type regularising substitutions in the spirit of Sauter & Schwab
(Boundary Element Methods, 2011, Sec. 5.2): after the substitution the weak
1/r singularity is cancelled by the Jacobian and the integrand is analytic on
[0,1]^4, so tensor Gauss converges exponentially.

Element-local coordinates (s1, s2) for the test element and (r1, r2) for the
trial element, both in [0,1]^2.  Canonical configurations:

* identical:  same element, singular on s = r;
* edge:       shared edge is s2 = r2 = 0, with s1 = r1 on the edge;
* vertex:     shared vertex is s = r = (0,0).

Every rule returns (xs, ys, w) with xs, ys of shape (Q, 2) and sum(w) = 1 (the
4-volume of [0,1]^4).

Pinned by: the closed form of the flat unit square self-interaction
int int 1/|x-y| = 4 ln(1+sqrt 2) - 4/3 (sqrt 2 - 1), and rectangle
decompositions for the edge / vertex rules (tests/test_oracle_quadrature.py).
"""
from __future__ import annotations

import functools

import numpy as np


@functools.lru_cache(maxsize=None)
def gauss01(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def tensor2(n: int):
    """Tensor Gauss rule on [0,1]^2: points (n^2, 2) with u fastest, weights."""
    x, w = gauss01(n)
    uu, vv = np.meshgrid(x, x, indexing="xy")
    wu, wv = np.meshgrid(w, w, indexing="xy")
    return np.stack([uu.ravel(), vv.ravel()], axis=1), (wu * wv).ravel()


def _grid4(n: int):
    x, w = gauss01(n)
    g = np.meshgrid(x, x, x, x, indexing="ij")
    gw = np.meshgrid(w, w, w, w, indexing="ij")
    pts = np.stack([a.ravel() for a in g], axis=1)
    wts = gw[0].ravel() * gw[1].ravel() * gw[2].ravel() * gw[3].ravel()
    return pts, wts


def _split_1d(u, w, sigma):
    """One coordinate pair (s, r) written through its offset u = |r - s| in
    [0,1] and a position w in [0,1]; the Jacobian of (s, r) -> (u, w) is 1-u."""
    base = w * (1.0 - u)
    if sigma > 0:
        return base, base + u
    return base + u, base


@functools.lru_cache(maxsize=None)
def identical(n: int):
    """Same element.  Per coordinate: sign of r-s (2 branches), offset u and
    position w; then (u1, u2) in [0,1]^2 is split along its diagonal and
    Duffy-transformed, u = rho (1, tau) or rho (tau, 1), Jacobian rho."""
    g, gw = _grid4(n)
    rho, tau, w1, w2 = g.T
    xs, ys, ws = [], [], []
    for sig1 in (1, -1):
        for sig2 in (1, -1):
            for tri in (0, 1):
                u1, u2 = (rho, rho * tau) if tri == 0 else (rho * tau, rho)
                s1, r1 = _split_1d(u1, w1, sig1)
                s2, r2 = _split_1d(u2, w2, sig2)
                xs.append(np.stack([s1, s2], 1))
                ys.append(np.stack([r1, r2], 1))
                ws.append(gw * (1 - u1) * (1 - u2) * rho)
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(ws)


@functools.lru_cache(maxsize=None)
def edge(n: int):
    """Shared edge s2 = r2 = 0.  The first coordinate is handled as in the
    identical rule (offset u1, position w1); the cube (u1, s2, r2) is split into
    three pyramids by its largest coordinate rho, Jacobian rho^2."""
    g, gw = _grid4(n)
    rho, t1, t2, w1 = g.T
    xs, ys, ws = [], [], []
    for sig1 in (1, -1):
        for pyr in range(3):
            if pyr == 0:
                u1, s2, r2 = rho, rho * t1, rho * t2
            elif pyr == 1:
                u1, s2, r2 = rho * t1, rho, rho * t2
            else:
                u1, s2, r2 = rho * t1, rho * t2, rho
            s1, r1 = _split_1d(u1, w1, sig1)
            xs.append(np.stack([s1, s2], 1))
            ys.append(np.stack([r1, r2], 1))
            ws.append(gw * (1 - u1) * rho ** 2)
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(ws)


@functools.lru_cache(maxsize=None)
def vertex(n: int):
    """Shared vertex at the origin: [0,1]^4 split into four pyramids by the
    largest coordinate rho, Jacobian rho^3."""
    g, gw = _grid4(n)
    rho, t1, t2, t3 = g.T
    xs, ys, ws = [], [], []
    for pyr in range(4):
        c = [rho * t1, rho * t2, rho * t3]
        c.insert(pyr, rho)
        s1, s2, r1, r2 = c
        xs.append(np.stack([s1, s2], 1))
        ys.append(np.stack([r1, r2], 1))
        ws.append(gw * rho ** 3)
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(ws)


# ----------------------------------------------------------------------------
# Symmetries of the unit square used to bring a touching element pair into the
# canonical configuration.  code = swap*4 + flip_t*2 + flip_s.
# ----------------------------------------------------------------------------

def d4_apply(code: int, st: np.ndarray) -> np.ndarray:
    s, t = st[..., 0], st[..., 1]
    if code & 4:
        s, t = t, s
    if code & 1:
        s = 1.0 - s
    if code & 2:
        t = 1.0 - t
    return np.stack([s, t], axis=-1)


def d4_find(maps_to: dict) -> int:
    """Smallest code whose map sends each local point key -> value."""
    for code in range(8):
        if all(np.allclose(d4_apply(code, np.array(k, float)), np.array(v, float))
               for k, v in maps_to.items()):
            return code
    raise ValueError("no square symmetry realises the requested corner map")
