"""NURBS patch maps F_j: [0,1]^2 -> Gamma_j (Sec. 3.2) and the pulled-back
surface quantities of Sec. 4.2: tangents d_u F, d_v F, the unnormalised normal
n~ = d_u F x d_v F and the surface measure a = |n~|.

Pinned by: enclosed volume (1/3) int F . n~ = 4 pi/3 and area 4 pi for the
sphere patches (up to the fitted geometry's radial error), and outward
orientation (positive volume).
"""
from __future__ import annotations

import numpy as np

from . import bspline


class PatchMap:
    """Evaluates one rational tensor-product B-spline patch."""

    def __init__(self, patch):
        self.pu, self.pv = patch.deg_u, patch.deg_v
        self.ku = np.asarray(patch.knots_u, dtype=np.float64)
        self.kv = np.asarray(patch.knots_v, dtype=np.float64)
        cpw = np.asarray(patch.cpw, dtype=np.float64)
        self.w = cpw[..., 3]                       # (nv, nu)
        self.cw = cpw[..., :3] * self.w[..., None]  # homogeneous numerators

    def eval(self, u, v):
        """F, d_u F, d_v F at the parameter points (u, v): each (n, 3)."""
        u = np.asarray(u, dtype=np.float64).ravel()
        v = np.asarray(v, dtype=np.float64).ravel()
        bu, dbu = bspline.basis_and_derivative(self.ku, self.pu, u)
        bv, dbv = bspline.basis_and_derivative(self.kv, self.pv, v)
        # numerator P(u,v) = sum_ij w_ij c_ij b_i(u) b_j(v), denominator W(u,v);
        # the u-contraction runs as one matrix product per factor
        nv_, nu_ = self.w.shape
        hom = np.concatenate([self.cw, self.w[..., None]], axis=-1)   # (nv, nu, 4)
        hu = hom.transpose(1, 0, 2).reshape(nu_, nv_ * 4)
        t0 = (bu @ hu).reshape(-1, nv_, 4)
        t1 = (dbu @ hu).reshape(-1, nv_, 4)
        Q = np.einsum("nj,njc->nc", bv, t0)
        Qu = np.einsum("nj,njc->nc", bv, t1)
        Qv = np.einsum("nj,njc->nc", dbv, t0)
        P, W = Q[:, :3], Q[:, 3]
        Pu, Wu = Qu[:, :3], Qu[:, 3]
        Pv, Wv = Qv[:, :3], Qv[:, 3]
        F = P / W[:, None]
        Fu = (Pu - F * Wu[:, None]) / W[:, None]
        Fv = (Pv - F * Wv[:, None]) / W[:, None]
        return F, Fu, Fv


def normal_and_measure(Fu: np.ndarray, Fv: np.ndarray):
    """n~ = d_u F x d_v F and a = |n~| (Sec. 4.2, surface measure)."""
    nt = np.cross(Fu, Fv)
    return nt, np.linalg.norm(nt, axis=-1)
