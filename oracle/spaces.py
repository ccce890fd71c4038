"""The discrete spaces S^2_{p,m}(Gamma) and S^0_{p,m}(Gamma) (Sec. 3.3).

Numbering (shared convention with the library, written independently):

* elements   e = patch * 4^m + ey * 2^m + ex, covering [ex, ex+1] x [ey, ey+1] / 2^m;
* S^2 dofs   i = patch * k^2 + iv * k + iu, k = 2^m + p, basis b_iu(u) b_iv(v)
  of S_{p,p}(Xi_{p,m}, Xi_{p,m}) on each patch; dim S^2 = n (2^m + p)^2;
* S^0 dofs   the globally continuous subspace.  An S^0 basis function is the sum
  of the S^2 functions whose Greville anchor points F_j(xi*_iu, xi*_iv) coincide
  on patch interfaces; S^0 dofs are numbered in increasing order of their lowest
  S^2 representative.

Pinned by the dimension formulas: n (2^m+p)^2 for S^2 (Sec. 3.3) and, on the
closed cube topology, 6 (k-2)^2 + 12 (k-2) + 8 for S^0 (Euler's formula).
"""
from __future__ import annotations

import numpy as np

from . import bspline
from .geometry import PatchMap


class Discretization:
    def __init__(self, patches, p: int, m: int):
        self.patches = list(patches)
        self.maps = [PatchMap(pt) for pt in self.patches]
        self.npatch = len(self.patches)
        self.p, self.m = p, m
        self.nel1 = 2 ** m
        self.h = 1.0 / self.nel1
        self.k = self.nel1 + p
        self.knots = bspline.refinement_knots(p, m)
        self.nelem = self.npatch * self.nel1 ** 2
        self.n2 = self.npatch * self.k ** 2
        self.nloc = (p + 1) ** 2
        e = np.arange(self.nelem)
        self.el_patch = e // self.nel1 ** 2
        self.el_ey = (e // self.nel1) % self.nel1
        self.el_ex = e % self.nel1
        a = np.arange(self.nloc)
        au, av = a % (p + 1), a // (p + 1)
        self.el_dofs = (self.el_patch[:, None] * self.k ** 2
                        + (self.el_ey[:, None] + av[None, :]) * self.k
                        + (self.el_ex[:, None] + au[None, :]))
        self._s0 = None

    # ------------------------------------------------------------------ S^0
    def greville(self) -> np.ndarray:
        kn, p = self.knots, self.p
        if p == 0:
            return 0.5 * (kn[:-1] + kn[1:])
        return np.array([kn[i + 1:i + p + 1].mean() for i in range(self.k)])

    def s0_map(self):
        """(s2_to_s0 [n2], n0): the glue map of S^0 into S^2."""
        if self._s0 is not None:
            return self._s0
        if self.p == 0:
            raise ValueError("S^0 needs p >= 1")
        k = self.k
        g = self.greville()
        parent = np.arange(self.n2)

        def find(i):
            while parent[i] != i:
                parent[i] = parent[parent[i]]
                i = parent[i]
            return i

        bidx, bpts = [], []
        for j, mp in enumerate(self.maps):
            for iv in range(k):
                for iu in range(k):
                    if iu in (0, k - 1) or iv in (0, k - 1):
                        bidx.append(j * k * k + iv * k + iu)
                        bpts.append((g[iu], g[iv]))
        bidx = np.array(bidx)
        bpts = np.array(bpts)
        pts = np.zeros((len(bidx), 3))
        for j, mp in enumerate(self.maps):
            sel = (bidx // (k * k)) == j
            F, _, _ = mp.eval(bpts[sel, 0], bpts[sel, 1])
            pts[sel] = F
        diam = np.ptp(pts, axis=0).max()
        tol = 1e-9 * diam
        order = np.lexsort((pts[:, 2], pts[:, 1], pts[:, 0]))
        # brute-force pairwise match within a sorted window along x
        xs = pts[order, 0]
        for a in range(len(order)):
            b = a + 1
            while b < len(order) and xs[b] - xs[a] <= tol:
                if np.linalg.norm(pts[order[a]] - pts[order[b]]) <= tol:
                    ra, rb = find(bidx[order[a]]), find(bidx[order[b]])
                    if ra != rb:
                        parent[max(ra, rb)] = min(ra, rb)
                b += 1
        roots = np.array([find(i) for i in range(self.n2)])
        uniq = np.unique(roots)
        s2_to_s0 = np.searchsorted(uniq, roots)
        self._s0 = (s2_to_s0, len(uniq))
        return self._s0

    def glue_matrix(self) -> np.ndarray:
        """P (n2 x n0) with psi_{0,k} = sum_i P[i,k] psi_{2,i}."""
        s2_to_s0, n0 = self.s0_map()
        P = np.zeros((self.n2, n0))
        P[np.arange(self.n2), s2_to_s0] = 1.0
        return P

    # ------------------------------------------------------------ evaluation
    def element_corners(self) -> np.ndarray:
        """Physical corners (E, 4, 3) at local (0,0), (1,0), (0,1), (1,1)."""
        out = np.zeros((self.nelem, 4, 3))
        loc = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], dtype=np.float64)
        for j, mp in enumerate(self.maps):
            sel = np.nonzero(self.el_patch == j)[0]
            u = (self.el_ex[sel, None] + loc[None, :, 0]) * self.h
            v = (self.el_ey[sel, None] + loc[None, :, 1]) * self.h
            F, _, _ = mp.eval(u.ravel(), v.ravel())
            out[sel] = F.reshape(len(sel), 4, 3)
        return out

    def element_centers(self) -> np.ndarray:
        out = np.zeros((self.nelem, 3))
        for j, mp in enumerate(self.maps):
            sel = np.nonzero(self.el_patch == j)[0]
            F, _, _ = mp.eval((self.el_ex[sel] + 0.5) * self.h, (self.el_ey[sel] + 0.5) * self.h)
            out[sel] = F
        return out

    def eval_on_elements(self, elems: np.ndarray, uv_local: np.ndarray):
        """Geometry and local basis at element-local points.

        elems: (B,), uv_local: (B, Q, 2) in [0,1]^2 of each element.
        Returns dict of X, Fu, Fv, nt, a with shape (B, Q, 3|.), and the local
        basis phi, d_u phi, d_v phi with shape (B, Q, (p+1)^2) (w.r.t. the patch
        parameters u, v).
        """
        elems = np.asarray(elems)
        B, Q = uv_local.shape[:2]
        p = self.p
        u = (self.el_ex[elems][:, None] + uv_local[..., 0]) * self.h
        v = (self.el_ey[elems][:, None] + uv_local[..., 1]) * self.h
        X = np.zeros((B, Q, 3))
        Fu = np.zeros((B, Q, 3))
        Fv = np.zeros((B, Q, 3))
        for j in np.unique(self.el_patch[elems]):
            sel = self.el_patch[elems] == j
            F, du, dv = self.maps[j].eval(u[sel].ravel(), v[sel].ravel())
            X[sel] = F.reshape(-1, Q, 3)
            Fu[sel] = du.reshape(-1, Q, 3)
            Fv[sel] = dv.reshape(-1, Q, 3)
        nt = np.cross(Fu, Fv)
        a = np.linalg.norm(nt, axis=-1)
        bu, dbu = bspline.basis_and_derivative(self.knots, p, u.ravel())
        bv, dbv = bspline.basis_and_derivative(self.knots, p, v.ravel())
        bu, dbu = bu.reshape(B, Q, -1), dbu.reshape(B, Q, -1)
        bv, dbv = bv.reshape(B, Q, -1), dbv.reshape(B, Q, -1)
        ex = self.el_ex[elems][:, None, None]
        ey = self.el_ey[elems][:, None, None]
        idx = np.arange(p + 1)[None, None, :]
        lu = np.take_along_axis(bu, np.broadcast_to(ex + idx, (B, Q, p + 1)), axis=2)
        ldu = np.take_along_axis(dbu, np.broadcast_to(ex + idx, (B, Q, p + 1)), axis=2)
        lv = np.take_along_axis(bv, np.broadcast_to(ey + idx, (B, Q, p + 1)), axis=2)
        ldv = np.take_along_axis(dbv, np.broadcast_to(ey + idx, (B, Q, p + 1)), axis=2)
        # local index a = av * (p+1) + au
        phi = (lv[..., :, None] * lu[..., None, :]).reshape(B, Q, -1)
        dphi_u = (lv[..., :, None] * ldu[..., None, :]).reshape(B, Q, -1)
        dphi_v = (ldv[..., :, None] * lu[..., None, :]).reshape(B, Q, -1)
        return dict(X=X, Fu=Fu, Fv=Fv, nt=nt, a=a, phi=phi, dphi_u=dphi_u, dphi_v=dphi_v)
