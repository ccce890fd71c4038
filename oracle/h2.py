"""O2: the reference-domain interpolation H^2 matrix, step by step (Sec. 4.4).

Algorithm (in the paper's order: clusters, admissibility, degenerate kernel by
interpolation of the pulled-back kernel on the reference domain, H^2 format):

1. Clusters: every patch's reference square [0,1]^2 is bisected dyadically; a
   cluster (patch, l, cx, cy) covers [cx, cx+1] x [cy, cy+1] / 2^l.  Leaves sit at
   level L = m - d (4^d elements each).
2. Block partition: starting from all pairs of patch roots, a pair is stored as
   a far (admissible) block if the admissibility condition holds, as a near
   block if both are leaves, and is subdivided into its 4 x 4 child pairs
   otherwise.  Admissibility (the paper gives only eta = 1.6; reading A):
       dist(B_t, B_s) >= eta * max(diam B_t, diam B_s)
   with B the axis-aligned box of the cluster's Bezier control points (these
   contain the surface piece by the convex hull property, weights > 0), plus the
   optional cap kappa * max(diam) <= kcap, and only for clusters that lie
   inside one knot span of their patch's geometry in both directions (Sec. 3.2
   takes the patch mappings to be smooth; across an interior knot a spline
   mapping is only finitely smooth, and the interpolant of the pulled-back
   kernel no longer converges geometrically in q).
3. Degenerate kernel: on an admissible pair the pulled-back kernel
   k(x^, y^) is replaced by its tensor Chebyshev interpolant of degree q in
   each reference coordinate of both clusters (rank (q+1)^2, Sec. 4.4):
       k(x^, y^) ~ sum_{a,b} k(x^_a, y^_b) L^t_a(x^) L^s_b(y^)
   with Chebyshev points of the first kind mapped to the cluster squares.
4. H^2 format: leaf moments  M_s[b, j] = int_s L^s_b psi_j  (geometry free),
   transfers T_c[g, a] = L^P_a(x^c_g) (nestedness: the parent's interpolant is
   reproduced exactly on the child), coupling matrices K_ts[a, b].
5. Matrix-vector product: upward pass x^_s = M_s x (leaves),
   x^_P = sum_c T_c^T x^_c; coupling y^_t += K_ts x^_s; downward pass
   y^_c += T_c y^_P; back projection y += M_t^T y^_t; plus the near blocks.

The near field is taken from O1 (``oracle.galerkin``) element blocks.

Pinned by: exact reproduction of a polynomial test kernel of degree <= q,
eta -> infinity giving exactly O1's matrix, geometric decay of the error
against O1 in q (tests/test_oracle_h2.py).
"""
from __future__ import annotations

import functools
from dataclasses import dataclass

import numpy as np

from . import quadrature as qd
from .galerkin import DenseBEM


def cheb_nodes01(q: int) -> np.ndarray:
    k = np.arange(q + 1)
    return 0.5 * (1.0 - np.cos((2 * k + 1) * np.pi / (2 * q + 2)))


def lagrange(nodes: np.ndarray, t) -> np.ndarray:
    """L_a(t) for all nodes a: (len(t), len(nodes))."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    out = np.ones((len(t), len(nodes)))
    for a in range(len(nodes)):
        for b in range(len(nodes)):
            if a != b:
                out[:, a] *= (t - nodes[b]) / (nodes[a] - nodes[b])
    return out


@dataclass(frozen=True)
class Cluster:
    patch: int
    level: int
    cx: int
    cy: int


class H2Oracle:
    def __init__(self, bem: DenseBEM, q: int, eta: float = 1.6, leaf_depth: int = 2,
                 kcap: float = 0.0, coupling_kernel=None):
        if bem.formulation != "cfie":
            raise ValueError("H2Oracle follows the CFIE operators only")
        self.bem = bem
        self.disc = disc = bem.disc
        self.q, self.eta, self.kcap = q, eta, kcap
        self.d = min(leaf_depth, disc.m)
        self.L = disc.m - self.d
        self.nq = (q + 1) ** 2
        self.t = cheb_nodes01(q)
        self.coupling_kernel = coupling_kernel
        self._element_boxes()
        self._build_blocks()

    # ------------------------------------------------------------ boxes
    def _element_boxes(self):
        """Per element: AABB of its rational Bezier control points."""
        disc = self.disc
        E = disc.nelem
        self.el_lo = np.zeros((E, 3))
        self.el_hi = np.zeros((E, 3))
        for j, mp in enumerate(disc.maps):
            pu, pv = mp.pu, mp.pv
            tu, tv = np.linspace(0, 1, pu + 1), np.linspace(0, 1, pv + 1)
            from math import comb
            Vu = np.array([[comb(pu, a) * t ** a * (1 - t) ** (pu - a) for a in range(pu + 1)] for t in tu])
            Vv = np.array([[comb(pv, a) * t ** a * (1 - t) ** (pv - a) for a in range(pv + 1)] for t in tv])
            Vu_inv, Vv_inv = np.linalg.inv(Vu), np.linalg.inv(Vv)
            for e in np.nonzero(disc.el_patch == j)[0]:
                u = (disc.el_ex[e] + tu) * disc.h
                v = (disc.el_ey[e] + tv) * disc.h
                uu, vv = np.meshgrid(u, v, indexing="xy")       # (pv+1, pu+1)
                F, _, _ = mp.eval(uu.ravel(), vv.ravel())
                W = self._weight(mp, uu.ravel(), vv.ravel())
                Hm = np.concatenate([F * W[:, None], W[:, None]], axis=1).reshape(pv + 1, pu + 1, 4)
                C = np.einsum("ab,bcx,dc->adx", Vv_inv, Hm, Vu_inv)  # Bernstein coefficients
                if np.any(C[..., 3] <= 0):
                    raise ValueError("non-positive Bezier weight")
                P = (C[..., :3] / C[..., 3:]).reshape(-1, 3)
                self.el_lo[e], self.el_hi[e] = P.min(0), P.max(0)

    @staticmethod
    def _weight(mp, u, v):
        from . import bspline
        bu = bspline.basis(mp.ku, mp.pu, u)
        bv = bspline.basis(mp.kv, mp.pv, v)
        return np.einsum("nj,ni,ji->n", bv, bu, mp.w)

    def cluster_elements(self, c: Cluster) -> np.ndarray:
        disc = self.disc
        s = 2 ** (disc.m - c.level)
        ex = np.arange(c.cx * s, (c.cx + 1) * s)
        ey = np.arange(c.cy * s, (c.cy + 1) * s)
        return (c.patch * disc.nel1 ** 2 + ey[:, None] * disc.nel1 + ex[None, :]).ravel()

    @functools.lru_cache(maxsize=None)
    def box(self, c: Cluster):
        el = self.cluster_elements(c)
        return self.el_lo[el].min(0), self.el_hi[el].max(0)

    def inside_one_span(self, c: Cluster) -> bool:
        """No interior geometry knot lies strictly inside the cluster's square."""
        mp = self.disc.maps[c.patch]
        w = 2.0 ** -c.level
        for knots, i in ((mp.ku, c.cx), (mp.kv, c.cy)):
            a, b = i * w, (i + 1) * w
            if np.any((knots > a + 1e-12) & (knots < b - 1e-12)):
                return False
        return True

    def admissible(self, t: Cluster, s: Cluster) -> bool:
        if not (self.inside_one_span(t) and self.inside_one_span(s)):
            return False
        lt, ht = self.box(t)
        ls, hs = self.box(s)
        gap = np.maximum(0.0, np.maximum(ls - ht, lt - hs))
        dist = float(np.sqrt(np.sum(gap * gap)))
        dm = max(float(np.linalg.norm(ht - lt)), float(np.linalg.norm(hs - ls)))
        if self.kcap > 0 and self.bem.kappa * dm > self.kcap:
            return False
        return dist >= self.eta * dm

    @staticmethod
    def children(c: Cluster):
        return [Cluster(c.patch, c.level + 1, 2 * c.cx + i, 2 * c.cy + j) for j in (0, 1) for i in (0, 1)]

    def _build_blocks(self):
        self.far, self.near = [], []
        stack = [(Cluster(a, 0, 0, 0), Cluster(b, 0, 0, 0))
                 for a in range(self.disc.npatch) for b in range(self.disc.npatch)]
        while stack:
            t, s = stack.pop()
            if self.admissible(t, s):
                self.far.append((t, s))
            elif t.level == self.L:
                self.near.append((t, s))
            else:
                stack.extend((tc, sc) for tc in self.children(t) for sc in self.children(s))
        self.far.sort(key=lambda b: (b[0].level, b[0].patch, b[0].cy, b[0].cx, b[1].patch, b[1].cy, b[1].cx))
        self.near.sort(key=lambda b: (b[0].patch, b[0].cy, b[0].cx, b[1].patch, b[1].cy, b[1].cx))

    # ------------------------------------------------------------ interpolation
    def nodes(self, c: Cluster):
        """Reference coordinates (nq, 2) of the cluster's tensor Chebyshev nodes,
        index a = a_v (q+1) + a_u."""
        s = 2.0 ** (-c.level)
        u = (c.cx + self.t) * s
        v = (c.cy + self.t) * s
        uu, vv = np.meshgrid(u, v, indexing="xy")
        return np.stack([uu.ravel(), vv.ravel()], axis=1)

    def transfer_1d(self, child_bit: int) -> np.ndarray:
        """T[g, a] = L^parent_a(child node g) in one coordinate; child_bit 0/1 is
        the lower/upper half of the parent interval."""
        return lagrange(self.t, 0.5 * (child_bit + self.t))

    @functools.lru_cache(maxsize=None)
    def leaf_moment_1d(self, level: int, c: int, deriv: bool = False) -> np.ndarray:
        """m[b, i] = int_{cluster interval} L_b(t) b_i(t) dt over the whole knot
        vector's basis (or b_i' for the derivative moments)."""
        from . import bspline
        disc = self.disc
        s = 2 ** (disc.m - level)
        x, w = qd.gauss01((self.q + disc.p) // 2 + 2)
        out = np.zeros((self.q + 1, disc.k))
        for e in range(c * s, (c + 1) * s):
            t = (e + x) * disc.h
            val, der = bspline.basis_and_derivative(disc.knots, disc.p, t)
            L = lagrange(self.t, t * 2 ** level - c)
            out += np.einsum("g,gb,gi->bi", w * disc.h, L, der if deriv else val)
        out.flags.writeable = False   # cached: shared by every caller
        return out

    def cluster_moment_patch(self, c: Cluster, kind=(0, 0)) -> np.ndarray:
        """The moments of cluster c against the B-splines of its own patch
        (nq, k^2), computed directly (not through the transfers):
        int_c L_a(x^) d^kind psi_j(x^) dx^.  Every other S^2 function vanishes
        on the cluster."""
        mu = self.leaf_moment_1d(c.level, c.cx, kind[0] == 1)
        mv = self.leaf_moment_1d(c.level, c.cy, kind[1] == 1)
        k = self.disc.k
        return np.einsum("ai,bj->baji", mu, mv).reshape(self.nq, k * k)

    def cluster_moment(self, c: Cluster, kind=(0, 0)) -> np.ndarray:
        """Moment matrix (nq, n2) of cluster c (zero outside its patch)."""
        k = self.disc.k
        M = np.zeros((self.nq, self.disc.n2))
        M[:, c.patch * k * k:(c.patch + 1) * k * k] = self.cluster_moment_patch(c, kind)
        return M

    # ------------------------------------------------------------ kernels at nodes
    @functools.lru_cache(maxsize=None)
    def node_geometry(self, c: Cluster):
        X = self.nodes(c)
        mp = self.disc.maps[c.patch]
        F, Fu, Fv = mp.eval(X[:, 0], X[:, 1])
        nt = np.cross(Fu, Fv)
        return dict(X=F, Fu=Fu, Fv=Fv, nt=nt, a=np.linalg.norm(nt, axis=1), uv=X)

    def coupling(self, t: Cluster, s: Cluster) -> dict:
        """Pulled-back CFIE kernel at node pairs; soft: {'pp'}, hard: {'pp',
        ('d', a, b)}.  pp acts between plain moments, ('d', a, b) between the
        derivative moments d_a psi (test) and d_b psi (trial)."""
        gx, gy = self.node_geometry(t), self.node_geometry(s)
        if self.coupling_kernel is not None:
            return {"pp": self.coupling_kernel(gx["uv"][:, None, :], gy["uv"][None, :, :])}
        k = self.bem.kappa
        eta = self.bem.eta
        D = gx["X"][:, None, :] - gy["X"][None, :, :]
        r = np.linalg.norm(D, axis=-1)
        G = np.exp(1j * k * r) / (4 * np.pi * r)
        H = G * (1j * k * r - 1.0) / (r * r)
        ax, ay = gx["a"][:, None], gy["a"][None, :]
        if self.bem.bc == "soft":
            kstar = ay * H * np.einsum("abc,ac->ab", D, gx["nt"])
            return {"pp": kstar - 1j * eta * ax * ay * G}
        kdl = -ax * H * np.einsum("abc,bc->ab", D, gy["nt"])
        nn = gx["nt"] @ gy["nt"].T
        out = {"pp": -kdl - 1j * eta * (-k * k * G * nn)}
        Jx = (gx["Fv"], -gx["Fu"])
        Jy = (gy["Fv"], -gy["Fu"])
        for a in range(2):
            for b in range(2):
                out[("d", a, b)] = -1j * eta * G * (Jx[a] @ Jy[b].T)
        return out

    # ------------------------------------------------------------ products
    def far_matrix(self) -> np.ndarray:
        """Dense S^2 matrix of the far field, built block by block from direct
        cluster moments (independent of the transfer recursion)."""
        n2 = self.disc.n2
        A = np.zeros((n2, n2), dtype=np.complex128)
        kinds = {"pp": ((0, 0), (0, 0))}
        for a in range(2):
            for b in range(2):
                kinds[("d", a, b)] = ((1, 0) if a == 0 else (0, 1), (1, 0) if b == 0 else (0, 1))
        kk = self.disc.k ** 2
        for t, s in self.far:
            K = self.coupling(t, s)
            rt = slice(t.patch * kk, (t.patch + 1) * kk)
            rs = slice(s.patch * kk, (s.patch + 1) * kk)
            for key, mat in K.items():
                kt, ks = kinds[key]
                A[rt, rs] += self.cluster_moment_patch(t, kt).T @ mat @ self.cluster_moment_patch(s, ks)
        return A

    def near_pairs(self):
        """Element pairs (e, f) covered by near blocks."""
        out = []
        for t, s in self.near:
            et, es = self.cluster_elements(t), self.cluster_elements(s)
            out.append(np.stack(np.meshgrid(et, es, indexing="ij"), -1).reshape(-1, 2))
        return np.concatenate(out) if out else np.zeros((0, 2), int)

    def near_matrix(self) -> np.ndarray:
        """Dense S^2 matrix of the near field (O1 element blocks on near pairs,
        plus 1/2 M)."""
        bem, disc = self.bem, self.disc
        n2 = disc.n2
        A = np.zeros((n2, n2), dtype=np.complex128)
        pairs = self.near_pairs()
        targets = np.unique(pairs[:, 0])
        sources = [pairs[pairs[:, 0] == e, 1] for e in targets]
        for e, fs, (blk, mass) in zip(targets, sources, bem.restricted_row_blocks(targets, sources)):
            comb = self._combine_blocks(blk)
            for f in fs:
                A[np.ix_(disc.el_dofs[e], disc.el_dofs[f])] += comb[f]
            A[np.ix_(disc.el_dofs[e], disc.el_dofs[e])] += 0.5 * mass
        return A

    def _combine_blocks(self, blk):
        eta = self.bem.eta
        if self.bem.bc == "soft":
            return blk["Kstar"] - 1j * eta * blk["V"]
        return -blk["K"] - 1j * eta * blk["W"]

    def to_solution_space(self, A2: np.ndarray) -> np.ndarray:
        if self.bem.bc == "soft":
            return A2
        P = self.disc.glue_matrix()
        return P.T @ A2 @ P

    # ------------------------------------------------------------ step by step
    def far_apply(self, x: np.ndarray) -> np.ndarray:
        """Far-field product by the upward / coupling / downward passes; x and the
        result in the solution space."""
        disc = self.disc
        if self.bem.bc == "hard":
            P = disc.glue_matrix()
            x2 = P @ x
        else:
            x2 = np.asarray(x, dtype=np.complex128)
        k = disc.k
        kinds = [(0, 0)] if self.bem.bc == "soft" else [(0, 0), (1, 0), (0, 1)]
        T1 = [self.transfer_1d(0), self.transfer_1d(1)]
        # upward pass
        up = {}
        for c in self._all_clusters(self.L):
            X = x2[c.patch * k * k:(c.patch + 1) * k * k].reshape(k, k)  # (iv, iu)
            for ki, kd in enumerate(kinds):
                mu = self.leaf_moment_1d(self.L, c.cx, kd[0] == 1)
                mv = self.leaf_moment_1d(self.L, c.cy, kd[1] == 1)
                up[(c, ki)] = (mv @ X @ mu.T).ravel()          # index a_v (q+1) + a_u
        for lev in range(self.L - 1, -1, -1):
            for c in self._all_clusters(lev):
                for ki in range(len(kinds)):
                    acc = np.zeros(self.nq, dtype=np.complex128)
                    for ch in self.children(c):
                        Tu, Tv = T1[ch.cx - 2 * c.cx], T1[ch.cy - 2 * c.cy]
                        Y = up[(ch, ki)].reshape(self.q + 1, self.q + 1)
                        acc += (Tv.T @ Y @ Tu).ravel()
                    up[(c, ki)] = acc
        # coupling
        down = {}
        keymap = {"pp": (0, 0)}
        for a in range(2):
            for b in range(2):
                keymap[("d", a, b)] = (1 + a, 1 + b)
        for t, s in self.far:
            for key, mat in self.coupling(t, s).items():
                ko, ki = keymap[key]
                down.setdefault((t, ko), np.zeros(self.nq, dtype=np.complex128))
                down[(t, ko)] += mat @ up[(s, ki)]
        # downward pass
        for lev in range(0, self.L):
            for c in self._all_clusters(lev):
                for ko in range(len(kinds)):
                    if (c, ko) not in down:
                        continue
                    Y = down[(c, ko)].reshape(self.q + 1, self.q + 1)
                    for ch in self.children(c):
                        Tu, Tv = T1[ch.cx - 2 * c.cx], T1[ch.cy - 2 * c.cy]
                        down.setdefault((ch, ko), np.zeros(self.nq, dtype=np.complex128))
                        down[(ch, ko)] += (Tv @ Y @ Tu.T).ravel()
        # back projection
        y2 = np.zeros(disc.n2, dtype=np.complex128)
        for c in self._all_clusters(self.L):
            for ko, kd in enumerate(kinds):
                if (c, ko) not in down:
                    continue
                mu = self.leaf_moment_1d(self.L, c.cx, kd[0] == 1)
                mv = self.leaf_moment_1d(self.L, c.cy, kd[1] == 1)
                Y = down[(c, ko)].reshape(self.q + 1, self.q + 1)
                y2[c.patch * k * k:(c.patch + 1) * k * k] += (mv.T @ Y @ mu).ravel()
        if self.bem.bc == "hard":
            return disc.glue_matrix().T @ y2
        return y2

    def _all_clusters(self, level: int):
        n = 2 ** level
        return [Cluster(p, level, cx, cy) for p in range(self.disc.npatch)
                for cy in range(n) for cx in range(n)]

    def matrix(self) -> np.ndarray:
        """Dense H^2 CFIE matrix in the solution space (small cases)."""
        return self.to_solution_space(self.far_matrix() + self.near_matrix())
