"""O1: the dense fp64 Galerkin discretisation of the CFIE (the plain definition).

What is computed (rows = test functions at x, columns = trial functions at y,
bilinear L^2 duality without conjugation, Sec. 4.1):

* M_ij   = int psi_j psi_i dsigma                                     (Sec. 4.1)
* V_ij   = int int G(x,y) psi_j(y) psi_i(x)                            (Sec. 2, single layer)
* K*_ij  = int int dG/dn_x psi_j(y) psi_i(x)                           (adjoint double layer)
* K_ij   = int int dG/dn_y psi_j(y) psi_i(x)                           (double layer)
* W_ij   = <V curl psi_j, curl psi_i> - kappa^2 int int G n_x.n_y psi_j psi_i
                                                                     (Sec. 4.3, Maue)

all pulled back to the reference square (Sec. 4.2, eq. of the pulled-back
kernel): with n~ = d_u F x d_v F, a = |n~|, G = e^{i kappa r}/(4 pi r) and
H = G (i kappa r - 1)/r^2 (so grad_y G = H (y - x)):

    V     : a_x a_y G
    K*    : a_y H (x - y) . n~_x
    K     : a_x H (y - x) . n~_y
    W     : G [ c_i(x) . c_j(y) - kappa^2 (n~_x . n~_y) psi_i psi_j ],
            c = d_u psi d_v F - d_v psi d_u F   (the surface curl times a, Sec. 4.3)

Readings of the paper taken here:

* the curl term of the regularised W uses c_i(x).c_j(y) -- the printed closed
  form's "K^{-1}" and the missing surface measures are read as adj(K)^T and the
  measure-free integrand that the surface-curl formula gives;
* sound-soft system  (1/2 M + K* - i eta V) t = <d_n u_inc - i eta u_inc, psi>;
* sound-hard system  (1/2 M - K - i eta W) g = <u_inc - i eta d_n u_inc, psi>
  (the sign of the printed N2D equation's W term and of the variational form's
  K term are read as typos; derivation from u = u_inc + D u, W = -d_n D);
* scattered field    soft u_s = -S t (the printed potential lacks the minus),
                     hard u_s = D g;
* far-field pattern  u_s ~ e^{i kappa |x|}/|x| u_inf, hence
                     soft u_inf(x) = -(1/4 pi) int e^{-i kappa x.y} t(y) dsigma,
                     hard u_inf(x) = -(i kappa/4 pi) int (x.n_y) e^{-i kappa x.y} g(y) dsigma;
* default CFIE coupling eta_c = kappa (soft), -1/kappa (hard); any real eta != 0
  gives a uniquely solvable system;
* indirect comparison solutions (Sec. 5.2 measures its CFIE results against
  indirect solutions from a single-layer or adjoint-double-layer ansatz, without
  equations), read as the single-layer ansatz u_s = -S t with t on S^2:
  soft V t = <u_inc, psi> (the trace of u_s equals -u_inc), hard
  (K* - 1/2 M) t = <d_n u_inc, psi> (the exterior normal derivative of S t is
  (K* - 1/2) t, and d_n u_s = -d_n u_inc); the representation, far field and
  potential are then the sound-soft ones for both.

Quadrature (the paper defers to its references): tensor Gauss for regular
pairs with the order chosen from centre distance / diameter, Duffy-type rules
for touching pairs (``oracle.quadrature``).

Pinned by (tests/test_oracle_*.py): Mie series far field of the sphere (soft and
hard), the Gauss identity K 1 = -1/2 at kappa = 0 on the closed surface, the
sphere eigenvalues of V and W for the constant mode, complex symmetry of V and
W and K* = K^T, the flat-square closed form for the singular rules.
"""
from __future__ import annotations

import os

import numpy as np

from . import quadrature as qd
from .spaces import Discretization

LOCAL_CORNERS = ((0, 0), (1, 0), (0, 1), (1, 1))
OPS_SOFT = ("V", "Kstar")
OPS_HARD = ("K", "W")


def host_cores() -> int:
    """The CPUs this process may run on, or the OMP_NUM_THREADS share if that
    is smaller (a host shared by several GPU jobs sets it to the job's share)."""
    n = len(os.sched_getaffinity(0))
    try:
        n = min(n, int(os.environ.get("OMP_NUM_THREADS", n)))
    except ValueError:
        pass
    return max(1, n)


def default_eta(kappa: float, bc: str) -> float:
    """CFIE coupling (Sec. 2 gives none): eta = kappa for the sound-soft system
    and eta = -1/kappa for the sound-hard one, i.e. the combination
    (1/2 - K) + (i/kappa) W.  On the sphere every mode of these operators has a
    positive real part (closed-form symbols), which is what restarted GMRES needs."""
    return kappa if bc == "soft" else -1.0 / kappa


# ---------------------------------------------------------------------------
# Kernels
# ---------------------------------------------------------------------------

def _green(D, kappa):
    r = np.sqrt(np.sum(D * D, axis=-1))
    G = np.exp(1j * kappa * r) / (4.0 * np.pi * r)
    H = G * (1j * kappa * r - 1.0) / (r * r)
    return G, H


def _curl_vectors(d):
    # c_a = d_u phi_a d_v F - d_v phi_a d_u F : (B, Q, nb, 3)
    return (d["dphi_u"][..., None] * d["Fv"][:, :, None, :]
            - d["dphi_v"][..., None] * d["Fu"][:, :, None, :])


def _blocks_tensor(xd, yd, wx, wy, kappa, ops):
    """Blocks for a batch of pairs on tensor rules: x-points (B,Q), y-points (B,P)."""
    D = xd["X"][:, :, None, :] - yd["X"][:, None, :, :]
    G, H = _green(D, kappa)
    W2 = wx[:, None] * wy[None, :]
    ax, ay = xd["a"][:, :, None], yd["a"][:, None, :]
    px, py = xd["phi"], yd["phi"]
    out = {}

    def bil(k, lx=px, ly=py):
        return np.matmul(np.matmul(np.swapaxes(lx, 1, 2), k * W2), ly)

    if "V" in ops:
        out["V"] = bil(ax * ay * G)
    if "Kstar" in ops:
        out["Kstar"] = bil(ay * H * np.sum(D * xd["nt"][:, :, None, :], axis=-1))
    if "K" in ops:
        out["K"] = bil(-ax * H * np.sum(D * yd["nt"][:, None, :, :], axis=-1))
    if "W" in ops:
        cx, cy = _curl_vectors(xd), _curl_vectors(yd)
        nn = np.sum(xd["nt"][:, :, None, :] * yd["nt"][:, None, :, :], axis=-1)
        w = sum(bil(G, cx[..., c], cy[..., c]) for c in range(3))
        out["W"] = w - kappa ** 2 * bil(G * nn)
    return out


def _blocks_paired(xd, yd, w, kappa, ops):
    """Blocks for a batch of pairs on paired (singular) rules: (B,Q) points."""
    D = xd["X"] - yd["X"]
    G, H = _green(D, kappa)
    px, py = xd["phi"], yd["phi"]
    out = {}

    def bil(k, lx=px, ly=py):
        return np.einsum("bq,bqa,bqc->bac", k * w[None, :], lx, ly)

    if "V" in ops:
        out["V"] = bil(xd["a"] * yd["a"] * G)
    if "Kstar" in ops:
        out["Kstar"] = bil(yd["a"] * H * np.sum(D * xd["nt"], axis=-1))
    if "K" in ops:
        out["K"] = bil(-xd["a"] * H * np.sum(D * yd["nt"], axis=-1))
    if "W" in ops:
        cx, cy = _curl_vectors(xd), _curl_vectors(yd)
        nn = np.sum(xd["nt"] * yd["nt"], axis=-1)
        wv = sum(bil(G, cx[..., c], cy[..., c]) for c in range(3))
        out["W"] = wv - kappa ** 2 * bil(G * nn)
    return out


# ---------------------------------------------------------------------------
# Element-pair classification and quadrature selection
# ---------------------------------------------------------------------------

class PairRules:
    """Oracle quadrature orders: regular pairs by centre distance / diameter,
    touching pairs by the Duffy rules at order n_sing."""

    def __init__(self, n_far=6, n_mid=8, n_near=10, n_sing=10, r_far=6.0, r_mid=3.0):
        self.n_far, self.n_mid, self.n_near, self.n_sing = n_far, n_mid, n_near, n_sing
        self.r_far, self.r_mid = r_far, r_mid

    def regular_order(self, ratio: np.ndarray) -> np.ndarray:
        n = np.full(ratio.shape, self.n_near)
        n[ratio >= self.r_mid] = self.n_mid
        n[ratio >= self.r_far] = self.n_far
        return n


class DenseBEM:
    """Dense Galerkin CFIE matrices, right-hand sides and far fields."""

    def __init__(self, patches, p: int, m: int, kappa: float, bc: str = "soft",
                 eta: float | None = None, rules: PairRules | None = None,
                 workers: int | None = None, formulation: str = "cfie"):
        if formulation not in ("cfie", "single_layer"):
            raise ValueError("formulation must be 'cfie' or 'single_layer'")
        self.disc = Discretization(patches, p, m)
        self.kappa = float(kappa)
        self.bc = bc
        self.formulation = formulation
        # operator family: "soft" = S^2 with V, K* and the single-layer representation
        self.family = "soft" if (bc == "soft" or formulation == "single_layer") else "hard"
        self.eta = default_eta(kappa, bc) if eta is None or eta == 0 else float(eta)
        self.rules = rules or PairRules()
        self.corners = self.disc.element_corners()
        self.centers = self.disc.element_centers()
        c = self.corners
        self.diam = np.max(np.linalg.norm(c[:, :, None, :] - c[:, None, :, :], axis=-1), axis=(1, 2))
        self.ops = OPS_SOFT if self.family == "soft" else OPS_HARD
        self.workers = workers if workers is not None else host_cores()

    # ------------------------------------------------------------ dimensions
    @property
    def n(self) -> int:
        return self.disc.n2 if self.family == "soft" else self.disc.s0_map()[1]

    # -------------------------------------------------------- classification
    def classify(self, e: int):
        """For target element e: per source element f its type (0 regular,
        1 vertex, 2 edge, 4 identical), the square symmetries bringing the pair
        into canonical position, and the regular Gauss order."""
        d = np.linalg.norm(self.corners[e][None, :, None, :] - self.corners[:, None, :, :], axis=-1)
        tol = 1e-9 * self.diam.max()
        shared = d < tol
        nsh = shared.sum(axis=(1, 2))
        typ = np.where(nsh >= 4, 4, nsh)
        te = np.zeros(len(typ), dtype=int)
        tf = np.zeros(len(typ), dtype=int)
        for f in np.nonzero((typ == 1) | (typ == 2))[0]:
            ij = np.argwhere(shared[f])
            if typ[f] == 1:
                ci, cj = ij[0]
                te[f] = qd.d4_find({(0, 0): LOCAL_CORNERS[ci]})
                tf[f] = qd.d4_find({(0, 0): LOCAL_CORNERS[cj]})
            else:
                (ci1, cj1), (ci2, cj2) = ij
                te[f] = qd.d4_find({(0, 0): LOCAL_CORNERS[ci1], (1, 0): LOCAL_CORNERS[ci2]})
                tf[f] = qd.d4_find({(0, 0): LOCAL_CORNERS[cj1], (1, 0): LOCAL_CORNERS[cj2]})
        ratio = np.linalg.norm(self.centers - self.centers[e], axis=1) / np.maximum(self.diam, self.diam[e])
        order = self.rules.regular_order(ratio)
        return typ, te, tf, order

    # ------------------------------------------------------------ the blocks
    def element_row_blocks(self, e: int, ops=None, chunk: int = 256, sources=None):
        """Blocks (e, f) for one target element and all (or the given) source
        elements f: dict op -> (E, nloc, nloc), zero for sources not computed."""
        ops = self.ops if ops is None else ops
        disc = self.disc
        E, nl = disc.nelem, disc.nloc
        out = {op: np.zeros((E, nl, nl), dtype=np.complex128) for op in ops}
        typ, te, tf, order = self.classify(e)
        if sources is not None:
            keep = np.zeros(E, dtype=bool)
            keep[np.asarray(sources)] = True
            typ = np.where(keep, typ, -1)
        h4 = disc.h ** 4
        # regular pairs, grouped by order
        for n in np.unique(order[typ == 0]):
            fs = np.nonzero((typ == 0) & (order == n))[0]
            pts, w = qd.tensor2(int(n))
            xd1 = disc.eval_on_elements(np.array([e]), pts[None])
            for s in range(0, len(fs), chunk):
                fb = fs[s:s + chunk]
                B = len(fb)
                xd = {k: np.broadcast_to(v, (B,) + v.shape[1:]) for k, v in xd1.items()}
                yd = disc.eval_on_elements(fb, np.broadcast_to(pts, (B,) + pts.shape))
                blk = _blocks_tensor(xd, yd, w, w, self.kappa, ops)
                for op in ops:
                    out[op][fb] = blk[op] * h4
        # touching pairs
        ns = self.rules.n_sing
        for t, rule in ((4, qd.identical), (2, qd.edge), (1, qd.vertex)):
            fs = np.nonzero(typ == t)[0]
            if len(fs) == 0:
                continue
            xs, ys, w = rule(ns)
            for f in fs:
                xl = qd.d4_apply(int(te[f]), xs)
                yl = qd.d4_apply(int(tf[f]), ys)
                xd = disc.eval_on_elements(np.array([e]), xl[None])
                yd = disc.eval_on_elements(np.array([f]), yl[None])
                blk = _blocks_paired(xd, yd, w, self.kappa, ops)
                for op in ops:
                    out[op][f] = blk[op][0] * h4
        return out

    def mass_block(self, e: int, n: int = 8) -> np.ndarray:
        pts, w = qd.tensor2(n)
        d = self.disc.eval_on_elements(np.array([e]), pts[None])
        return np.einsum("q,q,qa,qb->ab", w, d["a"][0], d["phi"][0], d["phi"][0]) * self.disc.h ** 2

    # ------------------------------------------------------------ assembly
    def operator_rows_s2(self, rows_s2, ops=None):
        """Rows (S^2 numbering) of each single operator and of M: op -> (R, n2)."""
        ops = self.ops if ops is None else ops
        disc = self.disc
        rows_s2 = np.asarray(rows_s2)
        assert len(np.unique(rows_s2)) == len(rows_s2), "rows must be distinct"
        where = {int(r): i for i, r in enumerate(rows_s2)}
        out = {op: np.zeros((len(rows_s2), disc.n2), dtype=np.complex128) for op in ops + ("M",)}
        targets = np.unique(np.nonzero(np.isin(disc.el_dofs, rows_s2))[0])
        cols = disc.el_dofs.ravel()
        for e, (blk, mb) in zip(targets, self._map_targets(targets, ops)):
            loc = [(where[int(disc.el_dofs[e, a])], a) for a in range(disc.nloc)
                   if int(disc.el_dofs[e, a]) in where]
            for ri, a in loc:
                for op in ops:
                    np.add.at(out[op][ri], cols, blk[op][:, a, :].ravel())
                np.add.at(out["M"][ri], disc.el_dofs[e], mb[a])
        return out

    def _one_restricted(self, e, fs):
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            return self.element_row_blocks(int(e), sources=fs), self.mass_block(int(e))

    def restricted_row_blocks(self, targets, sources):
        """element_row_blocks(e, sources=fs) and the mass block for every
        (e, fs) in zip(targets, sources), over the worker pool."""
        if self.workers <= 1 or len(targets) < 4:
            for e, fs in zip(targets, sources):
                yield self._one_restricted(e, fs)
            return
        import concurrent.futures as cf
        import multiprocessing as mp
        with cf.ProcessPoolExecutor(self.workers, mp_context=mp.get_context("fork")) as ex:
            yield from ex.map(self._one_restricted, targets, sources)

    def _one_target(self, e, ops):
        from threadpoolctl import threadpool_limits
        with threadpool_limits(1):
            return self.element_row_blocks(int(e), ops), self.mass_block(int(e))

    def _map_targets(self, targets, ops):
        """Element row blocks for many targets, over a pool of forked workers."""
        workers = self.workers
        if workers <= 1 or len(targets) < 4:
            for e in targets:
                yield self._one_target(e, ops)
            return
        import concurrent.futures as cf
        import multiprocessing as mp
        with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
            yield from ex.map(self._one_target, targets, [ops] * len(targets))

    def _combine(self, parts):
        if self.formulation == "single_layer":
            if self.bc == "soft":
                return parts["V"]
            return -0.5 * parts["M"] + parts["Kstar"]
        if self.bc == "soft":
            return 0.5 * parts["M"] + parts["Kstar"] - 1j * self.eta * parts["V"]
        return 0.5 * parts["M"] - parts["K"] - 1j * self.eta * parts["W"]

    def operator_matrices(self):
        """Full dense matrices in the solution space: dict op -> (n, n)."""
        disc = self.disc
        parts = self.operator_rows_s2(np.arange(disc.n2))
        if self.family == "hard":
            P = disc.glue_matrix()
            parts = {k: P.T @ v @ P for k, v in parts.items()}
        return parts

    def matrix(self) -> np.ndarray:
        return self._combine(self.operator_matrices())

    def rows(self, rows) -> np.ndarray:
        """Rows of the CFIE matrix in the solution space (S^2 soft, S^0 hard)."""
        disc = self.disc
        rows = np.asarray(rows)
        if self.family == "soft":
            return self._combine(self.operator_rows_s2(rows))
        s2_to_s0, n0 = disc.s0_map()
        reps = np.nonzero(np.isin(s2_to_s0, rows))[0]
        parts = self.operator_rows_s2(reps)
        R = np.zeros((len(rows), len(reps)))
        for k, r in enumerate(rows):
            R[k, s2_to_s0[reps] == r] = 1.0

        def glue(v):
            # (R v) P with P the S^0 -> S^2 gluing matrix, without forming P:
            # column i of R v adds to column s2_to_s0[i]
            rv = R @ v
            out = np.zeros((rv.shape[0], n0), dtype=rv.dtype)
            np.add.at(out, (slice(None), s2_to_s0), rv)
            return out

        parts = {k: glue(v) for k, v in parts.items()}
        return self._combine(parts)

    # ------------------------------------------------------------ rhs / far field
    def rhs(self, d, n: int = 8) -> np.ndarray:
        """Load vector for incidence direction d (Sec. 4.1 right-hand sides)."""
        disc = self.disc
        d = np.asarray(d, dtype=np.float64)
        d = d / np.linalg.norm(d)
        pts, w = qd.tensor2(n)
        E = disc.nelem
        dd = disc.eval_on_elements(np.arange(E), np.broadcast_to(pts, (E,) + pts.shape))
        k = self.kappa
        uinc = np.exp(1j * k * dd["X"] @ d)
        dn_a = 1j * k * (dd["nt"] @ d) * uinc          # a * d_n u_inc
        if self.formulation == "single_layer":
            f = dd["a"] * uinc if self.bc == "soft" else dn_a
        elif self.bc == "soft":
            f = dn_a - 1j * self.eta * dd["a"] * uinc
        else:
            f = dd["a"] * uinc - 1j * self.eta * dn_a
        loc = np.einsum("eq,q,eqa->ea", f, w, dd["phi"]) * disc.h ** 2
        b = np.zeros(disc.n2, dtype=np.complex128)
        np.add.at(b, disc.el_dofs.ravel(), loc.ravel())
        if self.family == "hard":
            b = disc.glue_matrix().T @ b
        return b

    def farfield(self, coeffs, obs, n: int = 8) -> np.ndarray:
        """Far-field pattern u_inf at unit directions obs for solution coeffs."""
        disc = self.disc
        c = np.asarray(coeffs, dtype=np.complex128)
        if self.family == "hard":
            c = disc.glue_matrix() @ c
        obs = np.asarray(obs, dtype=np.float64)
        obs = obs / np.linalg.norm(obs, axis=1, keepdims=True)
        pts, w = qd.tensor2(n)
        E = disc.nelem
        dd = disc.eval_on_elements(np.arange(E), np.broadcast_to(pts, (E,) + pts.shape))
        dens = np.einsum("eqa,ea->eq", dd["phi"], c[disc.el_dofs])  # density at points
        k = self.kappa
        ph = np.exp(-1j * k * np.einsum("eqc,oc->oeq", dd["X"], obs))
        wq = w[None, :] * disc.h ** 2
        if self.family == "soft":
            u = -np.einsum("oeq,eq,eq->o", ph, dens * dd["a"], np.broadcast_to(wq, dens.shape)) / (4 * np.pi)
        else:
            xn = np.einsum("eqc,oc->oeq", dd["nt"], obs)
            u = -1j * k * np.einsum("oeq,oeq,eq->o", ph, xn, dens * wq) / (4 * np.pi)
        return u

    def potential(self, coeffs, points, n: int = 10) -> np.ndarray:
        """Scattered field at points off the boundary from the representation
        formulas (Sec. 2 and the readings above): soft u_s(x) = -int G(x,y)
        t(y) dsigma_y, hard u_s(x) = int dG(x,y)/dn_y g(y) dsigma_y with
        G = e^{i kappa r}/(4 pi r), r = |x - y|, so that dG/dn_y =
        G (i kappa r - 1)/r^2 (y - x).n_y; tensor Gauss of order n on every
        element (for points well away from the surface)."""
        disc = self.disc
        c = np.asarray(coeffs, dtype=np.complex128)
        if self.family == "hard":
            c = disc.glue_matrix() @ c
        P = np.atleast_2d(np.asarray(points, dtype=np.float64))
        pts, w = qd.tensor2(n)
        E = disc.nelem
        dd = disc.eval_on_elements(np.arange(E), np.broadcast_to(pts, (E,) + pts.shape))
        dens = np.einsum("eqa,ea->eq", dd["phi"], c[disc.el_dofs]) * (w[None, :] * disc.h ** 2)
        k = self.kappa
        out = np.zeros(len(P), dtype=np.complex128)
        for i, x in enumerate(P):
            dy = dd["X"] - x                      # y - x
            r = np.linalg.norm(dy, axis=-1)
            G = np.exp(1j * k * r) / (4 * np.pi * r)
            if self.family == "soft":
                out[i] = -np.sum(G * dd["a"] * dens)
            else:
                out[i] = np.sum(G * (1j * k * r - 1) / r ** 2 * np.einsum("eqc,eqc->eq", dy, dd["nt"]) * dens)
        return out

    def solve(self, d) -> np.ndarray:
        """LU solve of the dense system (LAPACK zgesv through numpy)."""
        return np.linalg.solve(self.matrix(), self.rhs(d))
