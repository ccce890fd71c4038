"""Seeded, synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *constructs inputs*: NURBS control nets of the scatterers,
incident / observation directions and random test vectors.  It holds none of
the method's arithmetic (no basis evaluation of the discrete spaces, no kernel,
no quadrature); the oracle and the HIP library each evaluate these patches with
their own code.

Patches follow the NURBS form of the paper (Sec. 3.2, patch maps F_j: control
points c and weights w > 0 on open knot vectors).  A patch is stored as
``cpw[ncp_v][ncp_u][4] = (x, y, z, w)`` -- Cartesian control point and its weight,
*not* homogeneous coordinates.  All patches are oriented so that
d_u F x d_v F points out of the enclosed volume (outward normals, Sec. 2).
"""
from __future__ import annotations

import dataclasses
import functools
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class Patch:
    deg_u: int
    deg_v: int
    knots_u: np.ndarray  # (ncp_u + deg_u + 1,)
    knots_v: np.ndarray  # (ncp_v + deg_v + 1,)
    cpw: np.ndarray      # (ncp_v, ncp_u, 4): x, y, z, w

    @property
    def ncp_u(self) -> int:
        return self.cpw.shape[1]

    @property
    def ncp_v(self) -> int:
        return self.cpw.shape[0]


# Cube faces: outward axis n and tangent axes (e1, e2) with e1 x e2 = n, so that
# the parametrisation (u, v) -> n + (2u-1) e1 + (2v-1) e2 is outward oriented.
CUBE_FACES = (
    ((1, 0, 0), (0, 1, 0), (0, 0, 1)),
    ((-1, 0, 0), (0, 0, 1), (0, 1, 0)),
    ((0, 1, 0), (0, 0, 1), (1, 0, 0)),
    ((0, -1, 0), (1, 0, 0), (0, 0, 1)),
    ((0, 0, 1), (1, 0, 0), (0, 1, 0)),
    ((0, 0, -1), (0, 1, 0), (1, 0, 0)),
)


def _cube_point(face: int, u: float, v: float) -> np.ndarray:
    n, e1, e2 = (np.asarray(a, dtype=np.float64) for a in CUBE_FACES[face])
    return n + (2.0 * u - 1.0) * e1 + (2.0 * v - 1.0) * e2


def _open_uniform_knots(deg: int, nspan: int) -> np.ndarray:
    inner = [j / nspan for j in range(1, nspan)]
    return np.array([0.0] * (deg + 1) + inner + [1.0] * (deg + 1), dtype=np.float64)


# ---------------------------------------------------------------------------
# Unit sphere: six rational-quadratic Bezier patches over the cube projection.
# Edges are exact great-circle arcs (corner weights 1, edge weight cos(theta/2));
# the single free control point (face centre, on the face axis) and its weight
# are fitted to minimise the maximal radial deviation.  The fitted NURBS *is* the
# scatterer for every comparison between the oracle and the library.
# ---------------------------------------------------------------------------

def _sphere_face_net(face: int, zc: float, wc: float) -> np.ndarray:
    corners = {}
    for i in (0, 2):
        for j in (0, 2):
            p = _cube_point(face, i / 2, j / 2)
            corners[(i, j)] = p / np.linalg.norm(p)
    net = np.zeros((3, 3, 4))
    for j in range(3):
        for i in range(3):
            if i != 1 and j != 1:
                net[j, i, :3] = corners[(i, j)]
                net[j, i, 3] = 1.0
            elif i == 1 and j == 1:
                net[j, i, :3] = zc * np.asarray(CUBE_FACES[face][0], dtype=np.float64)
                net[j, i, 3] = wc
            else:
                if i == 1:
                    a, b = corners[(0, j)], corners[(2, j)]
                else:
                    a, b = corners[(i, 0)], corners[(i, 2)]
                c = float(a @ b)
                net[j, i, :3] = (a + b) / (1.0 + c)   # tangent intersection
                net[j, i, 3] = math.sqrt((1.0 + c) / 2.0)  # cos(theta/2)
    return net


def _rational_quadratic_bezier_radius(net: np.ndarray, g: np.ndarray) -> np.ndarray:
    """|F(u,v)| of a 3x3 rational Bezier net on the grid g x g (fitting only)."""
    b = np.stack([(1 - g) ** 2, 2 * g * (1 - g), g ** 2], axis=1)  # (ng, 3)
    w = net[..., 3]
    hom = net[..., :3] * w[..., None]
    num = np.einsum("vj,ui,jik->vuk", b, b, hom)
    den = np.einsum("vj,ui,ji->vu", b, b, w)
    return np.linalg.norm(num / den[..., None], axis=-1)


@functools.lru_cache(maxsize=1)
def sphere_center_fit() -> tuple[float, float]:
    """(z*, w*) of the face-centre control point, minimax radial error fit."""
    from scipy.optimize import minimize

    g = np.linspace(0.0, 1.0, 41)

    def err(x):
        net = _sphere_face_net(4, x[0], x[1])
        return float(np.max(np.abs(_rational_quadratic_bezier_radius(net, g) - 1.0)))

    best = None
    for z0, w0 in ((2.3, 0.47), (2.0, 0.5), (2.6, 0.42)):
        r = minimize(err, x0=[z0, w0], method="Nelder-Mead",
                     options={"xatol": 1e-10, "fatol": 1e-13, "maxiter": 4000})
        if best is None or r.fun < best.fun:
            best = r
    return float(best.x[0]), float(best.x[1])


def sphere_patches(radius: float = 1.0) -> list[Patch]:
    zc, wc = sphere_center_fit()
    knots = _open_uniform_knots(2, 1)
    out = []
    for f in range(6):
        net = _sphere_face_net(f, zc, wc)
        net[..., :3] *= radius
        out.append(Patch(2, 2, knots.copy(), knots.copy(), net))
    return out


# ---------------------------------------------------------------------------
# Torus (major radius R, minor radius r) as 4 x 4 rational biquadratic Bezier
# patches: each the tensor product of a quarter arc of the major circle (u)
# and one of the minor circle (v), which represents the torus exactly; u then
# v runs with the outward normal d_u F x d_v F.
# ---------------------------------------------------------------------------

def _quarter_arc(k: int):
    """Control points (unit circle) and weights of the k-th quarter arc."""
    a0, a1 = k * math.pi / 2, (k + 1) * math.pi / 2
    pts = np.array([[math.cos(a0), math.sin(a0)],
                    [math.cos(a0) + math.cos(a1), math.sin(a0) + math.sin(a1)],
                    [math.cos(a1), math.sin(a1)]])
    return pts, np.array([1.0, math.sqrt(0.5), 1.0])


def torus_patches(R: float = 2.0, r: float = 0.5) -> list[Patch]:
    knots = _open_uniform_knots(2, 1)
    out = []
    for j in range(4):            # minor circle (v)
        mp, mw = _quarter_arc(j)
        for i in range(4):        # major circle (u)
            Mp, Mw = _quarter_arc(i)
            net = np.zeros((3, 3, 4))
            for b in range(3):
                for a in range(3):
                    rad = R + r * mp[b, 0]
                    net[b, a, :3] = (rad * Mp[a, 0], rad * Mp[a, 1], r * mp[b, 1])
                    net[b, a, 3] = Mw[a] * mw[b]
            out.append(Patch(2, 2, knots.copy(), knots.copy(), net))
    return out


# ---------------------------------------------------------------------------
# Seeded smooth star-shaped scatterer r(s) = 1 + 0.1 * sum_{l<=4} c_lm Y_lm(s),
# c_lm ~ N(0,1) drawn in (l, m = -l..l) order.  Each cube face carries a
# degree-2 B-spline patch on 2^g uniform spans whose control points are the
# surface points at the Greville abscissae (Schoenberg's variation-diminishing
# approximation): boundary control rows of neighbouring faces coincide exactly,
# so the patches conform.
# ---------------------------------------------------------------------------

def _real_sph_harm(l: int, m: int, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Orthonormal real spherical harmonic (theta polar, phi azimuth)."""
    from scipy.special import sph_harm_y

    y = sph_harm_y(l, abs(m), theta, phi)
    if m == 0:
        return y.real
    if m > 0:
        return math.sqrt(2.0) * (-1) ** m * y.real
    return math.sqrt(2.0) * (-1) ** m * y.imag


def star_radius(seed: int, dirs: np.ndarray, lmax: int = 4, amp: float = 0.1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    coef = rng.standard_normal((lmax + 1) ** 2)
    d = dirs / np.linalg.norm(dirs, axis=-1, keepdims=True)
    theta = np.arccos(np.clip(d[..., 2], -1.0, 1.0))
    phi = np.arctan2(d[..., 1], d[..., 0])
    r = np.ones(d.shape[:-1])
    k = 0
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            r = r + amp * coef[k] * _real_sph_harm(l, m, theta, phi)
            k += 1
    return r


def star_patches(seed: int, g: int) -> list[Patch]:
    nspan = 2 ** g
    deg = 2
    knots = _open_uniform_knots(deg, nspan)
    ncp = nspan + deg
    grev = np.array([(knots[i + 1] + knots[i + 2]) / 2.0 for i in range(ncp)])
    out = []
    for f in range(6):
        pts = np.array([[_cube_point(f, grev[i], grev[j]) for i in range(ncp)]
                        for j in range(ncp)])  # (v, u, 3)
        s = pts / np.linalg.norm(pts, axis=-1, keepdims=True)
        r = star_radius(seed, s)
        net = np.zeros((ncp, ncp, 4))
        net[..., :3] = s * r[..., None]
        net[..., 3] = 1.0
        out.append(Patch(deg, deg, knots.copy(), knots.copy(), net))
    return out


def star_geometry_level(m: int) -> int:
    """Geometry span exponent g = min(max(m - 3, 0), 4) of the level-m star.

    The geometry knots nest in the mesh, and every cluster of up to 8 x 8
    elements (leaf depth <= 3) lies inside one geometry span.  The degree-2
    mapping is only C^1 across its knot lines, so its surface measure and
    normal have kinks there; a kernel interpolated on a cluster that straddles
    one converges only algebraically in the interpolation degree, whereas
    inside one polynomial piece the pulled-back kernel is analytic and the
    Chebyshev error decays geometrically.  (Sec. 3.2 takes the patch mappings
    to be smooth; Sec. 4.4 interpolates the kernel pulled back to them.)"""
    return min(max(m - 3, 0), 4)


# ---------------------------------------------------------------------------
# Directions and vectors
# ---------------------------------------------------------------------------

def fibonacci_directions(n: int) -> np.ndarray:
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def random_directions(seed: int, n: int) -> np.ndarray:
    v = np.random.default_rng(seed).standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def random_complex(seed: int, shape) -> np.ndarray:
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im).astype(np.complex128)


# ---------------------------------------------------------------------------
# Named workloads (sizes of the paper-style scattering configurations)
# ---------------------------------------------------------------------------

WORKLOADS = {
    "sphere_m2_p1": dict(geometry="sphere", m=2, p=1, kappa=1.0, bc="soft",
                          ndir=1, nobs=64),
    "sphere_m5_p2_k8": dict(geometry="sphere", m=5, p=2, kappa=8.0, bc="soft",
                             q=6, eta_adm=1.6, ndir=1, tol=1e-8),
    "star_m6_p2_k16": dict(geometry="star", seed=0, m=6, p=2, kappa=16.0, bc="soft",
                            q=8, eta_adm=1.6, ndir=64, tol=1e-8),
    "star_m7_p2_k32_hard": dict(geometry="star", seed=0, m=7, p=2, kappa=32.0,
                                 bc="hard", q=8, eta_adm=1.6, ndir=16, tol=1e-8),
}


def geometry_for(w: dict) -> list[Patch]:
    if w["geometry"] == "sphere":
        return sphere_patches()
    return star_patches(w.get("seed", 0), star_geometry_level(w["m"]))


# ---------------------------------------------------------------------------
# Scattering request stream: Poisson arrivals, each request a seeded star-shaped
# scatterer with its own level, wavenumber, incidence directions and boundary
# condition.
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    arrival: float          # seconds after the stream starts
    seed: int               # star scatterer seed
    m: int
    kappa: float
    bc: str                 # "soft" | "hard"
    dirs: np.ndarray        # (ndir, 3) unit incident directions


def request_stream(n: int, rate: float, seed: int = 3, m_values=(3, 4, 5, 6), kappa_range=(1.0, 32.0),
                   max_dirs: int = 16, catalog: int = 0) -> list[Request]:
    """Poisson arrivals at `rate`; each request a seeded star, level, wavenumber,
    boundary condition and 1..max_dirs incident directions.  With catalog > 0
    the (star, level, wavenumber, boundary condition) of each request is drawn
    from a seeded catalog of that many scattering problems, so that requests
    share operators (new directions on a known problem); the directions stay
    the request's own."""
    rng = np.random.default_rng(seed)
    problems = []
    if catalog > 0:
        crng = np.random.default_rng(seed + 1)
        for _ in range(catalog):
            problems.append((int(crng.integers(0, 10 ** 6 + 1)), int(crng.choice(m_values)),
                             float(crng.uniform(*kappa_range)), "soft" if crng.integers(0, 2) == 0 else "hard"))
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        if problems:
            rseed, m, kappa, bc = problems[int(rng.integers(0, len(problems)))]
            ndir = int(rng.integers(1, max_dirs + 1))
            out.append(Request(i, t, rseed, m, kappa, bc, random_directions(int(rng.integers(0, 2 ** 31)), ndir)))
            continue
        rseed = int(rng.integers(0, 10 ** 6 + 1))
        m = int(rng.choice(m_values))
        kappa = float(rng.uniform(*kappa_range))
        ndir = int(rng.integers(1, max_dirs + 1))
        bc = "soft" if rng.integers(0, 2) == 0 else "hard"
        out.append(Request(i, t, rseed, m, kappa, bc, random_directions(rseed, ndir)))
    return out
