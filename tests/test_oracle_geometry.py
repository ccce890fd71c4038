"""Pins of oracle.geometry / oracle.spaces: closed-form volume and area of the
sphere, outward orientation, conforming interfaces and the dimension formulas
of S^2 (Sec. 3.3) and S^0 (Euler's formula on the cube topology)."""
import numpy as np
import pytest

from oracle import quadrature as qd
from oracle.spaces import Discretization
from paper_2306_11324_amd import inputs


def _volume_area(patches, n=12):
    pts, w = qd.tensor2(n)
    disc = Discretization(patches, 0, 2)
    E = disc.nelem
    d = disc.eval_on_elements(np.arange(E), np.broadcast_to(pts, (E,) + pts.shape))
    wq = w * disc.h ** 2
    vol = np.sum(np.einsum("eqc,eqc->eq", d["X"], d["nt"]) * wq) / 3.0
    area = np.sum(d["a"] * wq)
    return vol, area, d


def test_sphere_volume_area_radius():
    vol, area, d = _volume_area(inputs.sphere_patches())
    r = np.linalg.norm(d["X"], axis=-1)
    rad_err = np.abs(r - 1).max()
    assert rad_err < 1e-4                      # fitted rational quadratic faces
    assert abs(vol - 4 * np.pi / 3) < 3 * rad_err * 4 * np.pi / 3
    assert abs(area - 4 * np.pi) < 3 * rad_err * 4 * np.pi
    # outward orientation: n~ . x > 0 everywhere
    assert np.all(np.einsum("eqc,eqc->eq", d["X"], d["nt"]) > 0)


def test_star_is_closed_and_outward():
    pts = inputs.star_patches(0, 2)
    vol, area, d = _volume_area(pts)
    assert vol > 0 and area > 0
    # closedness: divergence theorem for a constant field, int n~ = 0
    pts2, w = qd.tensor2(12)
    nt = d["nt"].reshape(-1, 3)
    tot = np.einsum("eqc,q->c", d["nt"], w) * (1 / 16)
    assert np.abs(tot).max() < 1e-10 * area


@pytest.mark.parametrize("m,p", [(1, 1), (2, 1), (2, 2), (3, 2), (2, 3)])
def test_dimension_formulas(m, p):
    disc = Discretization(inputs.sphere_patches(), p, m)
    k = 2 ** m + p
    assert disc.n2 == 6 * k * k
    assert disc.s0_map()[1] == 6 * (k - 2) ** 2 + 12 * (k - 2) + 8


def test_s0_dimension_on_star():
    disc = Discretization(inputs.star_patches(3, 2), 2, 3)
    k = 2 ** 3 + 2
    assert disc.s0_map()[1] == 6 * (k - 2) ** 2 + 12 * (k - 2) + 8


def test_torus_exact_volume_area_closed_outward():
    """16 rational biquadratic patches reproduce the torus (R = 2, r = 0.5)
    exactly: every point on (sqrt(x^2+y^2) - R)^2 + z^2 = r^2, volume
    2 pi^2 R r^2, area 4 pi^2 R r, normal along the minor-circle radius."""
    R, r = 2.0, 0.5
    vol, area, d = _volume_area(inputs.torus_patches(R, r), n=16)
    X = d["X"]
    rho = np.hypot(X[..., 0], X[..., 1])
    assert np.abs((rho - R) ** 2 + X[..., 2] ** 2 - r * r).max() < 1e-13
    assert abs(vol - 2 * np.pi ** 2 * R * r * r) < 1e-10
    assert abs(area - 4 * np.pi ** 2 * R * r) < 1e-10
    core = np.stack([R * X[..., 0] / rho, R * X[..., 1] / rho, 0 * rho], -1)
    nt = d["nt"] / np.linalg.norm(d["nt"], axis=-1, keepdims=True)
    assert np.abs(np.einsum("eqc,eqc->eq", X - core, nt) - r).max() < 1e-12


@pytest.mark.parametrize("m,p", [(0, 1), (1, 2), (2, 3)])
def test_dimensions_on_torus(m, p):
    """Genus one: the glued space is (4 (k - 1))^2-dimensional (every vertex,
    edge and face of the 4 x 4 periodic patch grid is shared)."""
    disc = Discretization(inputs.torus_patches(), p, m)
    k = 2 ** m + p
    assert disc.n2 == 16 * k * k
    assert disc.s0_map()[1] == 16 * (k - 1) ** 2
