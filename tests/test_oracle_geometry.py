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
