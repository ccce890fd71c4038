"""The torus of Sec. 5.2 (major radius 2, minor radius 0.5, 16 exact rational
biquadratic patches), kappa = 2.5, plane wave along x, scattered field at 100
points on the radius-5 sphere.

  * against the dense fp64 oracle (tests/golden/torus_k2p5_potential.npz):
    solution coefficients and scattered field, soft p = 1 on level 2 and hard
    p = 2 on level 1, with the default quadrature orders (which follow the
    3-5 : 1 aspect ratio of the torus elements and kappa times their size) and
    with three more points per direction;
  * the convergence rates the paper reports for the CFIE (l-infinity error of
    the scattered field O(h^{2p+2}) sound-soft, O(h^{2p+1}) sound-hard) on
    levels 2..4 against the level-5, degree-3 solution of the same boundary
    condition.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
D = np.array([[1.0, 0.0, 0.0]])


def _solve(ctx, bc, p, m, q=8, leaf_depth=3, quad_extra=2):
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    geo = B.Geometry(ctx, I.torus_patches(2.0, 0.5), m, p)
    op = B.Operator(ctx, geo, kappa=2.5, bc=B.SOFT if bc == "soft" else B.HARD, q=q, eta_adm=1.6,
                    leaf_depth=leaf_depth, quad_extra=quad_extra)
    c = torch.zeros((1, op.n), dtype=torch.complex128, device="cuda")
    info, st = op.cfie_solve(D, c, tol=1e-12, restart=50, maxit=3000)
    assert st == 0 and info.converged == 1
    pts = 5.0 * I.fibonacci_directions(100)
    u = torch.zeros((1, len(pts)), dtype=torch.complex128, device="cuda")
    op.potential(c, pts, u)
    torch.cuda.synchronize()
    return c.cpu().numpy()[0], u.cpu().numpy()[0]


@pytest.mark.parametrize("quad_extra", [0, 3])
@pytest.mark.parametrize("bc,p,m", [("soft", 1, 2), ("hard", 2, 1)])
def test_torus_against_dense_oracle(bc, p, m, quad_extra):
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    g = dict(np.load(os.path.join(GOLD, "torus_k2p5_potential.npz")))
    assert np.array_equal(g["pts"], 5.0 * I.fibonacci_directions(100))
    print(f"case: torus m={m} {bc} p={p} kappa=2.5 q=8 leaf depth 1 quad_extra {quad_extra}", flush=True)
    ctx = B.Context(0)
    c, u = _solve(ctx, bc, p, m, leaf_depth=1, quad_extra=quad_extra)
    ec = np.abs(c - g[f"{bc}_t"]).max() / np.abs(g[f"{bc}_t"]).max()
    eu = np.abs(u - g[f"{bc}_pot"]).max() / np.abs(g[f"{bc}_pot"]).max()
    print(f"coefficients {ec:.2e}, scattered field {eu:.2e} (relative to max)", flush=True)
    assert ec < 1e-6 and eu < 3e-7


@pytest.mark.parametrize("bc", ["soft", "hard"])
def test_torus_convergence_orders(bc):
    from paper_2306_11324_amd import binding as B
    ctx = B.Context(0)
    _, ref = _solve(ctx, bc, 3, 5)
    for p in (1, 2):
        err = [np.abs(_solve(ctx, bc, p, m)[1] - ref).max() for m in (2, 3, 4)]
        eoc = np.log2(np.array(err[:-1]) / np.array(err[1:]))
        want = 2 * p + 2 if bc == "soft" else 2 * p + 1
        print(f"{bc} p={p}: errors {['%.2e' % e for e in err]}, orders {np.round(eoc, 2)}, expected {want}",
              flush=True)
        assert eoc[-1] > want - 0.5
