"""Scattered field through the H^2 structure (potential_h2: octree boxes of
the points; admissible clusters act through their interpolation nodes, summed
at the points or, for boxes with more points than (q+1)^3, on the box's
Chebyshev nodes; near leaves summed directly) against the direct summation
(potential), whose own parity with the oracle and Mie is tested elsewhere:

  * a seeded shell of 200,000 points (1.2 <= |x| <= 4) around the level-5
    sphere, kappa = 3, q = 8, soft and hard, one and three columns;
  * a planar grid (a degenerate box direction) and a cylinder grid around the
    torus, kappa = 2.5;
  * the level-2 sphere's 72 golden points against the Mie series;
  * the level-5 sphere with seeded coefficients at 160 points against the
    oracle's representation formulas (both evaluations, kappa = 3 and 8);
  * a grid of 125-point boxes beside the level-4 sphere at q = 3 (box nodes)
    and q = 4 (cluster nodes at the points).
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _both(op, c, pts, ndir):
    out = []
    for f in (op.potential, op.potential_h2):
        u = torch.zeros((ndir, len(pts)), dtype=torch.complex128, device="cuda")
        f(c, pts, u, ndir=ndir)
        torch.cuda.synchronize()
        out.append(u.cpu().numpy())
    return out


def _solve(op, dirs):
    c = torch.zeros((len(dirs), op.n), dtype=torch.complex128, device="cuda")
    info, st = op.cfie_solve(dirs, c, tol=1e-10, restart=30, maxit=2000)
    assert st == 0 and info.converged == len(dirs)
    return c


@pytest.mark.parametrize("bc", ["soft", "hard"])
def test_h2_potential_matches_direct_sum_on_a_shell(bc):
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    print(f"case: sphere m=5 p=2 kappa=3 q=8 leaf depth 2 {bc}, 200000 points in 1.2 <= r <= 4, 3 directions",
          flush=True)
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.sphere_patches(), 5, 2)
    op = B.Operator(ctx, geo, kappa=3.0, bc=B.SOFT if bc == "soft" else B.HARD, q=8, leaf_depth=2)
    dirs = I.random_directions(11, 3)
    c = _solve(op, dirs)
    rng = np.random.default_rng(2024)
    npt = 200000
    xh = rng.normal(size=(npt, 3))
    pts = xh / np.linalg.norm(xh, axis=1, keepdims=True) * rng.uniform(1.2, 4.0, size=(npt, 1))
    import time
    t0 = time.perf_counter()
    ud, uh = _both(op, c, pts, 3)
    e = float(np.abs(uh - ud).max() / np.abs(ud).max())
    print(f"H^2 vs direct: {e:.2e} ({time.perf_counter() - t0:.2f} s for both)", flush=True)
    assert e < 1e-5
    # one column alone gives the same values as inside the block
    u1 = torch.zeros((1, len(pts)), dtype=torch.complex128, device="cuda")
    op.potential_h2(c[1:2].contiguous(), pts, u1)
    torch.cuda.synchronize()
    assert np.array_equal(u1.cpu().numpy()[0], uh[1])


def test_h2_potential_planar_and_cylinder_grids_around_the_torus():
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    print("case: torus m=4 p=2 kappa=2.5 q=8 soft, 60x60 plane z=0.8 and 40x90 cylinder r=3.2", flush=True)
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.torus_patches(), 4, 2)
    op = B.Operator(ctx, geo, kappa=2.5, q=8, leaf_depth=3)
    c = _solve(op, np.array([[1.0, 0.0, 0.0]]))
    g = np.linspace(-4, 4, 60)
    plane = np.stack(np.meshgrid(g, g, [0.8], indexing="ij"), -1).reshape(-1, 3)
    th, z = np.meshgrid(np.linspace(0, 2 * np.pi, 90, endpoint=False), np.linspace(-2, 2, 40), indexing="ij")
    cyl = np.stack([3.2 * np.cos(th), 3.2 * np.sin(th), z], -1).reshape(-1, 3)
    for name, pts in (("plane", plane), ("cylinder", cyl)):
        ud, uh = _both(op, c, pts, 1)
        e = float(np.abs(uh - ud).max() / np.abs(ud).max())
        print(f"{name}: H^2 vs direct {e:.2e}", flush=True)
        assert e < 1e-5


def test_h2_potential_against_mie_on_level2_sphere():
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    G = dict(np.load(os.path.join(GOLD, "sphere_m2_k1_potential.npz")))
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.sphere_patches(), 2, 1)
    op = B.Operator(ctx, geo, kappa=1.0, q=8, leaf_depth=0)
    t = torch.from_numpy(G["soft_t"]).cuda().reshape(1, -1)
    ud, uh = _both(op, t, G["pts"], 1)
    e_dir = float(np.abs(uh - ud).max() / np.abs(ud).max())
    e_mie = float(np.abs(uh[0] - G["soft_mie"]).max() / np.abs(G["soft_mie"]).max())
    print(f"72 points: H^2 vs direct {e_dir:.2e}, vs Mie {e_mie:.2e}", flush=True)
    assert e_dir < 1e-8 and e_mie < 1e-3


@pytest.mark.parametrize("bc", ["soft", "hard"])
@pytest.mark.parametrize("kappa,q", [(3.0, 8), (8.0, 6)])
def test_potentials_match_oracle_at_size(bc, kappa, q):
    """The level-5 sphere (6144 elements) with seeded density coefficients:
    the direct summation and the H^2 evaluation against the oracle's
    representation formulas at 160 seeded points in 1.2 <= |x| <= 4
    (tests/golden/sphere_m5_p2_potential.npz), at kappa = 3 (q = 8) and at the
    bench workload's kappa = 8 (q = 6)."""
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    G = dict(np.load(os.path.join(GOLD, "sphere_m5_p2_potential.npz")))
    print(f"case: sphere m=5 p=2 {bc} kappa={kappa} q={q}, 160 points, seeded coefficients", flush=True)
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.sphere_patches(), 5, 2)
    op = B.Operator(ctx, geo, kappa=kappa, bc=B.SOFT if bc == "soft" else B.HARD, q=q, leaf_depth=2)
    c = torch.from_numpy(G[f"{bc}_c"]).cuda().reshape(1, -1)
    assert c.shape[1] == op.n
    ud, uh = _both(op, c, G["pts"], 1)
    ref = G[f"{bc}_k{int(kappa)}_pot"]
    e_dir = float(np.abs(ud[0] - ref).max() / np.abs(ref).max())
    e_h2 = float(np.abs(uh[0] - ref).max() / np.abs(ref).max())
    print(f"direct vs oracle {e_dir:.2e}, H^2 vs oracle {e_h2:.2e}", flush=True)
    assert e_dir < 1e-6 and e_h2 < 1e-5


@pytest.mark.parametrize("q", [3, 4])
def test_box_interpolation_and_cluster_nodes_on_a_grid(q):
    """A 20 x 20 x 20 grid in a unit cube beside the level-4 sphere splits into
    octree boxes of 5 x 5 x 5 = 125 points: at q = 3 a box holds more points
    than its (q+1)^3 = 64 nodes, so admissible clusters act through the box's
    nodes (two-sided interpolation); at q = 4 (125 nodes) they act on the
    points through the cluster's nodes alone.  Both against the direct sum."""
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    print(f"case: sphere m=4 p=2 kappa=1 q={q} leaf depth 1 soft, 8000 grid points in [2, 3] x [-0.5, 0.5]^2",
          flush=True)
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.sphere_patches(), 4, 2)
    op = B.Operator(ctx, geo, kappa=1.0, q=q, leaf_depth=1)
    c = _solve(op, np.array([[1.0, 0.0, 0.0]]))
    g = np.linspace(0.0, 1.0, 20)
    pts = np.stack(np.meshgrid(g + 2.0, g - 0.5, g - 0.5, indexing="ij"), -1).reshape(-1, 3)
    ud, uh = _both(op, c, pts, 1)
    e = float(np.abs(uh - ud).max() / np.abs(ud).max())
    print(f"H^2 vs direct {e:.2e}", flush=True)
    assert e < {3: 3e-4, 4: 3e-5}[q]
