"""Indirect single-layer formulations (u_s = -S t on S^2; soft V t = u_inc,
hard (K* - 1/2) t = d_n u_inc), the comparison solutions of Sec. 5.2:

  * level-2 sphere, p = 1, kappa = 1 against the dense oracle
    (tests/golden/sphere_m2_k1_single_layer.npz) and the Mie series;
  * the torus of Sec. 5.2 (kappa = 2.5, 100 points on |x| = 5): the CFIE and
    the single-layer scattered fields agree to the discretisation error;
  * the bf16 far field inside fp64 refinement solves the single-layer systems
    to the fp64 tolerance.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
BCS = pytest.mark.parametrize("bc", ["soft", "hard"])


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _solve(op, d, pts, tol=1e-12):
    c = torch.zeros((1, op.n), dtype=torch.complex128, device="cuda")
    info, st = op.cfie_solve(np.atleast_2d(d), c, tol=tol, restart=50, maxit=3000)
    assert st == 0 and info.converged == 1, (info.iters, info.relres_true)
    u = torch.zeros((1, len(pts)), dtype=torch.complex128, device="cuda")
    op.potential(c, pts, u)
    torch.cuda.synchronize()
    return c.cpu().numpy()[0], u.cpu().numpy()[0], info


@BCS
def test_single_layer_sphere_against_dense_oracle_and_mie(bc):
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    g = dict(np.load(os.path.join(GOLD, "sphere_m2_k1_single_layer.npz")))
    mie = dict(np.load(os.path.join(GOLD, "sphere_m2_k1_potential.npz")))[f"{bc}_mie"]
    print(f"case: sphere m=2 p=1 kappa=1 single layer {bc}, q=8 leaf depth 0", flush=True)
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.sphere_patches(), 2, 1)
    op = B.Operator(ctx, geo, kappa=1.0, bc=B.SOFT if bc == "soft" else B.HARD, q=8, leaf_depth=0,
                    formulation=B.SINGLE_LAYER)
    assert op.n == geo.n2 and op.info.far_pairs > 0
    c, u, info = _solve(op, g["d"], g["pts"])
    ec, eu, em = _rel(c, g[f"{bc}_t"]), _rel(u, g[f"{bc}_pot"]), _rel(u, mie)
    print(f"coefficients {ec:.2e}, field vs oracle {eu:.2e}, vs Mie {em:.2e}, iterations {info.iters}", flush=True)
    assert ec < 1e-6 and eu < 1e-7 and em < 1e-3


@BCS
def test_single_layer_and_cfie_agree_on_torus(bc):
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    print(f"case: torus m=4 p=2 kappa=2.5 {bc}: CFIE and single layer", flush=True)
    ctx = B.Context(0)
    pts = 5.0 * I.fibonacci_directions(100)
    geo = B.Geometry(ctx, I.torus_patches(), 4, 2)
    out = {}
    for f in (B.CFIE, B.SINGLE_LAYER):
        op = B.Operator(ctx, geo, kappa=2.5, bc=B.SOFT if bc == "soft" else B.HARD, q=8, leaf_depth=3,
                        quad_extra=1, formulation=f)
        out[f] = _solve(op, [1.0, 0.0, 0.0], pts)[1]
        del op
    e = _rel(out[B.SINGLE_LAYER], out[B.CFIE])
    print(f"single layer vs CFIE scattered field: {e:.2e}", flush=True)
    assert e < (2e-6 if bc == "soft" else 1e-5)


@BCS
def test_single_layer_bf16_refinement_matches_fp64(bc):
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    print(f"case: sphere m=4 p=2 kappa=4 single layer {bc}: bf16 couplings + fp64 refinement vs fp64", flush=True)
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.sphere_patches(), 4, 2)
    pts = 2.0 * I.fibonacci_directions(50)
    res = {}
    for prec in (B.FP64, B.MIX_BF16):
        op = B.Operator(ctx, geo, kappa=4.0, bc=B.SOFT if bc == "soft" else B.HARD, q=6, leaf_depth=2,
                        precision=prec, formulation=B.SINGLE_LAYER)
        res[prec] = _solve(op, [0.0, 0.6, 0.8], pts, tol=1e-10)
        del op
    e = _rel(res[B.MIX_BF16][1], res[B.FP64][1])
    print(f"bf16-refined vs fp64 field {e:.2e}; refinements {res[B.MIX_BF16][2].refinements}", flush=True)
    assert res[B.MIX_BF16][2].relres_true <= 1e-10 and e < 1e-8
