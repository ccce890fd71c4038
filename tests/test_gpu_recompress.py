"""Recompressed coupling tiles (far_recompress_tol): every fp64 tile factored by
Householder QR with column pivoting, truncated where the trailing block's
Frobenius norm falls below tol times the tile's, the one-column products
streaming the factors.

  * the level-5 sphere workload (kappa = 8, q = 6, leaf depths 2 and 3): one-column matvec against
    the tiles (the truncation moves each tile by at most tol in Frobenius norm;
    the product by <= 200 tol relative to max |y|) and against the sampled
    oracle rows (tests/golden/sphere_m5_p2_k8_rows.npz): the error against the
    oracle stays that of the tiles (the interpolation error dominates); the
    factors hold fewer entries than the tiles (average rank < nq / 2);
  * the solve equals the one on the tiles; several columns still use the tiles.
"""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _apply(op, x):
    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    y = torch.zeros_like(xd)
    op.h2_matvec(xd, y, nrhs=x.shape[0] if x.ndim == 2 else 1)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("ld,tol", [(2, 1e-10), (2, 1e-8), (2, 1e-7), (3, 1e-8)])
def test_recompressed_tiles_match_tiles_and_oracle(ld, tol):
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    g = dict(np.load(os.path.join(GOLD, "sphere_m5_p2_k8_rows.npz")))
    print(f"case: sphere m=5 p=2 kappa=8 q=6 leaf depth {ld}, recompression tolerance {tol:g}", flush=True)
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.sphere_patches(), 5, 2)
    dense = B.Operator(ctx, geo, kappa=8.0, q=6, leaf_depth=ld)
    lr = B.Operator(ctx, geo, kappa=8.0, q=6, leaf_depth=ld, recompress_tol=tol)
    x = g["x"]
    yd, yl = _apply(dense, x), _apply(lr, x)
    e_dense = float(np.abs(yl - yd).max() / np.abs(yd).max())
    yr = yl[g["rows"]]
    e_or = float(np.max(np.abs(yr - g["y"]) / (g["rownorm1"] * np.abs(x).max())))
    print(f"one column: vs tiles {e_dense:.2e}, vs oracle rows {e_or:.2e} (operator-relative); "
          f"device bytes {lr.info.device_bytes / 1e9:.2f} GB vs {dense.info.device_bytes / 1e9:.2f} GB", flush=True)
    assert e_dense < 200 * tol and e_or < 1e-6
    yr_t = yd[g["rows"]]
    e_or_t = float(np.max(np.abs(yr_t - g["y"]) / (g["rownorm1"] * np.abs(x).max())))
    assert e_or < 1.01 * e_or_t + 1e-12, (e_or, e_or_t)
    avg_rank = lr.info.far_factor_entries / (2 * lr.info.nq * lr.info.far_pairs)
    print(f"average rank {avg_rank:.2f} of {lr.info.nq}", flush=True)
    assert 0 < avg_rank < lr.info.nq / 2
    # several columns use the tiles: bitwise equal to the dense operator
    X = I.random_complex(3, (3, dense.n))
    assert np.array_equal(_apply(lr, X), _apply(dense, X))
    d = np.array([[0.0, 0.0, 1.0]])
    sol = []
    for op in (dense, lr):
        c = torch.zeros((1, op.n), dtype=torch.complex128, device="cuda")
        info, st = op.cfie_solve(d, c, tol=1e-10, restart=30, maxit=2000)
        assert st == 0 and info.converged == 1
        sol.append(c.cpu().numpy())
    e_sol = float(np.abs(sol[1] - sol[0]).max() / np.abs(sol[0]).max())
    print(f"solution vs tiles {e_sol:.2e}", flush=True)
    assert e_sol < max(1e-8, 1e3 * tol)
