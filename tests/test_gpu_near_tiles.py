"""Near product of the inner matvecs of bf16 operators (fp32 tiles of rows over
a common column list, matrix cores) against the fp64 near field.

Bound: both sides sum the same entries of a row; the tile path rounds values
and columns to fp32 (unit roundoff u = 2^-24) and forms products and sums in
fp32, so each row differs from the fp64 product by at most
gamma_{n+2} * sum_j |v_ij| |x_j| with gamma_n = n u / (1 - n u) and n the row
length (the merged rows' zero entries add exact zeros).
"""
import functools
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
U32 = 2.0 ** -24


@functools.lru_cache(maxsize=None)
def B():
    from paper_2306_11324_amd import binding
    return binding


@functools.lru_cache(maxsize=None)
def ctx():
    return B().Context(0)


def bf16_operator(m, kappa, q, d, bc, eta=1.6):
    from paper_2306_11324_amd import inputs as I
    b = B()
    print(f"case: sphere m={m} p=2 kappa={kappa} q={q} leaf_depth={d} bc={bc} bf16", flush=True)
    geo = b.Geometry(ctx(), I.sphere_patches(), m, 2)
    op = b.Operator(ctx(), geo, kappa=kappa, q=q, eta_adm=eta, leaf_depth=d, precision=b.MIX_BF16,
                    bc=b.SOFT if bc == "soft" else b.HARD)
    return geo, op


def apply(op, X, parts):
    xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    yd = torch.zeros_like(xd)
    op.h2_matvec(xd, yd, nrhs=X.shape[0], parts=parts)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def row_bound(op, X):
    """gamma_{n+2} * sum_j |v_ij| |x_j| per row and column, from the fp64 CSR."""
    import scipy.sparse as sp
    rp, col, val = op.near_csr()
    n = len(rp) - 1
    A = sp.csr_matrix((np.abs(val), col, rp), shape=(n, n))
    lens = np.diff(rp).astype(np.float64) + 2
    gamma = lens * U32 / (1 - lens * U32)
    return (gamma[None, :] * (A @ np.abs(X).T).T), A


@pytest.mark.parametrize("bc", ["soft", "hard"])
def test_small_tiles_match_oracle_near_product(bc):
    """Level-3 sphere, leaf depth 1: the fp32 tile product against the oracle's
    near product (fp64 element blocks) within the rounding bound plus the
    quadrature tolerance of the fp64 near field (1e-8 of max |y|)."""
    b = B()
    g = dict(np.load(os.path.join(GOLD, ("sphere_m3_p2_k2_q4" if bc == "soft" else "sphere_m3_p2_k2_q4_hard")
                                  + ".npz")))
    geo, op = bf16_operator(3, 2.0, 4, 1, bc)
    X = g["x"][None, :]
    y = apply(op, X, b.PART_NEAR | b.MV_LOWPREC)[0]
    bound, _ = row_bound(op, X)
    err = np.abs(y - g["y_near"])
    scale = np.abs(g["y_near"]).max()
    print(f"{bc}: max err {err.max():.2e}, max bound {bound.max():.2e}, max |y| {scale:.2e}", flush=True)
    assert np.all(err <= bound[0] + 1e-8 * scale)
    assert err.max() < 1e-5 * scale


@pytest.mark.parametrize("bc,m,d", [("soft", 5, 2), ("hard", 4, 1)])
def test_tiles_at_size_within_fp32_bound(bc, m, d):
    """The bench workload's sphere (m = 5, kappa = 8, q = 6, leaf depth 2) and a
    level-4 sound-hard operator: 16 and 20 columns of the tile product against
    the fp64 near product of the same operator, entry by entry within the
    rounding bound; the far part adds the same fp64 values either way."""
    from paper_2306_11324_amd import inputs as I
    b = B()
    geo, op = bf16_operator(m, 8.0, 6, d, bc)
    for ncol in (16, 20):
        X = I.random_complex(31 + ncol, (ncol, op.n))
        y_lo = apply(op, X, b.PART_NEAR | b.MV_LOWPREC)
        y64 = apply(op, X, b.PART_NEAR)
        bound, A = row_bound(op, X)
        err = np.abs(y_lo - y64)
        print(f"{bc} m={m} ncol={ncol}: max err {err.max():.2e}, max err / bound "
              f"{(err / np.maximum(bound, 1e-300)).max():.3f}, rel {err.max() / np.abs(y64).max():.2e}", flush=True)
        assert np.all(err <= bound)
        # with the far part: same far values, added in fp64 after the near sum
        z_lo = apply(op, X, b.PART_ALL | b.MV_LOWPREC)
        z_far = apply(op, X, b.PART_FAR | b.MV_LOWPREC)
        assert np.abs(z_lo - (y_lo + z_far)).max() <= 1e-12 * np.abs(z_lo).max()
