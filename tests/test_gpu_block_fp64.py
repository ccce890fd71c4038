"""fp64 blocks on the matrix cores against the oracle (Sec. 4.4 coupling,
many incident directions as one block product).

An fp64 operator with stored couplings applies the coupling of blocks of 16 or
more columns with v_mfma_f64_16x16x4 (soft: m2l_mfma_soft, hard: m2l_mfma with
both G and H tiles); smaller blocks run the vector kernels.  The two paths sum
the same products in different orders, so:

* every column of a 16- or 20-column block (one full 16-column tile and a
  ragged tile of 4) matches O2's step-by-step far product (stored in
  tests/golden/sphere_m3_p2_k2_q4_block.npz, one column at a time) to 1e-11
  relative to max |y|, as the single-column path does;
* a column computed in a block of >= 16 equals the same column in any other
  block of >= 16 bitwise, and differs from the column computed alone by
  rounding only: at most 1e-12 relative to max |y| (the sums run over
  ~5,000 tiles of 25 x 25 products, so fp64 reordering moves them by ~1e-15);
* lockstep solves of 16 directions on the level-2 spheres reproduce the
  oracle's dense LU solution and far field of the one direction it stores;
* the near product of blocks of >= 16 columns runs on the fp64 matrix cores
  over tiles of up to 16 rows with a common column list: it matches O1's near
  product and, entry by entry, the one-column CSR product within the fp64
  rounding bound of the two summation orders;
* sound-hard operators without stored fp64 couplings (far_on_the_fly, fp64 or
  with a bf16 copy) evaluate G and H into LDS slab by slab and run blocks of
  >= 16 columns on the fp64 matrix cores (m2l_otf_mfma_hard): the same
  oracle, stored-tile, alone-vs-block and bitwise-between-blocks checks, at
  q = 4 (two waves, a ragged last slab) and q = 8 (six waves).
"""
import functools
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
BCS = pytest.mark.parametrize("bc", ["soft", "hard"])


def gold(name):
    return dict(np.load(os.path.join(GOLD, name + ".npz")))


@functools.lru_cache(maxsize=None)
def B():
    from paper_2306_11324_amd import binding
    return binding


@functools.lru_cache(maxsize=None)
def ctx():
    return B().Context(0)


@functools.lru_cache(maxsize=None)
def operator(m, p, kappa, q, d, bc):
    from paper_2306_11324_amd import inputs as I
    print(f"case: sphere m={m} p={p} kappa={kappa} q={q} leaf_depth={d} bc={bc} fp64 stored tiles", flush=True)
    geo = B().Geometry(ctx(), I.sphere_patches(), m, p)
    op = B().Operator(ctx(), geo, kappa=kappa, q=q, leaf_depth=d, bc=B().SOFT if bc == "soft" else B().HARD)
    return geo, op


def apply_block(op, X, parts):
    xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    yd = torch.zeros_like(xd)
    op.h2_matvec(xd, yd, nrhs=X.shape[0], parts=parts)
    torch.cuda.synchronize()
    return yd.cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@BCS
@pytest.mark.parametrize("ncol", [16, 20])
def test_fp64_matrix_core_block_matches_oracle(bc, ncol):
    g = gold("sphere_m3_p2_k2_q4_block")
    X, Yref = g[f"{bc}_X"][:ncol], g[f"{bc}_Y_far"][:ncol]
    geo, op = operator(3, 2, 2.0, 4, 1, bc)
    assert op.n == X.shape[1]
    Y = apply_block(op, X, B().PART_FAR)
    errs = [rel(Y[c], Yref[c]) for c in range(ncol)]
    alone = [rel(apply_block(op, X[c:c + 1], B().PART_FAR)[0], Y[c]) for c in range(ncol)]
    print(f"{bc} {ncol} columns: max rel err vs oracle {max(errs):.2e}; block vs alone {max(alone):.2e}", flush=True)
    assert max(errs) < 1e-11, errs
    assert max(alone) < 1e-12, alone
    assert max(alone) > 0, "the block did not take the matrix-core path"


@BCS
def test_blocks_of_16_or_more_agree_bitwise(bc):
    """Columns 0..15 of a 20-column block equal the 16-column block, and the
    last 4 equal a 17-column block whose last column is each of them."""
    g = gold("sphere_m3_p2_k2_q4_block")
    X = g[f"{bc}_X"]
    geo, op = operator(3, 2, 2.0, 4, 1, bc)
    Y20 = apply_block(op, X, B().PART_ALL)
    Y16 = apply_block(op, X[:16], B().PART_ALL)
    assert np.array_equal(Y20[:16], Y16)
    for c in range(16, 20):
        Y17 = apply_block(op, np.concatenate([X[:16], X[c:c + 1]]), B().PART_ALL)
        assert np.array_equal(Y17[16], Y20[c]), c


LEVEL2 = {"soft": ("sphere_m2_p1_k1", 1), "hard": ("sphere_m2_p2_k1_hard", 2)}


@BCS
def test_sixteen_direction_fp64_solve_matches_oracle_lu(bc):
    """16 directions in lockstep (matrix-core coupling at every Arnoldi step):
    the direction the oracle stores (d = (0, 0, 1), placed in column 5) matches
    its dense LU solution and far field (H^2 error at q = 8 ~1e-8), and Mie."""
    from paper_2306_11324_amd import inputs as I
    name, p = LEVEL2[bc]
    g = gold(name)
    geo, op = operator(2, p, 1.0, 8, 0, bc)
    dirs = I.random_directions(11, 16)
    dirs[5] = g["d"]
    T = torch.zeros((16, op.n), dtype=torch.complex128, device="cuda")
    info, st = op.cfie_solve(dirs, T, tol=1e-12, restart=30, maxit=600)
    assert st == 0 and info.converged == 16 and info.relres_true < 1e-11, (info.iters, info.relres_true)
    u = torch.zeros(len(g["obs"]), dtype=torch.complex128, device="cuda")
    op.farfield(T[5], g["obs"], u)
    torch.cuda.synchronize()
    u = u.cpu().numpy()
    e_t, e_u, e_mie = rel(T[5].cpu().numpy(), g["t"]), rel(u, g["uinf"]), rel(u, g["mie"])
    print(f"{bc}: 16-direction fp64 block, column 5 vs LU {e_t:.2e}, far field vs LU {e_u:.2e}, vs Mie "
          f"{e_mie:.2e}", flush=True)
    assert e_t < 1e-6 and e_u < 1e-6 and e_mie < 1e-3


U64 = 2.0 ** -53


def near_bound(op, X, factor=2.0):
    """factor * gamma_{n+2} * sum_j |v_ij| |x_j| per row and column (fp64
    rounding of a length-n complex inner product, each of the two summation
    orders), from the operator's CSR."""
    import scipy.sparse as sp
    rp, col, val = op.near_csr()
    n = len(rp) - 1
    A = sp.csr_matrix((np.abs(val), col, rp), shape=(n, n))
    lens = np.diff(rp).astype(np.float64) + 2
    gamma = lens * U64 / (1 - lens * U64)
    return factor * gamma[None, :] * (A @ np.abs(X).T).T


@BCS
@pytest.mark.parametrize("ncol", [16, 20])
def test_fp64_tile_near_product_matches_oracle(bc, ncol):
    """Blocks of >= 16 columns take the near product on the fp64 matrix cores
    (tiles of up to 16 rows over a common column list): column 0 (the oracle's
    vector) against O1's near product (quadrature tolerance 1e-8), and every
    column against the one-column CSR product within the fp64 rounding bound
    of the two summation orders."""
    g = gold(SMALL[bc])
    gb = gold("sphere_m3_p2_k2_q4_block")
    geo, op = operator(3, 2, 2.0, 4, 1, bc)
    X = np.concatenate([g["x"][None, :], gb[f"{bc}_X"][1:ncol]])
    Y = apply_block(op, X, B().PART_NEAR)
    e_or = rel(Y[0], g["y_near"])
    Y1 = np.stack([apply_block(op, X[c:c + 1], B().PART_NEAR)[0] for c in range(ncol)])
    bound = near_bound(op, X)
    err = np.abs(Y - Y1)
    print(f"{bc} {ncol}: near vs oracle {e_or:.2e}; tile vs CSR max err / bound "
          f"{(err / np.maximum(bound, 1e-300)).max():.3f}, rel {err.max() / np.abs(Y1).max():.2e}", flush=True)
    assert e_or < 1e-8
    assert np.all(err <= bound)
    assert err.max() > 0, "the block did not take the tile path"


SMALL = {"soft": "sphere_m3_p2_k2_q4", "hard": "sphere_m3_p2_k2_q4_hard"}


@pytest.mark.parametrize("bc,m,d", [("soft", 5, 2), ("hard", 4, 1)])
def test_fp64_tile_near_product_at_size(bc, m, d):
    """The bench workload's sphere (m = 5, kappa = 8, q = 6, leaf depth 2) and
    a level-4 hard operator: 16 and 20 columns of the fp64 tile near product
    against the one-column CSR product, entry by entry within the bound; with
    the far part added (PART_ALL) the block equals near + far."""
    from paper_2306_11324_amd import inputs as I
    geo, op = operator(m, 2, 8.0, 6, d, bc)
    for ncol in (16, 20):
        X = I.random_complex(41 + ncol, (ncol, op.n))
        Y = apply_block(op, X, B().PART_NEAR)
        Y1 = np.stack([apply_block(op, X[c:c + 1], B().PART_NEAR)[0] for c in range(ncol)])
        bound = near_bound(op, X)
        err = np.abs(Y - Y1)
        print(f"{bc} m={m} ncol={ncol}: max err / bound {(err / np.maximum(bound, 1e-300)).max():.3f}, rel "
              f"{err.max() / np.abs(Y1).max():.2e}", flush=True)
        assert np.all(err <= bound)
        Z = apply_block(op, X, B().PART_ALL)
        F = apply_block(op, X, B().PART_FAR)
        assert np.abs(Z - (Y + F)).max() <= 1e-12 * np.abs(Z).max()


@functools.lru_cache(maxsize=None)
def otf_operator(m, p, kappa, q, d, prec):
    from paper_2306_11324_amd import inputs as I
    print(f"case: sphere m={m} p={p} kappa={kappa} q={q} leaf_depth={d} hard {prec}, fp64 far on the fly", flush=True)
    geo = B().Geometry(ctx(), I.sphere_patches(), m, p)
    op = B().Operator(ctx(), geo, kappa=kappa, q=q, leaf_depth=d, bc=B().HARD, far_on_the_fly=True,
                      precision={"fp64": B().FP64, "bf16": B().MIX_BF16}[prec])
    return geo, op


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
@pytest.mark.parametrize("ncol", [16, 20])
def test_on_the_fly_hard_block_matches_oracle(ncol, prec):
    """The fp64 far product evaluated on the fly, blocks of 16 and 20 columns on
    the fp64 matrix cores: every column against O2 (1e-11), against the
    stored-tile operator's block (1e-12), against the column alone on the
    vector kernel (<= 1e-12, not bitwise), and columns 0..15 of the 20-column
    block equal the 16-column block."""
    g = gold("sphere_m3_p2_k2_q4_block")
    X, Yref = g["hard_X"][:ncol], g["hard_Y_far"][:ncol]
    geo, op = otf_operator(3, 2, 2.0, 4, 1, prec)
    geo_s, st = operator(3, 2, 2.0, 4, 1, "hard")
    Y = apply_block(op, X, B().PART_FAR)
    errs = [rel(Y[c], Yref[c]) for c in range(ncol)]
    e_st = rel(Y, apply_block(st, X, B().PART_FAR))
    alone = [rel(apply_block(op, X[c:c + 1], B().PART_FAR)[0], Y[c]) for c in range(ncol)]
    print(f"{prec} {ncol} columns: max rel err vs oracle {max(errs):.2e}; vs stored tiles {e_st:.2e}; "
          f"block vs alone {max(alone):.2e}", flush=True)
    assert max(errs) < 1e-11, errs
    assert e_st < 1e-12
    assert max(alone) < 1e-12, alone
    assert max(alone) > 0, "the block did not take the matrix-core path"
    if ncol == 20:
        assert np.array_equal(Y[:16], apply_block(op, X[:16], B().PART_FAR))


def test_on_the_fly_hard_block_q8():
    """q = 8 (81 nodes: six waves, slabs of 16 source nodes, the last one
    ragged) on the level-4 sphere: the on-the-fly block against the stored-tile
    block and against the columns alone."""
    from paper_2306_11324_amd import inputs as I
    geo, op = otf_operator(4, 2, 4.0, 8, 1, "fp64")
    geo_s, st = operator(4, 2, 4.0, 8, 1, "hard")
    X = I.random_complex(808, (16, op.n))
    Y = apply_block(op, X, B().PART_FAR)
    e_st = rel(Y, apply_block(st, X, B().PART_FAR))
    alone = max(rel(apply_block(op, X[c:c + 1], B().PART_FAR)[0], Y[c]) for c in (0, 7, 15))
    print(f"q=8: on the fly vs stored tiles {e_st:.2e}, block vs alone {alone:.2e}", flush=True)
    assert e_st < 1e-12 and 0 < alone < 1e-12
