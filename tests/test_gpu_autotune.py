"""Autotuner over leaf depth, stored / on-the-fly couplings and tiles /
recompressed factors: every candidate keeps the accuracy against the dense
oracle rows (same admissibility and q), the choice is the cheapest measured
candidate (with require_far, the cheapest with admissible blocks), and the
cache round-trips through its JSON file and is what the server's operator
arguments use."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_tuned_shape_is_cheapest_and_accurate(tmp_path):
    from paper_2306_11324_amd import autotune as T
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    g = dict(np.load(os.path.join(GOLD, "sphere_m5_p2_k8_rows.npz")))
    print("case: sphere m=5 p=2 kappa=8 q=6 fp64, one column, leaf depths 1-3, stored / on the fly / "
          "recompressed at 1e-8", flush=True)
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.sphere_patches(), 5, 2)
    cache = T.TuneCache(str(tmp_path / "tune.json"))
    best, measured = T.tune(ctx, geo, 5, 2, 1, 8.0, q=6, leaf_depths=(1, 2, 3), recompress_tols=(0.0, 1e-8),
                            cache=cache, reps=3)
    for c in measured:
        print(f"  d={c.leaf_depth} otf={c.far_on_the_fly} tol={c.recompress_tol:g}: matvec {c.matvec_ms:.3f} ms, "
              f"assembly {c.assembly_ms:.0f} ms, {c.device_bytes / 1e9:.2f} GB, {c.far_pairs} far pairs", flush=True)
    assert len(measured) >= 9 and {c.recompress_tol for c in measured} == {0.0, 1e-8}
    assert all(c.far_pairs > 0 for c in measured)
    cost = [c.assembly_ms + 200 * c.matvec_ms for c in measured]
    assert best.assembly_ms + 200 * best.matvec_ms == min(cost)
    # every candidate is as accurate as the default against the oracle rows
    x = torch.from_numpy(g["x"]).cuda()
    for c in measured:
        op = B.Operator(ctx, geo, kappa=8.0, q=6, leaf_depth=c.leaf_depth, far_on_the_fly=c.far_on_the_fly,
                        recompress_tol=c.recompress_tol)
        y = torch.zeros_like(x)
        op.h2_matvec(x, y)
        torch.cuda.synchronize()
        yr = y.cpu().numpy()[g["rows"]]
        e = float(np.max(np.abs(yr - g["y"]) / (g["rownorm1"] * np.abs(g["x"]).max())))
        assert e < 1e-6, (c, e)
        del op
    # the cache round-trips and answers without measuring
    again = T.TuneCache(str(tmp_path / "tune.json"))
    best2, measured2 = T.tune(ctx, geo, 5, 2, 1, 8.0, q=6, cache=again)
    assert measured2 == [] and best2 == best
    # the server's operator arguments take the cached shape for the request's class
    from paper_2306_11324_amd import serving as S
    req = I.Request(rid=0, arrival=0.0, seed=0, m=5, kappa=8.0, bc="soft", dirs=np.array([[0.0, 0.0, 1.0]]))
    srv = S.Server.__new__(S.Server)
    srv.cfg = S.ServeConfig(p=2, q=6, precision=B.FP64, tune_cache=again)
    args = srv._op_args(req)
    assert args["leaf_depth"] == best.leaf_depth and args["far_on_the_fly"] == best.far_on_the_fly
    assert args["recompress_tol"] == best.recompress_tol


def test_require_far_skips_the_dense_shape():
    """Leaf depth 4 on the level-5 sphere leaves no admissible block (the whole
    operator is near field): with require_far it is measured but not chosen."""
    from paper_2306_11324_amd import autotune as T
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    print("case: sphere m=5 p=2 kappa=8 q=6 fp64, one column, leaf depths 3 and 4, require_far", flush=True)
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.sphere_patches(), 5, 2)
    best, measured = T.tune(ctx, geo, 5, 2, 1, 8.0, q=6, leaf_depths=(3, 4), on_the_fly=(False,), reps=3,
                            require_far=True)
    assert {c.leaf_depth: c.far_pairs == 0 for c in measured} == {3: False, 4: True}
    assert best.leaf_depth == 3 and best.far_pairs > 0


@pytest.mark.parametrize("bc", ["soft", "hard"])
def test_tile_shapes_change_no_result_and_tuner_keeps_the_fastest(bc):
    """Every coupling / near column-tile shape of a 64-column fp64 block gives
    bitwise the automatic shape's result; the tuner leaves its fastest shape
    set; shapes other than 0, 1, 2, 4 are rejected."""
    from paper_2306_11324_amd import autotune as T
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    print(f"case: sphere m=3 p=2 kappa=2 q=4 leaf depth 1 {bc} fp64, 64 columns, tile shapes", flush=True)
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.sphere_patches(), 3, 2)
    op = B.Operator(ctx, geo, kappa=2.0, q=4, leaf_depth=1, bc=B.SOFT if bc == "soft" else B.HARD)
    X = torch.from_numpy(I.random_complex(64, (64, op.n))).cuda()

    def apply():
        y = torch.zeros_like(X)
        op.h2_matvec(X, y, nrhs=64)
        torch.cuda.synchronize()
        return y.cpu().numpy()

    ref = apply()
    for cc in (1, 2, 4):
        for nc in (1, 2, 4):
            op.set_tile_shape(cc, nc)
            assert np.array_equal(apply(), ref), (cc, nc)
    best, measured = T.tune_tile_shape(op, 64, reps=3)
    assert len(measured) == 9 and best == min(measured, key=lambda t: t[2])
    assert np.array_equal(apply(), ref)
    with pytest.raises(B.IgbError):
        op.set_tile_shape(3, 0)
