"""The allocation-free matvec (h2_matvec_noalloc) against h2_matvec.

Both run the same kernels in the same order; only the work buffers differ
(the operator's own against the library's per-GPU scratch array), so the
results agree bitwise.  Two calls in a row, the second with a smaller input
(fewer columns, a smaller operator), so the second runs on what the first left
in the scratch.  Neither call allocates: the context's and the operator's byte
counts do not move.  Too many columns for the scratch are rejected with an
error, and so is a host-array product.
"""
import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def B():
    from paper_2306_11324_amd import binding
    return binding


def build(ctx, m, bc, prec, kappa, q, d):
    from paper_2306_11324_amd import inputs as I
    b = B()
    print(f"case: sphere m={m} p=2 kappa={kappa} q={q} leaf_depth={d} bc={bc} precision={prec}", flush=True)
    geo = b.Geometry(ctx, I.sphere_patches(), m, 2)
    op = b.Operator(ctx, geo, kappa=kappa, q=q, leaf_depth=d, bc=b.SOFT if bc == "soft" else b.HARD,
                    precision={"fp64": b.FP64, "bf16": b.MIX_BF16}[prec])
    return geo, op


def both(ctx, op, X, parts):
    xd = torch.from_numpy(X).cuda()
    y_ref = torch.zeros_like(xd)
    op.h2_matvec(xd, y_ref, nrhs=X.shape[0], parts=parts)
    torch.cuda.synchronize()
    used, held = ctx.used_bytes(), op.held_bytes()
    y_na = torch.full_like(xd, float("nan"))
    op.h2_matvec_noalloc(xd, y_na, nrhs=X.shape[0], parts=parts)
    torch.cuda.synchronize()
    assert ctx.used_bytes() == used and op.held_bytes() == held
    return y_ref.cpu().numpy(), y_na.cpu().numpy()


def test_noalloc_matvec_equals_h2_matvec_on_two_calls():
    from paper_2306_11324_amd import inputs as I
    b = B()
    ctx = b.Context(0)
    # first call: 16 fp64 columns (matrix-core coupling) on the level-4 sphere
    geo1, big = build(ctx, 4, "soft", "fp64", 4.0, 5, 2)
    X1 = I.random_complex(31, (16, big.n))
    ref, got = both(ctx, big, X1, b.PART_ALL)
    assert np.array_equal(ref, got)
    # second call, smaller: 3 bf16 columns of a level-3 hard operator, reduced precision
    geo2, small = build(ctx, 3, "hard", "bf16", 2.0, 4, 1)
    X2 = I.random_complex(32, (3, small.n))
    ref, got = both(ctx, small, X2, b.PART_ALL | b.MV_LOWPREC)
    assert np.array_equal(ref, got)
    # and the far part alone of one fp64 column of the first operator
    ref, got = both(ctx, big, X1[:1].copy(), b.PART_FAR)
    assert np.array_equal(ref, got)


def test_noalloc_rejects_what_it_cannot_serve():
    from paper_2306_11324_amd import inputs as I
    b = B()
    ctx = b.Context(0)
    geo, op = build(ctx, 3, "soft", "fp64", 2.0, 4, 1)
    used = ctx.used_bytes()
    n = 20000    # columns whose work buffers exceed the scratch
    x = torch.zeros((n, op.n), dtype=torch.complex128, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(b.IgbError) as e:
        op.h2_matvec_noalloc(x, y, nrhs=n)
    assert e.value.status == -1 and "scratch" in str(e.value)
    X = I.random_complex(1, (1, op.n))
    with pytest.raises(b.IgbError):
        b._check("h2_matvec_noalloc", b._lib.h2_matvec_noalloc(
            op.h, b.C.c_void_p(X.ctypes.data), b.C.c_void_p(X.ctypes.data + 8), 1, b.PART_ALL | b.MV_HOST, None))
    assert ctx.used_bytes() == used
