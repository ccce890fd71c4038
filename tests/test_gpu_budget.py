"""HBM budget and the solve size model on the device, and host-pointer matvecs.

* Every device allocation is charged to the context: after a multi-direction
  solve the context holds exactly its geometry's and operator's bytes, and the
  operator holds no more than the solve size model (igb_op_solve_bytes)
  predicts, nor much less.
* The solver's buffers belong to the operator: a second solve allocates
  nothing.
* A budget that holds the operator but not a 1024-direction solve rejects the
  solve with IGB_ERR_BUDGET before any work and allocates nothing; a
  one-direction solve still runs.
* h2_matvec on host arrays (IGB_MV_HOST) equals the device-array product
  bitwise.
"""
import functools

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
CASES = [("soft", "fp64"), ("hard", "bf16"), ("soft", "fp32")]


@functools.lru_cache(maxsize=None)
def B():
    from paper_2306_11324_amd import binding
    return binding


def geometry(ctx):
    from paper_2306_11324_amd import inputs as I
    return B().Geometry(ctx, I.sphere_patches(), 3, 2)


def operator(ctx, geo, bc, prec):
    b = B()
    return b.Operator(ctx, geo, kappa=2.0, q=4, leaf_depth=1, bc=b.SOFT if bc == "soft" else b.HARD,
                      precision={"fp64": b.FP64, "fp32": b.MIX_FP32, "bf16": b.MIX_BF16}[prec])


@pytest.mark.parametrize("bc,prec", CASES)
def test_solve_stays_within_the_size_model(bc, prec):
    from paper_2306_11324_amd import inputs as I
    print(f"case: sphere m=3 p=2 kappa=2 q=4 bc={bc} precision={prec}, 16 directions", flush=True)
    ctx = B().Context(0)
    geo = geometry(ctx)
    g_bytes = ctx.used_bytes()
    op = operator(ctx, geo, bc, prec)
    assert ctx.used_bytes() == g_bytes + op.held_bytes()
    T = torch.zeros((16, op.n), dtype=torch.complex128, device="cuda")
    info, st = op.cfie_solve(I.random_directions(5, 16), T, tol=1e-8)
    assert st == 0 and info.converged == 16 and info.seconds > 0
    held, model = op.held_bytes(), op.solve_bytes(16)
    print(f"{bc} {prec}: held {held / 1e6:.2f} MB, model {model / 1e6:.2f} MB, solve {info.seconds:.3f} s",
          flush=True)
    assert held <= model and held >= 0.5 * model
    assert ctx.used_bytes() == g_bytes + held
    # the solver's buffers stay with the operator: the same solve again allocates nothing
    info2, st2 = op.cfie_solve(I.random_directions(6, 16), T, tol=1e-8)
    assert st2 == 0 and op.held_bytes() == held and ctx.used_bytes() == g_bytes + held


@pytest.mark.parametrize("bc,prec", CASES[:2])
def test_budget_rejects_solve_before_any_work(bc, prec):
    from paper_2306_11324_amd import inputs as I
    b = B()
    probe = b.Context(0)
    geo0 = geometry(probe)
    g_bytes = probe.used_bytes()
    op0 = operator(probe, geo0, bc, prec)
    held1 = op0.held_bytes()
    ndir = 1024
    one, many = op0.solve_bytes(1), op0.solve_bytes(ndir)
    del op0, geo0
    # room for the operator (and its assembly's staging) and half the growth of
    # an ndir-direction solve
    budget = g_bytes + held1 + (many - held1) // 2
    assert one <= budget - g_bytes, (one, many, held1)
    print(f"case: {bc} {prec}: budget {budget} bytes, model 1 / 16 directions {one} / {many}", flush=True)
    ctx = b.Context(0, hbm_budget=budget)
    geo = geometry(ctx)
    op = operator(ctx, geo, bc, prec)
    used = ctx.used_bytes()
    T = torch.zeros((ndir, op.n), dtype=torch.complex128, device="cuda")
    with pytest.raises(b.IgbError) as e:
        op.cfie_solve(I.random_directions(5, ndir), T, tol=1e-8)
    assert e.value.status == -3 and "budget" in str(e.value)
    assert ctx.used_bytes() == used
    info, st = op.cfie_solve(I.random_directions(5, 1), T[:1], tol=1e-8)
    assert st == 0 and info.converged == 1 and ctx.used_bytes() <= budget


@pytest.mark.parametrize("bc", ["soft", "hard"])
def test_host_array_matvec_equals_device_matvec(bc):
    from paper_2306_11324_amd import inputs as I
    b = B()
    ctx = b.Context(0)
    geo = geometry(ctx)
    op = operator(ctx, geo, bc, "fp64")
    X = I.random_complex(21, (3, op.n))
    Yh = np.zeros_like(X)
    op.h2_matvec(X, Yh, nrhs=3, parts=b.PART_ALL | b.MV_HOST)
    xd = torch.from_numpy(X).cuda()
    yd = torch.zeros_like(xd)
    op.h2_matvec(xd, yd, nrhs=3)
    torch.cuda.synchronize()
    assert np.array_equal(Yh, yd.cpu().numpy())
