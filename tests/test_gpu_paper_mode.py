"""Separate H^2 matrices per operator (the set-up of Sec. 5.1: each matrix of
the CFIE compressed on its own, their sum applied lazily) and the single
boundary integral operators exposed on their own:

  * IGB_OP_V, IGB_OP_KSTAR (S^2, p = 1) and IGB_OP_K, IGB_OP_W (S^0, p = 2) on
    the level-2 sphere, kappa = 1, against the dense oracle matrices
    (tests/golden/sphere_m2_k1_operators.npz);
  * the separate form against the fused one (one H^2 matrix of the combined
    kernel): the same interpolated operator, so matvecs and solves agree to
    rounding, at twice the coupling memory.
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


@pytest.mark.parametrize("name", ["V", "Kstar", "K", "W"])
def test_single_operator_against_dense_oracle(name):
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    g = dict(np.load(os.path.join(GOLD, "sphere_m2_k1_operators.npz")))
    soft = name in ("V", "Kstar")
    p = 1 if soft else 2
    form = {"V": B.OP_V, "Kstar": B.OP_KSTAR, "K": B.OP_K, "W": B.OP_W}[name]
    print(f"case: sphere m=2 p={p} kappa=1 q=8 leaf depth 0, single operator {name}", flush=True)
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.sphere_patches(), 2, p)
    op = B.Operator(ctx, geo, kappa=1.0, q=8, leaf_depth=0, formulation=form)
    assert op.n == (geo.n2 if soft else geo.n0) and op.info.far_pairs > 0
    x = g["soft_x" if soft else "hard_x"]
    y = _apply(op, x)
    e = float(np.max(np.abs(y - g[f"{name}_y"]) / (g[f"{name}_rownorm1"] * np.abs(x).max())))
    print(f"{name}: operator-relative error {e:.2e}", flush=True)
    assert e < 1e-7
    with pytest.raises(B.IgbError):
        op.cfie_rhs(np.array([[0.0, 0.0, 1.0]]), torch.zeros((1, op.n), dtype=torch.complex128, device="cuda"))


@pytest.mark.parametrize("bc", ["soft", "hard"])
def test_separate_matrices_equal_fused_operator(bc):
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    print(f"case: sphere m=4 p=2 kappa=4 q=6 leaf depth 2 {bc}: separate vs fused", flush=True)
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.sphere_patches(), 4, 2)
    ops = {sep: B.Operator(ctx, geo, kappa=4.0, bc=B.SOFT if bc == "soft" else B.HARD, q=6, leaf_depth=2,
                           separate=sep) for sep in (False, True)}
    fused, sepa = ops[False], ops[True]
    assert sepa.n == fused.n and sepa.info.far_pairs == 2 * fused.info.far_pairs
    print(f"device bytes fused {fused.info.device_bytes / 1e6:.0f} MB, separate {sepa.info.device_bytes / 1e6:.0f} MB",
          flush=True)
    x = I.random_complex(5, (3, fused.n))
    yf, ys = _apply(fused, x), _apply(sepa, x)
    e = float(np.abs(ys - yf).max() / np.abs(yf).max())
    print(f"matvec separate vs fused {e:.2e}", flush=True)
    assert e < 1e-12
    d = I.random_directions(3, 2)
    sol = {}
    for sep, op in ops.items():
        c = torch.zeros((2, op.n), dtype=torch.complex128, device="cuda")
        info, st = op.cfie_solve(d, c, tol=1e-10, restart=30, maxit=1000)
        assert st == 0 and info.converged == 2
        u = torch.zeros((2, 64), dtype=torch.complex128, device="cuda")
        op.farfield(c, I.fibonacci_directions(64), u, ndir=2)
        torch.cuda.synchronize()
        sol[sep] = u.cpu().numpy()
    e = float(np.abs(sol[True] - sol[False]).max() / np.abs(sol[False]).max())
    print(f"far field separate vs fused {e:.2e}", flush=True)
    assert e < 1e-9


def test_separate_matrices_in_bf16_refinement_and_potential():
    """The separate form with bf16 couplings inside fp64 refinement reaches the
    fp64 tolerance like the fused form, and its scattered field (direct and H^2
    evaluation, which read the first matrix's tree) equals the fused one's."""
    from paper_2306_11324_amd import binding as B
    from paper_2306_11324_amd import inputs as I
    print("case: sphere m=4 p=2 kappa=4 q=6 leaf depth 2 soft bf16: separate vs fused", flush=True)
    ctx = B.Context(0)
    geo = B.Geometry(ctx, I.sphere_patches(), 4, 2)
    d = I.random_directions(5, 2)
    pts = 2.5 * I.fibonacci_directions(500)
    out = {}
    for sep in (False, True):
        op = B.Operator(ctx, geo, kappa=4.0, q=6, leaf_depth=2, precision=B.MIX_BF16, separate=sep)
        c = torch.zeros((2, op.n), dtype=torch.complex128, device="cuda")
        info, st = op.cfie_solve(d, c, tol=1e-10, restart=30, maxit=1000)
        assert st == 0 and info.converged == 2 and info.relres_true <= 1e-10
        u = torch.zeros((2, len(pts)), dtype=torch.complex128, device="cuda")
        uh = torch.zeros_like(u)
        op.potential(c, pts, u, ndir=2)
        op.potential_h2(c, pts, uh, ndir=2)
        torch.cuda.synchronize()
        out[sep] = (u.cpu().numpy(), uh.cpu().numpy())
        del op
    e = float(np.abs(out[True][0] - out[False][0]).max() / np.abs(out[False][0]).max())
    eh = float(np.abs(out[True][1] - out[True][0]).max() / np.abs(out[True][0]).max())
    print(f"separate vs fused field {e:.2e}; H^2 vs direct on the separate form {eh:.2e}", flush=True)
    assert e < 1e-8 and eh < 1e-5
