"""GMRES on operators shorter than one 64-entry workgroup of the Gram-Schmidt
subtraction (level-1 sphere: n = 54 on S^2 with p = 1, fewer on the glued S^0
with p = 2), where one workgroup spans several columns: several directions
solved together equal each solved alone bitwise, and each converges to the
dense oracle's LU solution (same Galerkin matrix up to the H^2 interpolation
and quadrature differences, 1e-6)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("bc,p", [("soft", 1), ("hard", 2)])
def test_small_systems_block_equals_single_and_oracle(bc, p):
    from oracle import galerkin as G
    from paper_2306_11324_amd import binding as b, inputs as I
    ctx = b.Context(0)
    print(f"case: sphere m=1 p={p} kappa=1 q=6 leaf_depth=0 bc={bc}, 5 directions", flush=True)
    geo = b.Geometry(ctx, I.sphere_patches(), 1, p)
    op = b.Operator(ctx, geo, kappa=1.0, q=6, leaf_depth=0, bc=b.SOFT if bc == "soft" else b.HARD)
    n = op.n
    assert n < 64
    dirs = I.random_directions(11, 5)
    T = torch.zeros((5, n), dtype=torch.complex128, device="cuda")
    info, st = op.cfie_solve(dirs, T, tol=1e-12)
    assert st == 0 and info.converged == 5
    Tb = T.cpu().numpy()
    for c in range(5):
        t1 = torch.zeros(n, dtype=torch.complex128, device="cuda")
        i1, s1 = op.cfie_solve(dirs[c:c + 1], t1, tol=1e-12)
        assert s1 == 0
        assert np.array_equal(t1.cpu().numpy(), Tb[c]), c
    bem = G.DenseBEM(I.sphere_patches(), p=p, m=1, kappa=1.0, bc=bc)
    for c in range(5):
        t_ref = bem.solve(dirs[c])
        err = np.abs(Tb[c] - t_ref).max() / np.abs(t_ref).max()
        print(f"{bc} direction {c}: rel diff vs oracle LU {err:.2e}", flush=True)
        assert err < 1e-6
