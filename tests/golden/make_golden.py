"""Writes the stored oracle values used by the GPU parity tests.

Calls only ``oracle`` (and the seeded input generators); nothing here comes
from the HIP path.  Run from the repository root:

    python tests/golden/make_golden.py [case ...]

Cases
  sphere_m3_p2_k2_q4  sphere, m = 3, p = 2, kappa = 2, soft, q = 4, eta = 1.6,
                      leaf depth 1: O2 far product, O1 near product, sampled
                      near entries, right-hand side, for the seeded vector x.
  sphere_m3_p2_k2_q4_block  the same operators (soft on S^2, hard on S^0): O2's
                      far product of 20 seeded columns, one column at a time
                      (blocks of 16 and more columns run another code path).
  sphere_m2_p1_k1     the m = 2, p = 1, kappa = 1 sphere workload: dense O1
                      matrix, right-hand side for d = (0,0,1), LU solution,
                      far field at 64 Fibonacci directions and the Mie values.
  sphere_m5_p2_k8_rows  the m = 5, p = 2, kappa = 8 sphere workload: sampled
                      rows of the dense O1 matrix applied to the seeded vector.
  sphere_m3_p2_k2_q4_hard / sphere_m2_p2_k1_hard  the same two small checks for
                      the sound-hard operator (regularised W) on S^0.
  sphere_m2_k1_potential  scattered field at 72 points (r = 1.5, 2, 3) of the
                      dense LU solutions on the level-2 sphere (soft p = 1, hard
                      p = 2, kappa = 1), and the Mie series there.
  torus_k2p5_potential  the torus (R = 2, r = 0.5, 16 patches), kappa = 2.5,
                      d = (1, 0, 0): dense LU solutions (soft p = 1 on level 2,
                      hard p = 2 on level 1) and their scattered field at 100
                      Fibonacci points on the radius-5 sphere (Sec. 5.2's set-up),
                      with raised quadrature orders (TORUS_RULES, right-hand side
                      and potential 12 x 12): the elements are 3-5 times longer
                      around the major circle than around the minor one and up to
                      ~0.8 wavelengths long, where the default orders leave errors
                      near 1e-6; with these orders a further raise (regular
                      12/15/18, touching 16) moves the level-1 soft solution by
                      3.6e-8 (relative, coefficients) and its field by 1.1e-8.
  sphere_m2_k1_single_layer  the indirect single-layer formulations on the
                      level-2 sphere, p = 1, kappa = 1, d = (0, 0, 1): dense LU
                      solutions (soft V t = u_inc, hard (K* - 1/2) t = d_n u_inc)
                      and their scattered field at the 72 points of
                      sphere_m2_k1_potential.
  sphere_m2_k1_operators  the single Galerkin matrices on the level-2 sphere,
                      kappa = 1, applied to the seeded vector: V and K* on S^2
                      (p = 1), K and the regularised W on S^0 (p = 2).
  sphere_m5_p2_potential  the level-5 sphere (p = 2, 6144 elements), kappa = 3
                      and 8, soft (S^2) and hard (S^0): the scattered field of
                      seeded density coefficients at 160 seeded points in the
                      shell 1.2 <= |x| <= 4 (representation formulas, tensor
                      Gauss 10 x 10 per element; the points are at least four
                      element sizes from the surface).
  star_m6_p2_k16_rows  seed-0 star, m = 6, p = 2, kappa = 16, soft: sampled rows
                      of the dense O1 matrix applied to the seeded vector.
  star_m7_p2_k32_hard_rows  seed-0 star, m = 7, p = 2, kappa = 32, hard (S^0):
                      the same for four rows.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import galerkin as G  # noqa: E402
from oracle import h2, mie  # noqa: E402
from paper_2306_11324_amd import inputs as I  # noqa: E402

X_SEED = 12345
ROW_SEED = 777


def case_sphere_m3_p2_k2_q4():
    bem = G.DenseBEM(I.sphere_patches(), p=2, m=3, kappa=2.0, bc="soft")
    H = h2.H2Oracle(bem, q=4, eta=1.6, leaf_depth=1)
    x = I.random_complex(X_SEED, bem.n)
    A = H.near_matrix()
    nz = np.argwhere(A != 0)
    pick = nz[np.random.default_rng(ROW_SEED).choice(len(nz), 4000, replace=False)]
    d = np.array([0.3, -0.2, 0.9])
    return dict(x=x, y_far=H.far_apply(x), y_near=A @ x, ent_ij=pick.astype(np.int32),
                ent_val=A[pick[:, 0], pick[:, 1]], d=d, rhs=bem.rhs(d), nfar=len(H.far))


def case_sphere_m3_p2_k2_q4_block(ncol=20):
    out = {}
    for bc in ("soft", "hard"):
        bem = G.DenseBEM(I.sphere_patches(), p=2, m=3, kappa=2.0, bc=bc)
        H = h2.H2Oracle(bem, q=4, eta=1.6, leaf_depth=1)
        X = I.random_complex(X_SEED + 1, (ncol, bem.n))
        out[f"{bc}_X"] = X
        out[f"{bc}_Y_far"] = np.stack([H.far_apply(x) for x in X])
    return out


def case_sphere_m2_p1_k1():
    bem = G.DenseBEM(I.sphere_patches(), p=1, m=2, kappa=1.0, bc="soft")
    A = bem.matrix()
    d = np.array([0.0, 0.0, 1.0])
    b = bem.rhs(d)
    t = np.linalg.solve(A, b)
    obs = I.fibonacci_directions(64)
    return dict(A=A, d=d, rhs=b, t=t, obs=obs, uinf=bem.farfield(t, obs),
                mie=mie.farfield(1.0, obs @ d, "soft"), x=I.random_complex(X_SEED, bem.n))


def case_sphere_m5_p2_k8_rows(nrows=6):
    bem = G.DenseBEM(I.sphere_patches(), p=2, m=5, kappa=8.0, bc="soft")
    x = I.random_complex(X_SEED, bem.n)
    rows = np.sort(np.random.default_rng(ROW_SEED).choice(bem.n, nrows, replace=False))
    R = bem.rows(rows)
    return dict(rows=rows.astype(np.int64), y=R @ x, rownorm1=np.abs(R).sum(1), x=x)


def case_sphere_m3_p2_k2_q4_hard():
    bem = G.DenseBEM(I.sphere_patches(), p=2, m=3, kappa=2.0, bc="hard")
    H = h2.H2Oracle(bem, q=4, eta=1.6, leaf_depth=1)
    x = I.random_complex(X_SEED, bem.n)
    A = H.to_solution_space(H.near_matrix())
    nz = np.argwhere(A != 0)
    pick = nz[np.random.default_rng(ROW_SEED).choice(len(nz), 4000, replace=False)]
    d = np.array([0.3, -0.2, 0.9])
    return dict(x=x, y_far=H.far_apply(x), y_near=A @ x, ent_ij=pick.astype(np.int32),
                ent_val=A[pick[:, 0], pick[:, 1]], d=d, rhs=bem.rhs(d), nfar=len(H.far))


def case_sphere_m2_p2_k1_hard():
    bem = G.DenseBEM(I.sphere_patches(), p=2, m=2, kappa=1.0, bc="hard")
    A = bem.matrix()
    d = np.array([0.0, 0.0, 1.0])
    b = bem.rhs(d)
    t = np.linalg.solve(A, b)
    obs = I.fibonacci_directions(64)
    return dict(A=A, d=d, rhs=b, t=t, obs=obs, uinf=bem.farfield(t, obs),
                mie=mie.farfield(1.0, obs @ d, "hard"), x=I.random_complex(X_SEED, bem.n))


def case_sphere_m2_k1_potential():
    out = {}
    d = np.array([0.0, 0.0, 1.0])
    pts = np.concatenate([r * I.fibonacci_directions(24) for r in (1.5, 2.0, 3.0)])
    for bc, p in (("soft", 1), ("hard", 2)):
        bem = G.DenseBEM(I.sphere_patches(), p=p, m=2, kappa=1.0, bc=bc)
        t = bem.solve(d)
        out[f"{bc}_t"] = t
        out[f"{bc}_pot"] = bem.potential(t, pts)
        out[f"{bc}_mie"] = mie.scattered(1.0, pts, d, bc)
    out["pts"] = pts
    out["d"] = d
    return out


def case_sphere_m2_k1_single_layer():
    out = {}
    d = np.array([0.0, 0.0, 1.0])
    pts = np.concatenate([r * I.fibonacci_directions(24) for r in (1.5, 2.0, 3.0)])
    for bc in ("soft", "hard"):
        bem = G.DenseBEM(I.sphere_patches(), p=1, m=2, kappa=1.0, bc=bc, formulation="single_layer")
        t = bem.solve(d)
        out[f"{bc}_t"] = t
        out[f"{bc}_pot"] = bem.potential(t, pts)
    out["pts"] = pts
    out["d"] = d
    return out


def case_sphere_m2_k1_operators():
    out = {}
    for bc, p, ops in (("soft", 1, ("V", "Kstar")), ("hard", 2, ("K", "W"))):
        bem = G.DenseBEM(I.sphere_patches(), p=p, m=2, kappa=1.0, bc=bc)
        x = I.random_complex(X_SEED, bem.n)
        mats = bem.operator_matrices()
        out[f"{bc}_x"] = x
        for name in ops:
            out[f"{name}_y"] = mats[name] @ x
            out[f"{name}_rownorm1"] = np.abs(mats[name]).sum(1)
    return out


TORUS_RULES = dict(n_far=10, n_mid=12, n_near=14, n_sing=13)


def case_torus_k2p5_potential():
    out = {}
    d = np.array([1.0, 0.0, 0.0])
    pts = 5.0 * I.fibonacci_directions(100)
    for bc, p, m in (("soft", 1, 2), ("hard", 2, 1)):
        bem = G.DenseBEM(I.torus_patches(), p=p, m=m, kappa=2.5, bc=bc, rules=G.PairRules(**TORUS_RULES))
        t = np.linalg.solve(bem.matrix(), bem.rhs(d, n=12))
        out[f"{bc}_t"] = t
        out[f"{bc}_pot"] = bem.potential(t, pts, n=12)
    out["pts"] = pts
    out["d"] = d
    return out


POT_SEED = 2718


def case_sphere_m5_p2_potential():
    rng = np.random.default_rng(POT_SEED)
    dirs = rng.normal(size=(160, 3))
    pts = dirs / np.linalg.norm(dirs, axis=1, keepdims=True) * rng.uniform(1.2, 4.0, size=(160, 1))
    out = {"pts": pts}
    for bc in ("soft", "hard"):
        for kappa in (3.0, 8.0):
            bem = G.DenseBEM(I.sphere_patches(), p=2, m=5, kappa=kappa, bc=bc)
            c = I.random_complex(X_SEED + 2, bem.n)
            out[f"{bc}_c"] = c
            out[f"{bc}_k{int(kappa)}_pot"] = bem.potential(c, pts)
    return out


def _star_rows(m, kappa, bc, nrows):
    bem = G.DenseBEM(I.star_patches(0, I.star_geometry_level(m)), p=2, m=m, kappa=kappa, bc=bc)
    x = I.random_complex(X_SEED, bem.n)
    rows = np.sort(np.random.default_rng(ROW_SEED).choice(bem.n, nrows, replace=False))
    R = bem.rows(rows)
    return dict(rows=rows.astype(np.int64), y=R @ x, rownorm1=np.abs(R).sum(1), x=x)


def case_star_m6_p2_k16_rows():
    return _star_rows(6, 16.0, "soft", 6)


def case_star_m7_p2_k32_hard_rows():
    return _star_rows(7, 32.0, "hard", 4)


CASES = {
    "sphere_m3_p2_k2_q4_hard": case_sphere_m3_p2_k2_q4_hard,
    "sphere_m2_p2_k1_hard": case_sphere_m2_p2_k1_hard,
    "sphere_m3_p2_k2_q4": case_sphere_m3_p2_k2_q4,
    "sphere_m3_p2_k2_q4_block": case_sphere_m3_p2_k2_q4_block,
    "sphere_m2_p1_k1": case_sphere_m2_p1_k1,
    "sphere_m5_p2_k8_rows": case_sphere_m5_p2_k8_rows,
    "star_m6_p2_k16_rows": case_star_m6_p2_k16_rows,
    "sphere_m5_p2_potential": case_sphere_m5_p2_potential,
    "sphere_m2_k1_potential": case_sphere_m2_k1_potential,
    "star_m7_p2_k32_hard_rows": case_star_m7_p2_k32_hard_rows,
    "torus_k2p5_potential": case_torus_k2p5_potential,
    "sphere_m2_k1_single_layer": case_sphere_m2_k1_single_layer,
    "sphere_m2_k1_operators": case_sphere_m2_k1_operators,
}


def main(names):
    for name in names or CASES:
        t = time.time()
        data = CASES[name]()
        np.savez_compressed(os.path.join(HERE, name + ".npz"), **data)
        print(f"{name}: {time.time() - t:.1f} s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
