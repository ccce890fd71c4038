"""Pins of O1 (oracle.galerkin): the dense Galerkin CFIE against what the
mathematics fixes independently of the implementation.

* Mie series far field of the sphere, soft and hard (closed form; Sec. 2's
  far-field pattern), within the 1e-3 accuracy of the discretisation;
* Gauss's identity at kappa = 0: K 1 = -1/2 on a closed surface, so the
  Galerkin rows satisfy K 1 = -1/2 M 1 and the columns 1^T K* = -1/2 1^T M;
* complex symmetry V = V^T, W = W^T and K* = K^T (bilinear duality, Sec. 4.1);
* the sphere eigenvalues of V, K and W on the degree-0 and degree-1 modes;
* the optical theorem on the seeded star (any lossless scatterer);
* eta-independence of the exact solution (CFIE coupling bookkeeping).
"""
import functools

import numpy as np
import pytest

from oracle import galerkin as G
from oracle import mie
from paper_2306_11324_amd import inputs

ALL_OPS = ("V", "Kstar", "K", "W")


@functools.lru_cache(maxsize=None)
def sphere_s2(m, p, kappa):
    bem = G.DenseBEM(inputs.sphere_patches(), p=p, m=m, kappa=kappa, bc="soft")
    return bem, bem.operator_rows_s2(np.arange(bem.disc.n2), ops=ALL_OPS)


def test_gauss_identity_kappa0():
    bem = G.DenseBEM(inputs.star_patches(1, 1), p=1, m=1, kappa=0.0, bc="soft", eta=1.0)
    ops = bem.operator_rows_s2(np.arange(bem.disc.n2), ops=("K", "Kstar"))
    one = np.ones(bem.disc.n2)
    m1 = ops["M"] @ one
    assert np.abs(ops["K"] @ one + 0.5 * m1).max() < 1e-9 * np.abs(m1).max()
    assert np.abs(one @ ops["Kstar"] + 0.5 * (one @ ops["M"])).max() < 1e-9 * np.abs(m1).max()


def test_complex_symmetry():
    _, ops = sphere_s2(2, 2, 1.5)
    for op in ("V", "W", "M"):
        A = ops[op]
        assert np.abs(A - A.T).max() < 1e-10 * np.abs(A).max(), op
    assert np.abs(ops["Kstar"] - ops["K"].T).max() < 1e-10 * np.abs(ops["K"]).max()


def _project(bem, ops, f):
    """S^2 coefficients of the L^2 projection of f(x) onto the continuous S^0
    (the regularised W is the hypersingular operator only on continuous
    functions)."""
    from oracle import quadrature as qd
    disc = bem.disc
    pts, w = qd.tensor2(8)
    E = disc.nelem
    d = disc.eval_on_elements(np.arange(E), np.broadcast_to(pts, (E,) + pts.shape))
    loc = np.einsum("eq,q,eqa->ea", f(d["X"]) * d["a"], w, d["phi"]) * disc.h ** 2
    b = np.zeros(disc.n2)
    np.add.at(b, disc.el_dofs.ravel(), loc.ravel())
    P = disc.glue_matrix()
    return P @ np.linalg.solve(P.T @ ops["M"].real @ P, P.T @ b)


@pytest.mark.parametrize("n", [0, 1])
def test_sphere_eigenvalues(n):
    kappa = 1.5
    bem, ops = sphere_s2(2, 2, kappa)
    if n == 0:
        c = np.ones(bem.disc.n2)
    else:
        c = _project(bem, ops, lambda X: X[..., 2])
    mass = c @ ops["M"] @ c
    for op, lam in (("V", mie.eig_V), ("K", mie.eig_K), ("Kstar", mie.eig_K), ("W", mie.eig_W)):
        val = (c @ ops[op] @ c) / mass
        ref = lam(n, kappa)
        assert abs(val - ref) < 2e-3 * max(abs(ref), 0.05), (op, n, val, ref)


@pytest.mark.parametrize("bc,p,m", [("soft", 1, 2), ("hard", 3, 1)])
def test_mie_sphere(bc, p, m):
    """Sphere, kappa = 1, d = (0,0,1), 64 Fibonacci observation directions: far
    field within 1e-3 of the Mie series (soft: the m = 2, p = 1 workload)."""
    bem = G.DenseBEM(inputs.sphere_patches(), p=p, m=m, kappa=1.0, bc=bc)
    d = np.array([0.0, 0.0, 1.0])
    obs = inputs.fibonacci_directions(64)
    u = bem.farfield(bem.solve(d), obs)
    ref = mie.farfield(1.0, obs @ d, bc)
    assert np.abs(u - ref).max() / np.abs(ref).max() < 1e-3


def test_optical_theorem_and_eta_independence_star():
    bem = G.DenseBEM(inputs.star_patches(0, 2), p=1, m=2, kappa=1.0, bc="soft")
    d = inputs.random_directions(5, 1)[0]
    A = bem.matrix()
    t = np.linalg.solve(A, bem.rhs(d))
    obs = inputs.fibonacci_directions(400)
    u = bem.farfield(t, obs)
    lhs = np.mean(np.abs(u) ** 2) * 4 * np.pi
    rhs = 4 * np.pi / bem.kappa * bem.farfield(t, d[None])[0].imag
    assert abs(lhs - rhs) < 2e-3 * abs(rhs)
    bem2 = G.DenseBEM(inputs.star_patches(0, 2), p=1, m=2, kappa=1.0, bc="soft", eta=3.0)
    t2 = bem2.solve(d)
    u2 = bem2.farfield(t2, obs)
    assert np.abs(u2 - u).max() < 1e-3 * np.abs(u).max()


@pytest.mark.parametrize("kappa", [1.0, 4.0, 16.0, 32.0])
def test_default_coupling_keeps_sphere_modes_in_right_half_plane(kappa):
    """The default couplings (soft eta = kappa, hard eta = -1/kappa) give CFIE
    symbols 1/2 + K_n - i eta V_n and 1/2 - K_n - i eta W_n with positive real
    parts for every degree n on the unit sphere; the opposite hard sign does
    not (negative real parts from kappa = 2 on), which is why it is not used."""
    n = np.arange(0, int(1.5 * kappa) + 40)
    soft = 0.5 + mie.eig_K(n, kappa) - 1j * G.default_eta(kappa, "soft") * mie.eig_V(n, kappa)
    hard = 0.5 - mie.eig_K(n, kappa) - 1j * G.default_eta(kappa, "hard") * mie.eig_W(n, kappa)
    assert soft.real.min() > 0.4 and hard.real.min() > 0.4
    flipped = 0.5 - mie.eig_K(n, kappa) - 1j / kappa * mie.eig_W(n, kappa)
    assert (flipped.real < 0).any() == (kappa >= 2)


@pytest.mark.parametrize("bc", ["soft", "hard"])
def test_sampled_rows_equal_dense_matrix_rows(bc):
    """The sampled-row path used for large sizes (hard: S^0 gluing by index
    accumulation) reproduces rows of the dense matrix."""
    bem = G.DenseBEM(inputs.sphere_patches(), p=2, m=1, kappa=1.5, bc=bc)
    A = bem.matrix()
    rows = np.array([0, 7, bem.n // 2, bem.n - 1])
    R = bem.rows(rows)
    assert np.abs(R - A[rows]).max() < 1e-12 * np.abs(A).max()


def test_mie_scattered_field_tends_to_far_field():
    """The Mie series of the scattered field, times r e^{-i kappa r} at large r,
    approaches the far-field series (independent forms of the same solution)."""
    d = np.array([0.0, 0.0, 1.0])
    xh = inputs.fibonacci_directions(16)
    for bc in ("soft", "hard"):
        R = 2.0e4
        u = mie.scattered(2.0, R * xh, d, bc) * R * np.exp(-2.0j * R)
        ref = mie.farfield(2.0, xh @ d, bc)
        assert np.abs(u - ref).max() < 1e-3 * np.abs(ref).max(), bc


@pytest.mark.parametrize("bc,p,m", [("soft", 1, 2), ("hard", 3, 1)])
def test_potential_matches_mie_outside_sphere(bc, p, m):
    """Scattered field of the discrete solution at points 0.5, 1 and 2 radii
    outside the sphere against the Mie series (within the discretisation error
    the far field shows, 1e-3); at large distance it tends to the discrete far
    field."""
    bem = G.DenseBEM(inputs.sphere_patches(), p=p, m=m, kappa=1.0, bc=bc)
    d = np.array([0.0, 0.0, 1.0])
    t = bem.solve(d)
    xh = inputs.fibonacci_directions(24)
    pts = np.concatenate([r * xh for r in (1.5, 2.0, 3.0)])
    u = bem.potential(t, pts)
    ref = mie.scattered(1.0, pts, d, bc)
    assert np.abs(u - ref).max() < 1e-3 * np.abs(ref).max()
    R = 1.0e4
    far = bem.potential(t, R * xh) * R * np.exp(-1.0j * R)
    uinf = bem.farfield(t, xh)
    assert np.abs(far - uinf).max() < 1e-3 * np.abs(uinf).max()


@pytest.mark.parametrize("bc,p,m", [("soft", 1, 2), ("hard", 1, 2)])
def test_single_layer_formulations_match_mie(bc, p, m):
    """Indirect single-layer ansatz u_s = -S t (soft: V t = u_inc, hard:
    (K* - 1/2) t = d_n u_inc) on the sphere, kappa = 1: far field and scattered
    field within 1e-3 of the Mie series of the same boundary condition (a wrong
    sign of the mass term, of the right-hand side or of the representation
    fails this by O(1))."""
    bem = G.DenseBEM(inputs.sphere_patches(), p=p, m=m, kappa=1.0, bc=bc, formulation="single_layer")
    assert bem.n == bem.disc.n2
    d = np.array([0.0, 0.0, 1.0])
    t = bem.solve(d)
    obs = inputs.fibonacci_directions(64)
    ref = mie.farfield(1.0, obs @ d, bc)
    assert np.abs(bem.farfield(t, obs) - ref).max() / np.abs(ref).max() < 1e-3
    pts = 2.0 * inputs.fibonacci_directions(24)
    ref = mie.scattered(1.0, pts, d, bc)
    assert np.abs(bem.potential(t, pts) - ref).max() < 1e-3 * np.abs(ref).max()


def test_single_layer_hard_operator_is_kstar_minus_half_mass():
    """The hard single-layer matrix is K* - 1/2 M on S^2 and the soft one V:
    on the sphere their actions on the constant mode are the Mie symbols
    lambda(K*) - 1/2 and lambda(V) of degree 0 (mass-weighted)."""
    bem_h = G.DenseBEM(inputs.sphere_patches(), p=0, m=2, kappa=1.0, bc="hard", formulation="single_layer")
    bem_s = G.DenseBEM(inputs.sphere_patches(), p=0, m=2, kappa=1.0, bc="soft", formulation="single_layer")
    parts = bem_s.operator_matrices()
    one = np.ones(bem_s.n)
    mass1 = parts["M"] @ one
    for bem, lam in ((bem_h, mie.eig_K(0, 1.0) - 0.5), (bem_s, mie.eig_V(0, 1.0))):
        y = bem._combine(parts) @ one
        assert np.abs(y - lam * mass1).max() < 3e-3 * np.abs(lam * mass1).max()
