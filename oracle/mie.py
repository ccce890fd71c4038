"""Closed-form solutions on the sphere (textbook separation of variables).

Used as pins of the whole discretisation (not of any single step):

* Mie far-field pattern of a plane wave e^{i kappa d.x} scattered by the
  sphere of radius a (the far-field normalisation of Sec. 2:
  u_s ~ e^{i kappa |x|}/|x| u_inf):
      soft  u_inf(theta) = (i/kappa) sum_n (2n+1) j_n(ka)/h_n(ka)   P_n(cos theta)
      hard  u_inf(theta) = (i/kappa) sum_n (2n+1) j_n'(ka)/h_n'(ka) P_n(cos theta)
* eigenvalues of the boundary integral operators of Sec. 2 on spherical
  harmonics of degree n (h_n = h_n^(1)):
      V : i kappa a^2 j_n h_n
      K = K* : (i kappa^2 a^2 / 2) (j_n h_n' + j_n' h_n)
      W : -i kappa^3 a^2 j_n' h_n'
* optical theorem  int_{S^2} |u_inf|^2 = (4 pi / kappa) Im u_inf(d).
* scattered field outside the sphere (plane-wave expansion of the incident
  wave, outgoing spherical Hankel functions), x = r x^, cos theta = d.x^:
      u_s(x) = - sum_n (2n+1) i^n c_n h_n(kappa r) P_n(cos theta),
      c_n = j_n(ka)/h_n(ka) (soft), j_n'(ka)/h_n'(ka) (hard);
  h_n(z) ~ (-i)^(n+1) e^{iz}/z recovers the far-field pattern above.
"""
from __future__ import annotations

import numpy as np
from scipy.special import eval_legendre, spherical_jn, spherical_yn


def _h(n, z, derivative=False):
    return spherical_jn(n, z, derivative) + 1j * spherical_yn(n, z, derivative)


def farfield(kappa: float, cos_theta, bc: str = "soft", a: float = 1.0, nmax: int | None = None):
    ka = kappa * a
    nmax = nmax or int(ka + 4 * ka ** (1 / 3) + 20)
    ct = np.asarray(cos_theta, dtype=np.float64)
    u = np.zeros(ct.shape, dtype=np.complex128)
    for n in range(nmax + 1):
        if bc == "soft":
            c = spherical_jn(n, ka) / _h(n, ka)
        else:
            c = spherical_jn(n, ka, True) / _h(n, ka, True)
        u += (2 * n + 1) * c * eval_legendre(n, ct)
    return 1j / kappa * u


def eig_V(n, kappa, a=1.0):
    return 1j * kappa * a * a * spherical_jn(n, kappa * a) * _h(n, kappa * a)


def eig_K(n, kappa, a=1.0):
    z = kappa * a
    return 0.5j * z * z * (spherical_jn(n, z) * _h(n, z, True) + spherical_jn(n, z, True) * _h(n, z))


def eig_W(n, kappa, a=1.0):
    z = kappa * a
    return -1j * kappa ** 3 * a * a * spherical_jn(n, z, True) * _h(n, z, True)


def scattered(kappa: float, points, d, bc: str = "soft", a: float = 1.0, nmax: int | None = None):
    """Scattered field u_s at points with |x| > a for the incident direction d."""
    x = np.atleast_2d(np.asarray(points, dtype=np.float64))
    d = np.asarray(d, dtype=np.float64) / np.linalg.norm(d)
    r = np.linalg.norm(x, axis=1)
    ct = (x @ d) / r
    ka = kappa * a
    # c_n h_n(kappa r) ~ ka (a/r)^(n+1) (ka)^n / (2n+1)!! for n > ka: the
    # truncation depends on ka only, for any r > a
    nmax = nmax or int(ka + 4 * max(ka, 1.0) ** (1 / 3) + 25)
    u = np.zeros(len(r), dtype=np.complex128)
    for n in range(nmax + 1):
        c = spherical_jn(n, ka) / _h(n, ka) if bc == "soft" else spherical_jn(n, ka, True) / _h(n, ka, True)
        u -= (2 * n + 1) * (1j ** n) * c * _h(n, kappa * r) * eval_legendre(n, ct)
    return u
