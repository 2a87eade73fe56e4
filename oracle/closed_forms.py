"""Analytic potentials used as physics pins (test infrastructure only).

All functions take coordinates relative to the body's centre and the product
``G_rho`` = G * rho (the source is S = 4 pi G rho inside the body, Sec. 4.1).

* :func:`phi_sphere` -- uniform sphere of radius R, Sec. 4.1:
  inside  -(2/3) pi G rho (3 R^2 - r^2), outside -(4/3) pi G rho R^3 / r.
* :func:`phi_spheroid` -- homogeneous oblate spheroid with semi-axes a (in x, y)
  and b (in z), a > b, Sec. 4.2: eccentricity e = sqrt(1 - (b/a)^2); inside,
  Eq. (spheroid_potential_inside) with the coefficients A and B; outside,
  Eq. (spheroid_potential_outside) with eta = a e / sqrt(b^2 + lambda), lambda
  the positive root of Eq. (spheroid_potential_auxiliary).
* :func:`phi_binary_spheroid` -- Sec. 4.3: superposition of two spheroids with
  x replaced by x - c for each centre c.
"""
from __future__ import annotations

import numpy as np


def phi_sphere(x, y, z, R: float, G_rho: float = 1.0):
    x, y, z = (np.asarray(v, dtype=np.float64) for v in (x, y, z))
    r2 = x * x + y * y + z * z
    r = np.sqrt(r2)
    inside = -(2.0 / 3.0) * np.pi * G_rho * (3.0 * R * R - r2)
    with np.errstate(divide="ignore", invalid="ignore"):
        outside = -(4.0 / 3.0) * np.pi * G_rho * R**3 / r
    return np.where(r <= R, inside, outside)


def spheroid_coefficients(e: float):
    """A and B of Eq. (spheroid_potential_inside), as functions of e."""
    s = np.sqrt(1.0 - e * e)
    ase = np.arcsin(e)
    A = s / e**3 * ase - (1.0 - e * e) / (e * e)
    B = 2.0 / (e * e) - 2.0 * s / e**3 * ase
    return A, B


def spheroid_lambda(x, y, z, a: float, b: float):
    """Positive root of (x^2+y^2)/(a^2+lam) + z^2/(b^2+lam) = 1 (valid outside)."""
    w2 = x * x + y * y
    z2 = z * z
    B = a * a + b * b - w2 - z2
    C = a * a * b * b - w2 * b * b - z2 * a * a
    disc = np.maximum(B * B - 4.0 * C, 0.0)
    return 0.5 * (-B + np.sqrt(disc))


def phi_spheroid(x, y, z, a: float, b: float, G_rho: float = 1.0):
    if not a > b > 0:
        raise ValueError("phi_spheroid expects an oblate spheroid, a > b > 0")
    x, y, z = (np.asarray(v, dtype=np.float64) for v in (x, y, z))
    e = np.sqrt(1.0 - (b / a) ** 2)
    A, B = spheroid_coefficients(e)
    w2 = x * x + y * y
    z2 = z * z
    inside_mask = w2 / (a * a) + z2 / (b * b) <= 1.0
    phi_in = -np.pi * G_rho * (A * (2.0 * a * a - w2) + B * (b * b - z2))
    lam = np.where(inside_mask, 0.0, spheroid_lambda(x, y, z, a, b))
    eta = a * e / np.sqrt(b * b + lam)
    at = np.arctan(eta)
    phi_out = -2.0 * np.pi * G_rho * (a * b / e) * (
        at - (w2 * (at - eta / (1.0 + eta * eta)) + 2.0 * z2 * (eta - at)) / (2.0 * a * a * e * e)
    )
    return np.where(inside_mask, phi_in, phi_out)


def phi_binary_spheroid(x, y, z, a: float, b: float, centres_x, G_rho: float = 1.0):
    x = np.asarray(x, dtype=np.float64)
    total = 0.0
    for c in centres_x:
        total = total + phi_spheroid(x - c, y, z, a, b, G_rho)
    return total
