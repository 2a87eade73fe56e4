"""Analytic potentials used as physics pins (test infrastructure only).

All functions take coordinates relative to the body's centre and the product
``G_rho`` = G * rho (the source is S = 4 pi G rho inside the body, Sec. 4.1).
They accept numpy arrays, or torch tensors (evaluated where the tensors live),
so that large meshes can be checked without moving them to the host.

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

import math

import numpy as np


class _Ops:
    """The few array operations the formulas need, for numpy or torch inputs."""

    def __init__(self, *arrays):
        self.torch = None
        for a in arrays:
            if type(a).__module__.startswith("torch"):
                import torch

                self.torch = torch
                break

    def asarray(self, v):
        if self.torch is not None:
            t = self.torch
            return v.to(t.float64) if isinstance(v, t.Tensor) else t.tensor(v, dtype=t.float64)
        return np.asarray(v, dtype=np.float64)

    def where(self, c, a, b):
        if self.torch is not None:
            t = self.torch
            return t.where(c, a if isinstance(a, t.Tensor) else t.tensor(a, dtype=t.float64, device=c.device),
                           b if isinstance(b, t.Tensor) else t.tensor(b, dtype=t.float64, device=c.device))
        return np.where(c, a, b)

    def sqrt(self, x):
        return self.torch.sqrt(x) if self.torch is not None else np.sqrt(x)

    def arctan(self, x):
        return self.torch.atan(x) if self.torch is not None else np.arctan(x)

    def clamp0(self, x):
        return self.torch.clamp(x, min=0.0) if self.torch is not None else np.maximum(x, 0.0)


def phi_sphere(x, y, z, R: float, G_rho: float = 1.0):
    o = _Ops(x, y, z)
    x, y, z = (o.asarray(v) for v in (x, y, z))
    r2 = x * x + y * y + z * z
    inside = -(2.0 / 3.0) * math.pi * G_rho * (3.0 * R * R - r2)
    outside = -(4.0 / 3.0) * math.pi * G_rho * R**3 / o.sqrt(o.where(r2 > 0, r2, 1.0))
    return o.where(r2 <= R * R, inside, outside)


def spheroid_coefficients(e: float):
    """A and B of Eq. (spheroid_potential_inside), as functions of e."""
    s = math.sqrt(1.0 - e * e)
    ase = math.asin(e)
    A = s / e**3 * ase - (1.0 - e * e) / (e * e)
    B = 2.0 / (e * e) - 2.0 * s / e**3 * ase
    return A, B


def spheroid_lambda(x, y, z, a: float, b: float):
    """Positive root of (x^2+y^2)/(a^2+lam) + z^2/(b^2+lam) = 1 (valid outside)."""
    o = _Ops(x, y, z)
    w2 = x * x + y * y
    z2 = z * z
    B = a * a + b * b - w2 - z2
    C = a * a * b * b - w2 * b * b - z2 * a * a
    disc = o.clamp0(B * B - 4.0 * C)
    return 0.5 * (-B + o.sqrt(disc))


def phi_spheroid(x, y, z, a: float, b: float, G_rho: float = 1.0):
    if not a > b > 0:
        raise ValueError("phi_spheroid expects an oblate spheroid, a > b > 0")
    o = _Ops(x, y, z)
    x, y, z = (o.asarray(v) for v in (x, y, z))
    e = math.sqrt(1.0 - (b / a) ** 2)
    A, B = spheroid_coefficients(e)
    w2 = x * x + y * y
    z2 = z * z
    inside_mask = w2 / (a * a) + z2 / (b * b) <= 1.0
    phi_in = -math.pi * G_rho * (A * (2.0 * a * a - w2) + B * (b * b - z2))
    lam = o.where(inside_mask, 0.0, spheroid_lambda(x, y, z, a, b))
    eta = a * e / o.sqrt(b * b + lam)
    at = o.arctan(eta)
    phi_out = -2.0 * math.pi * G_rho * (a * b / e) * (
        at - (w2 * (at - eta / (1.0 + eta * eta)) + 2.0 * z2 * (eta - at)) / (2.0 * a * a * e * e)
    )
    return o.where(inside_mask, phi_in, phi_out)


def phi_binary_spheroid(x, y, z, a: float, b: float, centres_x, G_rho: float = 1.0):
    total = 0.0
    for c in centres_x:
        total = total + phi_spheroid(x - c, y, z, a, b, G_rho)
    return total
