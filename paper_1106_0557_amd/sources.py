"""Seeded synthetic sources shaped like the paper's test problems.

This module only builds source arrays S (and request traces); it holds none of
the solver's arithmetic.  Both the HIP path and the CPU oracle receive the very
same arrays from here.

Geometry convention (cell-centred mesh): cell (i, j, k) of an (nx, ny, nz) grid
with spacings h sits at ``origin + (i + 1/2, j + 1/2, k + 1/2) * h``.  A point
belongs to a body when it lies inside or on its surface.  Arrays have shape
(nz, ny, nx), x fastest, float64.

Bodies follow Sec. 4 of the paper: the uniform sphere (Sec. 4.1), the
homogeneous oblate spheroid (Sec. 4.2) and the binary spheroid (Sec. 4.3), with
source value 4 pi G rho inside.  The Gaussian-blob fields stand in for the
generic astrophysical systems the paper mentions; their recipe is fixed here:
S(x) = sum_b A_b exp(-|x - c_b|^2 / (2 sigma_b^2)) with c_b ~ U(0.25, 0.75)^3
(box units), sigma_b ~ U(0.02, 0.08), A_b ~ N(1, 0.3), drawn in the order
(c, sigma, A) per blob from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

FOUR_PI = 4.0 * math.pi


def _as3(v, kind=float):
    if np.isscalar(v):
        return (kind(v),) * 3
    v = tuple(kind(x) for x in v)
    if len(v) != 3:
        raise ValueError("expected a scalar or a 3-sequence")
    return v


def cell_centres(n, h, origin=(0.0, 0.0, 0.0), device="cpu"):
    """1D coordinate vectors (x, y, z) of the cell centres."""
    nx, ny, nz = _as3(n, int)
    hx, hy, hz = _as3(h)
    ox, oy, oz = _as3(origin)
    f = dict(dtype=torch.float64, device=device)
    x = ox + (torch.arange(nx, **f) + 0.5) * hx
    y = oy + (torch.arange(ny, **f) + 0.5) * hy
    z = oz + (torch.arange(nz, **f) + 0.5) * hz
    return x, y, z


def _sub_offsets(sub, device):
    """Offsets (in cells) of sub x sub x sub sample points inside one cell, centred."""
    return (torch.arange(sub, dtype=torch.float64, device=device) + 0.5) / sub - 0.5


def _ellipsoid_fraction(n, h, origin, centre, semi, sub, device, zchunk=64):
    """Fraction of the ``sub^3`` sample points of each cell with sum((x-c)/semi)^2 <= 1.

    ``sub = 1`` is point sampling at the cell centre; larger ``sub`` approximates the
    volume fraction of the cell inside the body.  Computed in slabs of ``zchunk``
    planes to bound temporary memory on large meshes.
    """
    x, y, z = cell_centres(n, h, origin=origin, device=device)
    hx, hy, hz = _as3(h)
    cx, cy, cz = _as3(centre)
    ax, ay, az = _as3(semi)
    off = _sub_offsets(sub, device)
    qx = (((x[:, None] + off[None, :] * hx) - cx) / ax) ** 2      # (nx, sub)
    qy = (((y[:, None] + off[None, :] * hy) - cy) / ay) ** 2
    qz = (((z[:, None] + off[None, :] * hz) - cz) / az) ** 2
    nx, ny, nz = x.numel(), y.numel(), z.numel()
    acc = torch.zeros((nz, ny, nx), dtype=torch.float64, device=device)
    for z0 in range(0, nz, zchunk):
        z1 = min(nz, z0 + zchunk)
        for k in range(sub):
            for j in range(sub):
                q = qz[z0:z1, k][:, None, None, None] + qy[:, j][None, :, None, None] + qx[None, None, :, :]
                acc[z0:z1] += (q <= 1.0).to(torch.float64).sum(dim=-1)
    return acc / float(sub ** 3)


def sphere(n, h, radius, centre, value=1.0, sub=1, origin=(0.0, 0.0, 0.0), device="cpu"):
    """``value`` inside a sphere (config 1: n=32, h=1/32, R=0.25, centre 1/2, value 1)."""
    return value * _ellipsoid_fraction(n, h, origin, centre, radius, sub, device)


def spheroid(n, h, a, b, centre, value=FOUR_PI, sub=1, origin=(0.0, 0.0, 0.0), device="cpu"):
    """``value`` inside (x^2+y^2)/a^2 + z^2/b^2 <= 1 around ``centre`` (config 2: a=0.3, b=0.15)."""
    return value * _ellipsoid_fraction(n, h, origin, centre, (a, a, b), sub, device)


def binary_spheroid(n, h, a, b, centres_x, origin, value=FOUR_PI, sub=1, device="cpu"):
    """Two spheroids centred at (c, 0, 0) for c in ``centres_x`` (Sec. 4.3)."""
    out = None
    for c in centres_x:
        part = value * _ellipsoid_fraction(n, h, origin, (c, 0.0, 0.0), (a, a, b), sub, device)
        out = part if out is None else out + part
    return out


@dataclass
class Blob:
    centre: tuple
    sigma: float
    amplitude: float


def draw_blobs(rng: np.random.Generator, count: int):
    blobs = []
    for _ in range(count):
        c = tuple(float(v) for v in rng.uniform(0.25, 0.75, size=3))
        s = float(rng.uniform(0.02, 0.08))
        a = float(rng.normal(1.0, 0.3))
        blobs.append(Blob(c, s, a))
    return blobs


def blob_field(n, blobs, h=None, device="cpu"):
    """Sum of Gaussian blobs on the unit box (h = 1/n per axis unless given)."""
    nx, ny, nz = _as3(n, int)
    if h is None:
        h = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    x, y, z = cell_centres((nx, ny, nz), h, device=device)
    out = torch.zeros((nz, ny, nx), dtype=torch.float64, device=device)
    for bl in blobs:
        cx, cy, cz = bl.centre
        k = -0.5 / (bl.sigma * bl.sigma)
        ex = torch.exp(k * (x - cx) ** 2)
        ey = torch.exp(k * (y - cy) ** 2)
        ez = torch.exp(k * (z - cz) ** 2)
        out += bl.amplitude * ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
    return out


def random_field(n, seed, device="cpu"):
    """Uniform(-1, 1) noise source, for parity tests."""
    nx, ny, nz = _as3(n, int)
    g = np.random.default_rng(seed)
    return torch.from_numpy(g.uniform(-1.0, 1.0, size=(nz, ny, nx))).to(device)


# ----------------------------------------------------------- configurations --

def config1(device="cpu"):
    """Plain FP64, n=32, h=1/32, S=1 in a centred sphere of radius 0.25."""
    n = 32
    return n, 1.0 / n, sphere(n, 1.0 / n, 0.25, 0.5, 1.0, device=device)


def config2(n=128, device="cpu"):
    """n=128 (256^3 padded), homogeneous oblate spheroid a=0.3, b=0.15, S=4 pi inside."""
    return n, 1.0 / n, spheroid(n, 1.0 / n, 0.3, 0.15, 0.5, FOUR_PI, device=device)


CONFIG3_SIZES = (32, 48, 64, 96, 128)


def config3(seed=3, count=64, blobs_per_source=8, device="cpu"):
    """64 independent Gaussian-blob sources, n ~ U{32,48,64,96,128}."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice(CONFIG3_SIZES))
        blobs = draw_blobs(rng, blobs_per_source)
        out.append((n, blob_field(n, blobs, device=device)))
    return out


CONFIG4_SIZES = (64, 96, 128, 192, 256)
CONFIG4_WEIGHTS = (0.3, 0.25, 0.2, 0.15, 0.1)


@dataclass
class Request:
    index: int
    arrival: float       # seconds from trace start
    n: int
    blobs: list


def config4_trace(rate_hz: float, count=2000, seed=4, sizes=CONFIG4_SIZES, weights=CONFIG4_WEIGHTS,
                  blobs_per_source=8):
    """Poisson arrivals at ``rate_hz``; sizes drawn with the given weights.

    Draw order per request: inter-arrival gap, size, then the blobs.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    w = np.asarray(weights, dtype=np.float64)
    w = w / w.sum()
    for i in range(count):
        t += float(rng.exponential(1.0 / rate_hz)) if rate_hz > 0 else 0.0
        n = int(rng.choice(np.asarray(sizes), p=w))
        reqs.append(Request(i, t, n, draw_blobs(rng, blobs_per_source)))
    return reqs


def config5(n=512, seed=5, device="cpu"):
    """64 Gaussian blobs plus 1 inside a centred sphere of radius 0.2, unit box."""
    rng = np.random.default_rng(seed)
    blobs = draw_blobs(rng, 64)
    S = blob_field(n, blobs, device=device)
    S += sphere(n, 1.0 / n, 0.2, 0.5, 1.0, device=device)
    return n, 1.0 / n, S
