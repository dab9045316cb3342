"""Seeded synthetic workloads (parameters only; no tracing arithmetic here).

`batch_instances` draws the uneven multi-image workload: every instance has
M = 0.5, spin a ~ U[0, 0.49], charge Q ~ U[0, 0.95 sqrt(M^2 - a^2)], camera
radius r0 ~ U[10, 50], inclination theta0 ~ U[5, 90] deg, square image side
drawn from {128, 256, 384, 512} and field of view ~ U[30, 90] deg, traced with
dt = 0.01 and the usual cutoffs.  `scale` divides the image sides (for small
parity runs); the draws themselves do not depend on it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BATCH_SEED = 20231015
SIDES = (128, 256, 384, 512)


@dataclass(frozen=True)
class Instance:
    M: float
    a: float
    Q: float
    r0: float
    theta0: float
    phi0: float
    fov: float
    width: int
    height: int


def batch_instances(n: int = 256, seed: int = BATCH_SEED, scale: int = 1) -> list[Instance]:
    rng = np.random.default_rng(seed)
    out = []
    M = 0.5
    for _ in range(n):
        a = rng.uniform(0.0, 0.49)
        Q = rng.uniform(0.0, math.sqrt(M * M - a * a) * 0.95)
        r0 = rng.uniform(10.0, 50.0)
        th0 = math.radians(rng.uniform(5.0, 90.0))
        side = int(SIDES[rng.integers(0, len(SIDES))])
        fov = math.radians(rng.uniform(30.0, 90.0))
        s = max(1, side // scale)
        out.append(Instance(M, float(a), float(Q), float(r0), th0, 0.0, fov, s, s))
    return out


def kerr_newman_frame(f32_params: bool = True, width: int = 1000, height: int = 1000):
    """The 1000x1000 Kerr-Newman frame: M=0.5, a=0.24, Q=0.3, r0=20,
    theta0=80 deg, fov 75 deg (parameters rounded to binary32 when asked)."""
    deg = math.pi / 180.0
    vals = dict(M=0.5, a=0.24, Q=0.3, r0=20.0, theta0=80 * deg, phi0=0.0, fov=75 * deg)
    if f32_params:
        vals = {k: float(np.float32(v)) for k, v in vals.items()}
    return Instance(width=width, height=height, **vals)


def sky_texture(width: int, height: int, seed: int = 7) -> np.ndarray:
    """A seeded synthetic equirectangular sky (height x width 32-bit texels,
    bytes R, G, B, A): smooth colour gradients across the sphere with seeded
    random stars, standing in for the paper's panorama (not available)."""
    rng = np.random.default_rng(seed)
    j, i = np.meshgrid(np.arange(height), np.arange(width), indexing="ij")
    r = (40 + 80 * (i / max(width - 1, 1))).astype(np.int64)
    gch = (30 + 120 * (j / max(height - 1, 1))).astype(np.int64)
    b = (60 + 60 * ((i + 2 * j) % 64) / 63).astype(np.int64)
    stars = rng.random((height, width)) < 0.02
    bright = rng.integers(150, 256, (height, width))
    r, gch, b = (np.where(stars, bright, c) for c in (r, gch, b))
    return (r | (gch << 8) | (b << 16) | (255 << 24)).astype(np.uint32)
