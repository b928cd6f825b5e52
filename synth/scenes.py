"""Tiny hand-built scenes shared by the oracle pins and the GPU parity tests.

Pure input construction (positions, radii, velocities, walls); no contact,
drag or integration arithmetic.
"""
import math

import numpy as np

from . import MATERIAL, WALL_PLANE


def material(**kw):
    m = dict(MATERIAL)
    m.update(kw)
    return m


def two_spheres(r1, r2, gap, speed, axis=(1.0, 0.0, 0.0), offset=(0.0, 0.0, 0.0)):
    """Sphere 0 at the origin, sphere 1 along `axis` at distance r1 + r2 + gap;
    they approach each other with relative speed `speed` (split by mass)."""
    ax = np.asarray(axis, dtype=np.float64)
    ax = ax / np.linalg.norm(ax)
    x = np.zeros((2, 3))
    x[1] = ax * (r1 + r2 + gap)
    x += np.asarray(offset)
    m1, m2 = r1 ** 3, r2 ** 3
    v = np.zeros((2, 3))
    v[0] = ax * speed * m2 / (m1 + m2)
    v[1] = -ax * speed * m1 / (m1 + m2)
    return x, np.array([r1, r2]), v


def random_gas(rng, n, side, rmin, rmax, vmax):
    """n non-overlapping spheres at random positions in a cube (rejection
    sampling) with random velocities: a dilute collision test."""
    r = rng.uniform(rmin, rmax, n)
    x = np.zeros((n, 3))
    for i in range(n):
        for _ in range(10000):
            p = rng.uniform(rmax, side - rmax, 3)
            if i == 0 or np.all(np.linalg.norm(x[:i] - p, axis=1) > r[:i] + r[i]):
                x[i] = p
                break
        else:
            raise ValueError("cube too small for a dilute gas")
    v = rng.uniform(-vmax, vmax, (n, 3))
    return x, r, v


def plane(normal, offset):
    nrm = np.asarray(normal, dtype=np.float64)
    nrm = nrm / np.linalg.norm(nrm)
    return (WALL_PLANE, (nrm[0], nrm[1], nrm[2], offset))


def incline_gravity(theta, g=9.81):
    """Gravity for a floor z = 0 tilted by theta about y: the slope points +x."""
    return (g * math.sin(theta), 0.0, -g * math.cos(theta))
