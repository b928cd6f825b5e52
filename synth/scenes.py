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


def shells_in_gas(rng, side=2.0e-3, r_big=3.0e-4, r_small=4.0e-5, shell_n=100, n_gas=3000, overlap=1e-7):
    """Two large spheres, each carrying a shell of shell_n small spheres that
    touch it (Fibonacci points, overlap `overlap`), in a gas of n_gas small
    spheres placed by rejection sampling.  The large spheres have rows of more
    than shell_n partners and the binning cells (sized by the large radius)
    hold many small spheres: the crowded corners of the neighbour search."""
    centres = np.array([[0.3 * side, 0.5 * side, 0.5 * side], [0.7 * side, 0.5 * side, 0.5 * side]])
    xs, rs = [c for c in centres], [r_big, r_big]
    k = np.arange(shell_n) + 0.5
    phi = np.arccos(1.0 - 2.0 * k / shell_n)
    th = math.pi * (1.0 + 5.0 ** 0.5) * k
    u = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], axis=1)
    for c in centres:
        for e in u:
            xs.append(c + (r_big + r_small - overlap) * e)
            rs.append(r_small)
    x = np.array(xs)
    r = np.array(rs)
    placed = 0
    gas = []
    while placed < n_gas:
        p = rng.uniform(r_small, side - r_small, 3)
        allx = np.vstack([x] + gas) if gas else x
        allr = np.concatenate([r, np.full(len(gas), r_small)])
        if np.all(np.linalg.norm(allx - p, axis=1) > allr + r_small + 1e-6):
            gas.append(p[None, :])
            placed += 1
    x = np.vstack([x] + gas)
    r = np.concatenate([r, np.full(n_gas, r_small)])
    return x, r
