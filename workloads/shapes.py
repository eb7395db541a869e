"""Small structured particle sets for edge cases: two bodies, coincident points, a
line, a lattice, tight clusters and a uniform cube. Each returns (pos, vel, mass) as
float64 arrays; velocities are zero unless stated.
"""

import numpy as np


def _pack(pos, mass=None):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n = pos.shape[0]
    if mass is None:
        mass = np.full(n, 1.0 / n)
    return pos, np.zeros_like(pos), np.ascontiguousarray(mass, dtype=np.float64)


def two_body(sep=1.0, m1=0.5, m2=0.5):
    pos = np.array([[-0.5 * sep, 0.0, 0.0], [0.5 * sep, 0.0, 0.0]])
    return _pack(pos, np.array([m1, m2]))


def coincident(n, point=(0.25, -0.5, 1.0)):
    pos = np.tile(np.asarray(point, dtype=np.float64), (n, 1))
    return _pack(pos)


def on_a_line(n, seed=0):
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(-1.0, 1.0, n))
    pos = np.stack([t, 0.5 * t, np.zeros(n)], axis=1)
    return _pack(pos)


def lattice(k, spacing=1.0):
    g = np.arange(k, dtype=np.float64) * spacing
    xx, yy, zz = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    return _pack(pos)


def clustered(n, seed=0, nclusters=7, width=1e-3):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-1.0, 1.0, (nclusters, 3))
    which = rng.integers(0, nclusters, n)
    pos = centres[which] + width * rng.standard_normal((n, 3))
    mass = rng.uniform(0.5, 1.5, n)
    mass /= mass.sum()
    return _pack(pos, mass)


def uniform_cube(n, seed=0, side=1.0):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, side, (n, 3))
    mass = rng.uniform(0.5, 1.5, n)
    mass /= mass.sum()
    return _pack(pos, mass)
