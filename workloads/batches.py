"""Seeded inputs for the batched and served forms of the tree-code: many small
independent systems evaluated together, and a trace of arriving requests.

Recipes (inputs only; none of the method's arithmetic):

* cluster batch: k Plummer spheres (AHW74, Henon units); sizes
  N_i = floor(exp(U(ln nmin, ln nmax))) from default_rng(seed); cluster i is drawn
  from the i-th child of SeedSequence(seed); softening eps_i = 0.04 N_i^(-1/3);
  opening angle 0.75;
* Hernquist sphere (total mass 1, scale a): radius r = a sqrt(X) / (1 - sqrt(X)),
  X ~ U(0, xmax), the inverse of M(<r) = r^2 / (r + a)^2; isotropic Gaussian
  velocities with the dispersion of the isotropic Jeans equation (numerical
  integral on a radial grid); centre of mass and mean velocity removed;
* request trace: Poisson arrivals at a given rate; each request is a Plummer or
  Hernquist sphere (even odds), N log-uniform in [nmin, nmax], opening angle 0.5
  or 0.75 (even odds), softening 0.01, one force evaluation plus a number of
  leapfrog steps of dt = 1/128.
"""

import numpy as np

from .plummer import plummer


def cluster_sizes(k, seed, nmin=1024, nmax=65536):
    rng = np.random.default_rng(seed)
    return np.floor(np.exp(rng.uniform(np.log(nmin), np.log(nmax), k))).astype(np.int64)


def cluster_batch(k=512, seed=4, nmin=1024, nmax=65536, theta=0.75):
    """List of k dicts: pos, vel, mass, n, eps, theta."""
    sizes = cluster_sizes(k, seed, nmin, nmax)
    seeds = np.random.SeedSequence(seed).spawn(k)
    out = []
    for n, ss in zip(sizes, seeds):
        n = int(n)
        pos, vel, mass = plummer(n, int(ss.generate_state(1)[0]))
        out.append(dict(pos=pos, vel=vel, mass=mass, n=n, eps=0.04 * n ** (-1.0 / 3.0),
                        theta=theta))
    return out


def _isotropic(rng, n):
    cz = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([sz * np.cos(ph), sz * np.sin(ph), cz], axis=1)


def hernquist(n, seed, a=1.0, xmax=0.99):
    """Return (pos, vel, mass) for an n-body Hernquist sphere (G = M = 1)."""
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.default_rng(seed)
    sx = np.sqrt(rng.uniform(0.0, xmax, n))
    r = a * sx / (1.0 - sx)
    pos = r[:, None] * _isotropic(rng, n)
    # isotropic Jeans: sigma^2(r) = 1/rho int_r^inf rho M / s^2 ds
    grid = np.geomspace(1e-4 * a, 1e4 * a, 4000)
    rho = a / (2 * np.pi) / (grid * (grid + a) ** 3)
    menc = grid ** 2 / (grid + a) ** 2
    f = rho * menc / grid ** 2
    seg = 0.5 * (f[1:] + f[:-1]) * np.diff(grid)
    tail = np.concatenate([np.cumsum(seg[::-1])[::-1], [0.0]])
    sig = np.sqrt(np.maximum(tail / rho, 0.0))
    vel = np.interp(r, grid, sig)[:, None] * rng.standard_normal((n, 3))
    mass = np.full(n, 1.0 / n)
    pos -= pos.mean(axis=0)
    vel -= vel.mean(axis=0)
    return np.ascontiguousarray(pos), np.ascontiguousarray(vel), mass


def request_trace(count=2000, rate=200.0, seed=5, nmin=1024, nmax=2097152, steps=10):
    """Arrival times (s) and request descriptions of a Poisson trace."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    n = np.floor(np.exp(rng.uniform(np.log(nmin), np.log(nmax), count))).astype(np.int64)
    shape = np.where(rng.uniform(size=count) < 0.5, "plummer", "hernquist")
    theta = np.where(rng.uniform(size=count) < 0.5, 0.5, 0.75)
    seeds = rng.integers(0, 2 ** 31, count)
    return [dict(arrival=float(t[i]), n=int(n[i]), shape=str(shape[i]), theta=float(theta[i]),
                 eps=0.01, dt=1.0 / 128, steps=int(steps), seed=int(seeds[i]))
            for i in range(count)]
