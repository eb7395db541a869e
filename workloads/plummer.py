"""Plummer sphere initial conditions (Aarseth, Henon & Wielen 1974 sampling).

The paper's performance and accuracy measurements (Sect. 4.1, 4.2.1) use Plummer
spheres of N = 2^15 ... 2^24 equal-mass particles. The paper does not say how its
spheres were drawn; this is the standard inverse-CDF recipe in Henon units
(G = M = 1, total energy -1/4):

* cumulative mass fraction X ~ U(0, xmax) with xmax = 0.999, radius
  r = (X^(-2/3) - 1)^(-1/2) in units of the Plummer scale length;
* isotropic direction;
* speed q * v_esc with v_esc = sqrt(2) (1 + r^2)^(-1/4) and q drawn by rejection
  from g(q) = q^2 (1 - q^2)^(7/2) (its maximum is below 0.1);
* positions scaled by 3 pi / 16 and velocities by sqrt(16 / (3 pi)) to Henon units;
* centre of mass and mean velocity removed.
"""

import numpy as np

_LEN = 3.0 * np.pi / 16.0
_VEL = np.sqrt(16.0 / (3.0 * np.pi))


def _isotropic(rng, n):
    cz = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([sz * np.cos(ph), sz * np.sin(ph), cz], axis=1)


def plummer_radii(rng, n, xmax=0.999):
    x = rng.uniform(0.0, xmax, n)
    # guard the (measure-zero) draw x == 0
    x = np.maximum(x, 1e-300)
    return 1.0 / np.sqrt(x ** (-2.0 / 3.0) - 1.0)


def _speed_fraction(rng, n):
    out = np.empty(n)
    filled = 0
    while filled < n:
        want = max(1024, int(1.2 * (n - filled) / 0.2) + 16)
        q = rng.uniform(0.0, 1.0, want)
        y = rng.uniform(0.0, 0.1, want)
        ok = q[y < q * q * (1.0 - q * q) ** 3.5]
        take = min(ok.size, n - filled)
        out[filled:filled + take] = ok[:take]
        filled += take
    return out


def plummer(n, seed, xmax=0.999):
    """Return (pos, vel, mass) for an n-body Plummer sphere in Henon units."""
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = np.random.default_rng(seed)
    r = plummer_radii(rng, n, xmax)
    pos = r[:, None] * _isotropic(rng, n)
    q = _speed_fraction(rng, n)
    v = q * np.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    vel = v[:, None] * _isotropic(rng, n)
    pos *= _LEN
    vel *= _VEL
    mass = np.full(n, 1.0 / n)
    pos -= pos.mean(axis=0)
    vel -= vel.mean(axis=0)
    return (np.ascontiguousarray(pos, dtype=np.float64),
            np.ascontiguousarray(vel, dtype=np.float64),
            mass)
