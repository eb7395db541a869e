"""Two-galaxy encounter with the particle numbers of the paper's merger test (Sect.
4.2.2): two galaxies of 10^5 halo particles, 2 x 10^4 star particles and one
central black hole each (240,002 bodies), mass ratio 1:3, on a parabolic orbit.
The paper's initial conditions are not available; this recipe stands in for them.

Recipe (G = 1):

* each galaxy is ``galaxy.galaxy`` (disk : bulge : halo = 1 : 0.3 : 10) with the
  2 x 10^4 star particles split between disk and bulge in their mass ratio
  (15,385 and 4,615), plus a black hole of 0.1% of the galaxy's mass at rest at
  its centre; the primary has mass 1 (plus its hole);
* the secondary is the same model with mass 1/3, lengths and velocities scaled
  by (1/3)^(1/3) (the same mean density), its disk tilted by 60 degrees about the
  x axis; drawn with its own seed;
* the two centres of mass start ``d0`` apart (default 40, outside both truncated
  halos) on the parabolic two-body orbit of point masses with pericentre ``rp``
  (default 4, four disk scale lengths), in the orbit's (x, y) plane, with the
  system's centre of mass at rest at the origin.
"""

import numpy as np

from .galaxy import galaxy

N_HALO, N_STARS = 100_000, 20_000
N_DISK = 15_385
N_BULGE = N_STARS - N_DISK
BH_FRACTION = 1e-3


def _model(seed, scale_mass, tilt):
    pos, vel, mass = galaxy(n_disk=N_DISK, n_bulge=N_BULGE, n_halo=N_HALO, seed=seed)
    s = scale_mass ** (1.0 / 3.0)
    pos = pos * s
    vel = vel * s
    mass = mass * scale_mass
    if tilt:
        c, sn = np.cos(tilt), np.sin(tilt)
        rot = np.array([[1.0, 0.0, 0.0], [0.0, c, -sn], [0.0, sn, c]])
        pos = pos @ rot.T
        vel = vel @ rot.T
    pos = np.concatenate([pos, np.zeros((1, 3))])
    vel = np.concatenate([vel, np.zeros((1, 3))])
    mass = np.concatenate([mass, [BH_FRACTION * scale_mass]])
    return pos, vel, mass


def parabolic_orbit(m1, m2, d0, rp):
    """Relative position and velocity (of body 2 with respect to body 1) at
    separation d0 on the approaching branch of the parabolic orbit with
    pericentre rp, in the (x, y) plane."""
    M = m1 + m2
    v = np.sqrt(2.0 * M / d0)                 # parabolic: zero orbital energy
    vt = np.sqrt(2.0 * M * rp) / d0           # angular momentum rp * v_peri over d0
    vr = -np.sqrt(max(v * v - vt * vt, 0.0))  # approaching
    r = np.array([d0, 0.0, 0.0])
    u = np.array([vr, vt, 0.0])
    return r, u


def merger(seed=6, d0=40.0, rp=4.0):
    """Return (pos, vel, mass) float64 arrays of the encounter (primary first)."""
    pa, va, ma = _model(seed, 1.0, 0.0)
    pb, vb, mb = _model(seed + 1, 1.0 / 3.0, np.pi / 3.0)
    Ma, Mb = ma.sum(), mb.sum()
    r, u = parabolic_orbit(Ma, Mb, d0, rp)
    M = Ma + Mb
    pa = pa - (Mb / M) * r
    va = va - (Mb / M) * u
    pb = pb + (Ma / M) * r
    vb = vb + (Ma / M) * u
    pos = np.concatenate([pa, pb])
    vel = np.concatenate([va, vb])
    mass = np.concatenate([ma, mb])
    return (np.ascontiguousarray(pos), np.ascontiguousarray(vel), np.ascontiguousarray(mass))


def black_holes(n_total=2 * (N_HALO + N_STARS + 1)):
    """Indices of the two black holes in the arrays ``merger`` returns."""
    half = n_total // 2
    return np.array([half - 1, n_total - 1])
