"""Three-component model galaxy: exponential disk with sech^2 vertical profile, a
Hernquist bulge and a truncated NFW halo (G = 1).

Stands in for the shape of the paper's production runs (a galaxy merger of disk,
bulge and halo particles, Sect. 4.2.2), whose initial conditions are not available.

Recipe (all draws from one seeded generator):

* masses disk : bulge : halo = 1 : 0.3 : 10, total 1; particles within a component
  have equal mass;
* disk: cylindrical radius from the exponential-disk enclosed-mass fraction
  1 - (1 + R/Rd) exp(-R/Rd) (Rd = 1, inverted by bisection), height
  z = z0 atanh(2u - 1) (sech^2 profile, z0 = 0.1), uniform azimuth;
* bulge: Hernquist radius r = a sqrt(X) / (1 - sqrt(X)), X ~ U(0, 0.99), a = 0.2;
* halo: NFW with scale radius r200 / c (r200 = 20, c = 10), truncated at r200, radius
  from the enclosed-mass fraction ln(1+x) - x/(1+x) (bisection);
* velocities: disk particles on circular orbits of the spherically averaged
  enclosed mass with 10% Gaussian dispersion; bulge and halo particles isotropic
  Gaussian with the dispersion of the isotropic Jeans equation of their own density
  in the total enclosed mass (numerical integral on a radial grid);
* centre of mass and mean velocity removed.
"""

import numpy as np

DISK_MASS, BULGE_MASS, HALO_MASS = 1.0, 0.3, 10.0


def _bisect(cdf, target, lo, hi, iters=60):
    lo = np.full_like(target, lo)
    hi = np.full_like(target, hi)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        below = cdf(mid) < target
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
    return 0.5 * (lo + hi)


def _isotropic(rng, n):
    cz = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([sz * np.cos(ph), sz * np.sin(ph), cz], axis=1)


def _jeans_sigma(r_grid, rho, menc):
    """sigma^2(r) = 1/rho(r) * int_r^inf rho(s) M(s) / s^2 ds (isotropic, G = 1)."""
    f = rho * menc / r_grid ** 2
    # cumulative trapezoid from the outer edge inwards
    seg = 0.5 * (f[1:] + f[:-1]) * np.diff(r_grid)
    tail = np.concatenate([np.cumsum(seg[::-1])[::-1], [0.0]])
    return np.sqrt(np.maximum(tail / np.maximum(rho, 1e-300), 0.0))


def galaxy(n_disk=1 << 20, n_bulge=1 << 19, n_halo=5 * (1 << 19), seed=3,
           rd=1.0, z0=0.1, a_bulge=0.2, r200=20.0, conc=10.0):
    """Return (pos, vel, mass) float64 arrays for the model galaxy."""
    rng = np.random.default_rng(seed)
    tot = DISK_MASS + BULGE_MASS + HALO_MASS
    md, mb, mh = DISK_MASS / tot, BULGE_MASS / tot, HALO_MASS / tot
    rs = r200 / conc

    # disk
    u = rng.uniform(0.0, 1.0 - 1e-12, n_disk)
    R = _bisect(lambda x: 1.0 - (1.0 + x / rd) * np.exp(-x / rd), u, 0.0, 60.0 * rd)
    z = z0 * np.arctanh(np.clip(2.0 * rng.uniform(0.0, 1.0, n_disk) - 1.0, -1 + 1e-12, 1 - 1e-12))
    phd = rng.uniform(0.0, 2.0 * np.pi, n_disk)
    pd = np.stack([R * np.cos(phd), R * np.sin(phd), z], axis=1)

    # bulge
    sx = np.sqrt(rng.uniform(0.0, 0.99, n_bulge))
    rb = a_bulge * sx / (1.0 - sx)
    pb = rb[:, None] * _isotropic(rng, n_bulge)

    # halo
    m_nfw = lambda x: np.log1p(x) - x / (1.0 + x)
    uh = rng.uniform(0.0, 1.0, n_halo) * m_nfw(conc)
    xh = _bisect(m_nfw, uh, 0.0, conc)
    rh = xh * rs
    ph = rh[:, None] * _isotropic(rng, n_halo)

    pos = np.concatenate([pd, pb, ph])
    mass = np.concatenate([np.full(n_disk, md / n_disk), np.full(n_bulge, mb / n_bulge),
                           np.full(n_halo, mh / n_halo)])

    # spherically averaged enclosed mass on a radial grid
    r_all = np.linalg.norm(pos, axis=1)
    grid = np.geomspace(1e-4, 1.5 * r_all.max(), 4000)
    order = np.argsort(r_all)
    cm = np.cumsum(mass[order])
    menc = np.interp(grid, r_all[order], cm, left=0.0, right=cm[-1])

    def menc_at(r):
        return np.interp(r, grid, menc)

    # disk: circular speed with 10% dispersion
    vc = np.sqrt(menc_at(R) / np.maximum(R, 1e-6))
    vd = np.stack([-vc * np.sin(phd), vc * np.cos(phd), np.zeros(n_disk)], axis=1)
    vd += 0.1 * vc[:, None] * rng.standard_normal((n_disk, 3))

    # spheroids: isotropic Jeans dispersion of their own density profiles
    rho_b = a_bulge / (2 * np.pi) / (grid * (grid + a_bulge) ** 3)
    xg = grid / rs
    rho_h = np.where(grid <= r200, 1.0 / (xg * (1.0 + xg) ** 2), 1e-300)
    sig_b = np.interp(rb, grid, _jeans_sigma(grid, rho_b, menc))
    sig_h = np.interp(rh, grid, _jeans_sigma(grid, rho_h, menc))
    vb = sig_b[:, None] * rng.standard_normal((n_bulge, 3))
    vh = sig_h[:, None] * rng.standard_normal((n_halo, 3))
    vel = np.concatenate([vd, vb, vh])

    msum = mass.sum()
    pos -= (mass[:, None] * pos).sum(axis=0) / msum
    vel -= (mass[:, None] * vel).sum(axis=0) / msum
    return (np.ascontiguousarray(pos), np.ascontiguousarray(vel), np.ascontiguousarray(mass))
