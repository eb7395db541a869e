"""Generators against the closed forms of the models they sample."""

import numpy as np
import pytest

import workloads


def test_galaxy_components_follow_their_profiles():
    nd, nb, nh = 40_000, 20_000, 100_000
    pos, vel, m = workloads.galaxy(nd, nb, nh, seed=3)
    assert pos.shape == (nd + nb + nh, 3) and m.sum() == pytest.approx(1.0)
    tot = 11.3
    assert m[:nd].sum() == pytest.approx(1 / tot) and m[nd:nd + nb].sum() == pytest.approx(0.3 / tot)
    # component positions are drawn before the centre-of-mass shift; the shift is tiny
    d, b, h = pos[:nd], pos[nd:nd + nb], pos[nd + nb:]
    R = np.hypot(d[:, 0], d[:, 1])
    for r0 in (0.5, 1.0, 2.0, 4.0):        # exponential disk, scale length 1
        assert np.mean(R < r0) == pytest.approx(1 - (1 + r0) * np.exp(-r0), abs=0.01)
    for z0 in (0.05, 0.1, 0.2):            # sech^2 layer, z0 = 0.1
        assert np.mean(np.abs(d[:, 2]) < z0) == pytest.approx(np.tanh(z0 / 0.1), abs=0.01)
    rb = np.linalg.norm(b, axis=1)
    for r0 in (0.1, 0.2, 0.5):             # Hernquist a = 0.2, truncated at 99% of the mass
        assert np.mean(rb < r0) == pytest.approx((r0 / (r0 + 0.2)) ** 2 / 0.99, abs=0.01)
    rh = np.linalg.norm(h, axis=1)
    mn = lambda x: np.log1p(x) - x / (1 + x)
    for r0 in (1.0, 2.0, 5.0, 10.0):       # NFW rs = 2 truncated at 20
        assert np.mean(rh < r0) == pytest.approx(mn(r0 / 2) / mn(10), abs=0.01)
    assert rh.max() <= 20.05          # truncation radius, up to the centre-of-mass shift
    # disk rotates, spheroids do not
    vphi = (d[:, 0] * vel[:nd, 1] - d[:, 1] * vel[:nd, 0]) / R
    assert np.median(vphi) > 0.1
    assert abs(np.mean(vel[nd + nb:, 0])) < 0.05


def test_plummer_is_seeded_and_reproducible():
    a = workloads.plummer(1000, 4)
    b = workloads.plummer(1000, 4)
    c = workloads.plummer(1000, 5)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not np.array_equal(a[0], c[0])


def test_hernquist_follows_its_mass_profile():
    pos, vel, m = workloads.hernquist(200_000, 9, a=1.0)
    assert m.sum() == pytest.approx(1.0)
    r = np.linalg.norm(pos, axis=1)
    for r0 in (0.3, 1.0, 3.0, 10.0):      # M(<r) = r^2 / (r + a)^2, truncated at 99%
        assert np.mean(r < r0) == pytest.approx((r0 / (r0 + 1.0)) ** 2 / 0.99, abs=0.01)
    # isotropic Jeans dispersions: virial ratio 2T/|W| near 1 for the whole sphere
    # (truncation and sampling noise allowed); W from the analytic potential energy
    # -1/(6a) of the untruncated model
    T = 0.5 * np.sum(m * np.sum(vel * vel, axis=1))
    assert 2 * T / (1.0 / 6.0) == pytest.approx(1.0, abs=0.1)


def test_cluster_batch_sizes_and_softening():
    sizes = workloads.cluster_sizes(512, 4)
    assert sizes.min() >= 1024 and sizes.max() < 65536
    # log-uniform: E[N] = (65536 - 1024) / ln 64 = 15,512
    assert sizes.mean() == pytest.approx(15512, rel=0.15)
    b = workloads.cluster_batch(8, 4)
    assert [q["n"] for q in b] == list(sizes[:8])
    for q in b:
        assert q["pos"].shape == (q["n"], 3) and q["theta"] == 0.75
        assert q["eps"] == pytest.approx(0.04 * q["n"] ** (-1 / 3))
    # clusters are independent draws
    assert not np.array_equal(b[0]["pos"][:10], b[1]["pos"][:10])


def test_request_trace_is_poisson():
    tr = workloads.request_trace(4000, 200.0, 5)
    t = np.array([q["arrival"] for q in tr])
    gaps = np.diff(t)
    assert np.all(gaps > 0)
    assert gaps.mean() == pytest.approx(1 / 200, rel=0.05)
    assert np.std(gaps) == pytest.approx(1 / 200, rel=0.1)       # exponential: sd = mean
    n = np.array([q["n"] for q in tr])
    assert n.min() >= 1024 and n.max() <= 2097152
    assert np.mean(np.log(n)) == pytest.approx((np.log(1024) + np.log(2097152)) / 2, rel=0.02)
    assert {q["shape"] for q in tr} == {"plummer", "hernquist"}
    assert {q["theta"] for q in tr} == {0.5, 0.75}


def test_merger_recipe():
    # two galaxies of 10^5 halo + 2 x 10^4 star particles + one black hole each
    # (the paper's 240,002 bodies), mass ratio 1:3, parabolic orbit of the two
    # centres of mass with the requested pericentre, whole system at rest
    pos, vel, mass = workloads.merger(seed=6, d0=40.0, rp=4.0)
    n = pos.shape[0]
    assert n == 240_002 and vel.shape == (n, 3) and mass.shape == (n,)
    half = n // 2
    a, b = slice(0, half), slice(half, n)
    Ma, Mb = mass[a].sum(), mass[b].sum()
    assert Mb / Ma == pytest.approx(1.0 / 3.0, rel=1e-12)
    M = Ma + Mb
    assert np.allclose((mass[:, None] * pos).sum(axis=0) / M, 0.0, atol=1e-12)
    assert np.allclose((mass[:, None] * vel).sum(axis=0) / M, 0.0, atol=1e-12)
    ca = (mass[a, None] * pos[a]).sum(axis=0) / Ma
    cb = (mass[b, None] * pos[b]).sum(axis=0) / Mb
    ua = (mass[a, None] * vel[a]).sum(axis=0) / Ma
    ub = (mass[b, None] * vel[b]).sum(axis=0) / Mb
    bh = workloads.black_holes(n)
    assert np.allclose(pos[bh[0]], ca, atol=1e-9) and np.allclose(pos[bh[1]], cb, atol=1e-9)
    r, u = cb - ca, ub - ua
    assert np.linalg.norm(r) == pytest.approx(40.0, rel=1e-9)
    # zero orbital energy and pericentre L^2 / (2 M) of a parabola
    assert 0.5 * u @ u - M / np.linalg.norm(r) == pytest.approx(0.0, abs=1e-9)
    L = np.linalg.norm(np.cross(r, u))
    assert L * L / (2.0 * M) == pytest.approx(4.0, rel=1e-9)
    assert r @ u < 0                                   # approaching
    # each black hole holds 0.1% of its galaxy's particle mass
    assert mass[bh[0]] == pytest.approx(1e-3 * (Ma - mass[bh[0]]), rel=1e-9)
    assert mass[bh[1]] == pytest.approx(1e-3 * (Mb - mass[bh[1]]), rel=1e-9)
