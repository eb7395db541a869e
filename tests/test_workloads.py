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
