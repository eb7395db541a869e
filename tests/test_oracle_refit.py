"""Pins of the oracle's multipole-only update (Sect. 5: between rebuilds only the
moments of the cells whose particles moved are recomputed; the walk of a refitted
tree slows down because the cells' size l grows, so a refit also grows each
cell's side to the extent of its particles)."""

import numpy as np
import pytest

import oracle
import workloads


def _moments(t):
    mo = t.moments()
    return mo["mass"], mo["com"], mo["S"]


def test_refit_at_the_build_positions_changes_nothing():
    pos, _, m = workloads.plummer(3000, 31)
    t = oracle.Tree(pos, m)
    M0, c0, S0 = _moments(t)
    g0 = t.groups()
    r0, _ = t.rcrit(0.6)
    t.refit(pos)
    M1, c1, S1 = _moments(t)
    g1 = t.groups()
    r1, _ = t.rcrit(0.6)
    assert np.array_equal(M0, M1) and np.array_equal(c0, c1) and np.array_equal(S0, S1)
    assert np.array_equal(g0["centre"], g1["centre"]) and np.array_equal(g0["half"], g1["half"])
    assert np.array_equal(r0, r1)


def _grown_rcrit2(t, pos, theta):
    """Eq. (1) radius of every cell with the side grown to its particles' extent,
    from the exported cells, domain and sorted positions."""
    c = t.cells()
    perm, _ = t.order()
    x = pos[perm]
    lo, L, _ = t.domain()
    l = L * np.ldexp(1.0, -c["level"].astype(np.int64))
    ext = np.zeros(t.ncells)
    for i in range(t.ncells):
        p = x[c["first"][i]:c["first"][i] + c["count"][i]]
        ext[i] = (p.max(axis=0) - p.min(axis=0)).max()
    side = np.maximum(l, ext)
    _, centre = t.rcrit(theta)
    d = t.moments()["com"] - centre
    delta = np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
    r = side / np.float64(np.float32(theta)) + delta
    return (r * r).astype(np.float32), side, l


@pytest.mark.parametrize("dt", [1 / 64, 1 / 8])
def test_refit_grows_the_cell_side_to_the_particles_extent(dt):
    pos, vel, m = workloads.plummer(4000, 36)
    t = oracle.Tree(pos, m)
    new = pos + vel * dt
    t.refit(new)
    want, side, l = _grown_rcrit2(t, new, 0.7)
    got, _ = t.rcrit(0.7)
    assert np.array_equal(got, want)
    assert np.any(side > l)            # some cells have spread beyond their cube
    if dt >= 1 / 8:
        # the refitted tree's walk is costlier than a fresh build's (Sect. 5)
        fresh = oracle.Tree(new, m)
        npp0, npc0 = fresh.walk_counts(0.7)
        npp1, npc1 = t.walk_counts(0.7)
        i0 = (fresh.groups()["count"] * (npp0 + npc0)).sum()
        i1 = (t.groups()["count"] * (npp1 + npc1)).sum()
        assert i1 > 1.2 * i0


def test_refit_side_of_a_spread_system():
    # positions scaled by 3 about the first particle: every cell holding two or
    # more distinct points now spans three times its former extent
    pos, _, m = workloads.plummer(1500, 37)
    t = oracle.Tree(pos, m)
    new = pos[0] + 3.0 * (pos - pos[0])
    t.refit(new)
    _, side, l = _grown_rcrit2(t, new, 0.5)
    c = t.cells()
    perm, _ = t.order()
    x = pos[perm]
    grown = 0
    for i in range(t.ncells):
        p = x[c["first"][i]:c["first"][i] + c["count"][i]]
        e = (p.max(axis=0) - p.min(axis=0)).max()
        assert side[i] >= 3.0 * e * (1 - 1e-9)
        if 3.0 * e * (1 + 1e-9) < l[i]:
            assert side[i] == l[i]
        else:
            grown += 1
    assert grown > t.ncells // 10


def test_refit_equals_a_fresh_build_with_the_same_cells():
    # move every particle inside its own integer key cell, keeping the particles
    # that set the domain's extremes fixed: a fresh build then has the same keys,
    # order, cells and groups, and its moments must equal the refit's bit for bit
    pos, _, m = workloads.plummer(5000, 32)
    t = oracle.Tree(pos, m, 8, 32)
    lo, L, scale = t.domain()
    q = np.floor((pos - lo) * scale)
    rng = np.random.default_rng(33)
    new = lo + (q + rng.uniform(0.05, 0.95, pos.shape)) / scale
    ext = np.concatenate([np.argmin(pos, axis=0), np.argmax(pos, axis=0)])
    new[ext] = pos[ext]
    fresh = oracle.Tree(new, m, 8, 32)
    assert np.array_equal(fresh.order()[1], t.order()[1])      # same keys
    for k in ("first", "count", "level", "child", "nchild"):
        assert np.array_equal(fresh.cells()[k], t.cells()[k])
    t.refit(new)
    for a, b in zip(_moments(t), _moments(fresh)):
        assert np.array_equal(a, b)
    gt, gf = t.groups(), fresh.groups()
    assert np.array_equal(gt["centre"], gf["centre"]) and np.array_equal(gt["half"], gf["half"])
    assert np.array_equal(t.walk_counts(0.6)[0], fresh.walk_counts(0.6)[0])


def test_refit_moves_only_the_ancestors_of_a_moved_particle():
    pos, _, m = workloads.plummer(4000, 34)
    t = oracle.Tree(pos, m)
    M0, c0, S0 = _moments(t)
    perm, _ = t.order()
    cells = t.cells()
    j = 1234                                   # caller index of the moved particle
    sj = int(np.nonzero(perm == j)[0][0])      # its sorted position
    new = pos.copy()
    new[j] += 1e-3
    t.refit(new)
    M1, c1, S1 = _moments(t)
    holds = (cells["first"] <= sj) & (sj < cells["first"] + cells["count"])
    assert np.array_equal(M0, M1)              # masses never change
    assert np.array_equal(c0[~holds], c1[~holds]) and np.array_equal(S0[~holds], S1[~holds])
    assert np.all(np.any(c0[holds] != c1[holds], axis=1))
    # the root's centre of mass moved by m_j * shift / M
    assert c1[0] == pytest.approx(c0[0] + m[j] * 1e-3 / m.sum(), abs=1e-15)


def test_refit_translation_shifts_centres_and_keeps_second_moments():
    pos, _, m = workloads.plummer(2000, 35)
    t = oracle.Tree(pos, m)
    M0, c0, S0 = _moments(t)
    shift = np.array([0.25, -0.5, 0.125])     # exact binary fractions
    t.refit(pos + shift)
    M1, c1, S1 = _moments(t)
    assert np.allclose(c1, c0 + shift, rtol=0, atol=1e-14)
    scale = np.abs(S0).max(axis=1, keepdims=True) + 1e-300
    # (a one-particle cell keeps S = 0 up to the rounding of its shifted centre)
    assert np.all(np.abs(S1 - S0) <= 1e-10 * scale + 1e-18)


def test_refit_rejects_non_finite_positions():
    pos, _, m = workloads.plummer(500, 36)
    t = oracle.Tree(pos, m)
    bad = pos.copy()
    bad[7, 1] = np.inf
    with pytest.raises(ValueError):
        t.refit(bad)
    M0, c0, _ = _moments(t)
    assert np.all(np.isfinite(c0))
