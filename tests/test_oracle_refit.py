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


def _refit_geometry(t, build_pos, pos):
    """Side and centre of every cell's opening test after a refit to pos, from
    the exported cells and domain and the build positions: a cell whose particles
    all keep their key cell (inside the build's bounding box, same integer
    coordinates at the cell's level) keeps its cube of side L 2^-level about the
    geometric centre; any other cell takes its particles' tight box (its centre,
    side max(L 2^-level, largest extent))."""
    c = t.cells()
    perm, _ = t.order()
    x0 = build_pos[perm]
    x = pos[perm]
    lo, L, scale = t.domain()
    hi = build_pos.max(axis=0)
    lev = c["level"].astype(np.int64)
    l = L * np.ldexp(1.0, -lev)
    side = np.zeros(t.ncells)
    centre = np.zeros((t.ncells, 3))
    for i in range(t.ncells):
        s, e = c["first"][i], c["first"][i] + c["count"][i]
        sh = 20 - lev[i]
        cell = np.minimum(np.floor((x0[s] - lo) * scale), 2 ** 20 - 1).astype(np.int64) >> sh
        p = x[s:e]
        inb = np.all((p >= lo) & (p <= hi))
        qp = np.minimum(np.floor((p - lo) * scale), 2 ** 20 - 1).astype(np.int64) >> sh
        if inb and np.all(qp == cell):
            side[i] = l[i]
            centre[i] = lo + (cell + 0.5) * l[i]
        else:
            ext = (p.max(axis=0) - p.min(axis=0)).max()
            side[i] = max(l[i], ext)
            centre[i] = 0.5 * (p.min(axis=0) + p.max(axis=0))
    return side, centre, l


def _grown_rcrit2(t, build_pos, pos, theta):
    """Eq. (1) radius of every cell after a refit to pos (side and centre from
    _refit_geometry)."""
    side, centre, l = _refit_geometry(t, build_pos, pos)
    d = t.moments()["com"] - centre
    delta = np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
    r = side / np.float64(np.float32(theta)) + delta
    return (r * r).astype(np.float32), side, l, centre


@pytest.mark.parametrize("dt", [1 / 64, 1 / 8])
def test_refit_grows_the_cell_side_to_the_particles_extent(dt):
    pos, vel, m = workloads.plummer(4000, 36)
    t = oracle.Tree(pos, m)
    new = pos + vel * dt
    t.refit(new)
    want, side, l, centre = _grown_rcrit2(t, pos, new, 0.7)
    got, got_centre = t.rcrit(0.7)
    assert np.array_equal(got, want)
    assert np.array_equal(got_centre, centre)
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
    _, side, l, _ = _grown_rcrit2(t, pos, new, 0.5)
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


def _box_dist(x, centre, half):
    """Distance of each point of x from the box (centre, half sides), float64."""
    u = np.maximum(np.abs(x - centre) - half.astype(np.float64), 0.0)
    return np.sqrt((u * u).sum(axis=1))


def _drifted_refit(n, seed, dt, mac):
    pos, vel, m = workloads.plummer(n, seed)
    t = oracle.Tree(pos, m, mac=mac)
    new = pos + vel * dt
    t.refit(new)
    perm, _ = t.order()
    return t, new[perm]


@pytest.mark.parametrize("dt", [1 / 8, 1 / 2])
def test_refit_min_distance_accepts_only_cells_whose_particles_are_beyond_the_radius(dt):
    # Sect. 3.3's alternative test accepts a cell only when its cube lies farther
    # than l / theta from the group's box; after a refit that guarantee must hold
    # for the cell's particles themselves, wherever they drifted
    theta = 0.75
    t, x = _drifted_refit(3000, 41, dt, mac=1)
    rmin2, _ = t.rcrit(theta)
    g = t.groups()
    c = t.cells()
    checked = 0
    for gi in range(t.ngroups):
        pc, _ = t.group_lists(theta, gi)
        for ci in pc:
            p = x[c["first"][ci]:c["first"][ci] + c["count"][ci]]
            d = _box_dist(p, g["centre"][gi], g["half"][gi]).min()
            assert d >= np.sqrt(np.float64(rmin2[ci])) * (1 - 1e-6), (gi, ci)
            checked += 1
    assert checked > 1000


@pytest.mark.parametrize("dt", [1 / 8, 1 / 2])
def test_refit_eq1_accepted_cells_hold_no_target_of_the_group(dt):
    # Eq. (1) with theta <= 1: every particle of an accepted cell lies closer to
    # the cell's centre of mass than the group's box does (the expansion about
    # the centre of mass converges at every target), also after a refit
    theta = 0.9
    t, x = _drifted_refit(3000, 42, dt, mac=0)
    com = t.moments()["com"]
    g = t.groups()
    c = t.cells()
    checked = 0
    for gi in range(t.ngroups):
        pc, _ = t.group_lists(theta, gi)
        for ci in pc:
            p = x[c["first"][ci]:c["first"][ci] + c["count"][ci]]
            reach = np.sqrt(((p - com[ci]) ** 2).sum(axis=1)).max()
            d = _box_dist(com[ci][None, :], g["centre"][gi], g["half"][gi])[0]
            assert reach < d * (1 + 1e-6), (gi, ci)
            checked += 1
    assert checked > 1000


def _spread_leaf(mac):
    """Two clusters of three particles (a leaf of N_leaf = 3 each at level 1);
    the refit moves the upper leaf's particles so that their centre of mass stays
    at the leaf's geometric centre (0.7, 0.7, 0.7) while one of them runs off:
    (1.1, 1.1, 1.1) and twice (0.5, 0.5, 0.5)."""
    pos = np.array([[0.1, 0.1, 0.1], [0.2, 0.1, 0.1], [0.1, 0.2, 0.1],
                    [0.7, 0.7, 0.7], [0.8, 0.8, 0.8], [0.9, 0.9, 0.9]])
    m = np.full(6, 1.0 / 6)
    t = oracle.Tree(pos, m, nleaf=3, ncrit=3, mac=mac)
    c = t.cells()
    assert t.ncells == 3 and list(c["count"]) == [6, 3, 3]
    new = pos.copy()
    new[3] = [1.1, 1.1, 1.1]
    new[4] = [0.5, 0.5, 0.5]
    new[5] = [0.5, 0.5, 0.5]
    t.refit(new)
    perm, _ = t.order()
    return t, new[perm], c


@pytest.mark.parametrize("theta", [0.5, 0.9, 1.0])
def test_refit_eq1_radius_holds_every_particle_of_a_spread_leaf(theta):
    # Eq. (1) with theta <= 1: the sphere of radius r_crit about a cell's centre
    # of mass holds all of the cell's particles (a box beyond r_crit is beyond
    # every source).  After the refit above, the cell of side 0.6 centred on its
    # particles' box (0.8, 0.8, 0.8) gives r_crit = 0.6 / theta + 0.1 sqrt(3)
    t, x, c = _spread_leaf(mac=0)
    r2, centre = t.rcrit(theta)
    com = t.moments()["com"]
    for ci in range(t.ncells):
        p = x[c["first"][ci]:c["first"][ci] + c["count"][ci]]
        reach = np.sqrt(((p - com[ci]) ** 2).sum(axis=1)).max()
        assert np.sqrt(np.float64(r2[ci])) >= reach * (1 - 1e-6), ci
    assert np.allclose(centre[2], [0.8, 0.8, 0.8], rtol=0, atol=1e-15)
    want = 0.6 / np.float64(np.float32(theta)) + np.sqrt(3 * 0.1 ** 2)
    assert np.sqrt(np.float64(r2[2])) == pytest.approx(want, rel=1e-6)


def test_refit_min_distance_cube_holds_every_particle_of_a_spread_leaf():
    theta = 0.8
    t, x, c = _spread_leaf(mac=1)
    rmin2, centre = t.rcrit(theta)
    for ci in range(t.ncells):
        p = x[c["first"][ci]:c["first"][ci] + c["count"][ci]]
        half = 0.5 * np.float64(np.float32(theta)) * np.sqrt(np.float64(rmin2[ci]))
        assert np.all(np.abs(p - centre[ci]) <= half * (1 + 1e-6)), ci
    # the lower leaf kept its particles: its geometry is the build's
    assert np.allclose(centre[1], [0.3, 0.3, 0.3], rtol=0, atol=1e-15)


def test_refit_at_the_build_positions_keeps_both_tests_lists():
    pos, _, m = workloads.plummer(3000, 43)
    for mac in (0, 1):
        t = oracle.Tree(pos, m, mac=mac)
        c0 = t.walk_counts(0.7)
        r0, g0 = t.rcrit(0.7)
        t.refit(pos)
        r1, g1 = t.rcrit(0.7)
        assert np.array_equal(r0, r1) and np.array_equal(g0, g1)
        c1 = t.walk_counts(0.7)
        assert np.array_equal(c0[0], c1[0]) and np.array_equal(c0[1], c1[1])
