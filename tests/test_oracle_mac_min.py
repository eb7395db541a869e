"""Pins of the oracle's minimum-distance opening test, the alternative to Eq. (1)
that Sect. 3.3 names (Salmon & Warren 1994): a cell is accepted for a group when
the smallest distance between the group's box and the cell's cube exceeds
l/theta.  The pins use an independent formulation (interval separation of the two
boxes in float64, the cube's centre de-interleaved from the exported key prefix),
the theta -> 0 limit (direct summation), brute-force enumeration of the lists, and
the two properties the paper states for this test: more interactions and a
smaller force error than Eq. (1) at the same theta."""

import numpy as np
import pytest

import oracle
import workloads


def _deinterleave(prefix, level):
    """Integer cube coordinates of a level-`level` key prefix (x bits at 3b, y at
    3b + 1, z at 3b + 2)."""
    p = np.zeros((prefix.shape[0], 3), np.int64)
    for b in range(int(level.max()) + 1):
        for k in range(3):
            bit = (prefix >> np.uint64(3 * b + k)) & np.uint64(1)
            p[:, k] |= (bit.astype(np.int64) << b) * (b < level)
    return p


def _cubes(t):
    c = t.cells()
    lo, L, _ = t.domain()
    lev = c["level"].astype(np.int64)
    side = L * np.ldexp(1.0, -lev)
    p = _deinterleave(c["prefix"].astype(np.uint64), lev)
    centre = np.asarray(lo)[None, :] + (p + 0.5) * side[:, None]
    return centre, side


def test_radius_and_centre_of_the_minimum_distance_test():
    pos, _, m = workloads.plummer(1500, 21)
    t = oracle.Tree(pos, m, 16, 64, mac=1)
    assert t.mac == 1
    centre, side = _cubes(t)
    for theta in (0.3, 0.75, 1.0):
        r2, cen = t.rcrit(theta)
        want = (side / np.float64(np.float32(theta))) ** 2
        assert np.array_equal(r2, want.astype(np.float32))
        assert np.array_equal(cen, centre)


@pytest.mark.parametrize("theta", [0.4, 0.75])
def test_decision_equals_interval_separation_of_the_boxes(theta):
    pos, _, m = workloads.plummer(800, 22)
    t = oracle.Tree(pos, m, 8, 32, mac=1)
    centre, side = _cubes(t)
    g = t.groups()
    r2, _ = t.rcrit(theta)
    checked = [0, 0]
    for gi in range(0, t.ngroups, 5):
        glo = g["centre"][gi] - g["half"][gi].astype(np.float64)
        ghi = g["centre"][gi] + g["half"][gi].astype(np.float64)
        clo = centre - 0.5 * side[:, None]
        chi = centre + 0.5 * side[:, None]
        gap = np.maximum(0.0, np.maximum(clo - ghi[None, :], glo[None, :] - chi))
        d2 = (gap ** 2).sum(axis=1)
        lim = (side / np.float64(np.float32(theta))) ** 2
        clear = np.abs(d2 - lim) > 1e-4 * lim      # away from float32 rounding ties
        for c in np.nonzero(clear)[0]:
            want = d2[c] > lim[c]
            assert t.mac_accept(gi, c, r2[c]) == want, (gi, c)
            checked[int(want)] += 1
    assert checked[0] > 100 and checked[1] > 100


def test_minimum_distance_test_is_strict():
    pos, _, m = workloads.plummer(2000, 23)
    t = oracle.Tree(pos, m, mac=1)
    g = t.groups()
    _, cen = t.rcrit(0.5)
    c = t.cells()
    lo, L, _ = t.domain()
    found = 0
    for gi in range(0, t.ngroups, 3):
        for ci in range(1, t.ncells, 11):
            h = np.float32(0.5 * L * 2.0 ** -int(c["level"][ci]))
            o = (cen[ci] - g["centre"][gi]).astype(np.float32)
            u = np.maximum((np.abs(o) - g["half"][gi]) - h, np.float32(0))
            d2 = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]
            if not d2 > 0:
                continue
            assert d2.dtype == np.float32
            assert not t.mac_accept(gi, ci, d2)
            assert t.mac_accept(gi, ci, np.nextafter(d2, np.float32(0)))
            found += 1
    assert found > 20


def test_a_group_never_accepts_a_cell_that_holds_its_particles():
    # the cube of such a cell overlaps the group's box: distance 0
    pos, _, m = workloads.plummer(3000, 24)
    t = oracle.Tree(pos, m, mac=1)
    c = t.cells()
    g = t.groups()
    for gi in range(0, t.ngroups, 5):
        pc, _ = t.group_lists(1.0, gi)
        s, e = g["first"][gi], g["first"][gi] + g["count"][gi]
        for i in pc:
            assert c["first"][i] + c["count"][i] <= s or c["first"][i] >= e


@pytest.mark.parametrize("n", [2, 300, 700])
def test_tiny_theta_reduces_to_direct_summation(n):
    pos, _, m = workloads.plummer(n, 25)
    t = oracle.Tree(pos, m, 16, 64, mac=1)
    npp, npc = t.walk_counts(1e-6)
    assert np.all(npc == 0) and np.all(npp == n)
    acc, pot, _, _ = t.forces(1e-6, 0.01)
    ad, pd = oracle.direct(pos, m, 0.01)
    assert np.allclose(acc, ad, rtol=1e-12, atol=1e-12 * np.abs(ad).max())
    assert np.allclose(pot, pd, rtol=1e-12, atol=0)


@pytest.mark.parametrize("theta", [0.4, 0.75])
def test_lists_equal_brute_force_enumeration(theta):
    pos, _, m = workloads.plummer(600, 26)
    t = oracle.Tree(pos, m, 8, 32, mac=1)
    c = t.cells()
    r2, _ = t.rcrit(theta)
    for g in range(0, t.ngroups, 3):
        acc_cell = np.array([t.mac_accept(g, i, r2[i]) for i in range(t.ncells)])
        opened_path = np.zeros(t.ncells, bool)
        opened_path[0] = True
        for i in range(1, t.ncells):
            p = c["parent"][i]
            opened_path[i] = opened_path[p] and not acc_cell[p]
        want_pc = np.nonzero(opened_path & acc_cell)[0]
        want_pp = np.nonzero(opened_path & ~acc_cell & (c["is_leaf"] == 1))[0]
        pc, ppl = t.group_lists(theta, g)
        assert np.array_equal(pc, want_pc)
        assert np.array_equal(ppl, want_pp)


@pytest.mark.parametrize("theta", [0.4, 0.5, 0.75])
def test_more_interactions_and_smaller_error_than_eq1(theta):
    # Sect. 3.3: at the same theta the minimum-distance test opens more cells and
    # gives a smaller acceleration error than Eq. (1)
    pos, _, m = workloads.plummer(4096, 1)
    ad, _ = oracle.direct(pos, m, 0.01)
    out = []
    for mac in (0, 1):
        t = oracle.Tree(pos, m, 16, 64, mac=mac)
        npp, npc = t.walk_counts(theta)
        inter = int((t.groups()["count"] * (npp + npc)).sum())
        acc, _, _, _ = t.forces(theta, 0.01)
        err = np.linalg.norm(acc - ad, axis=1) / np.linalg.norm(ad, axis=1)
        out.append((inter, np.median(err), np.percentile(err, 99)))
    (i0, m0, p0), (i1, m1, p1) = out
    assert i1 > i0
    assert m1 < m0 and p1 < p0
