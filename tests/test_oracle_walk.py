"""Pins of the oracle's opening test (Sect. 3.3, Eq. (1)), breadth-first group walk
(Sect. 2.2) and float64 force evaluation (Sect. 3.2 moments, Plummer softening)."""

import numpy as np
import pytest

import oracle
import workloads


def _dumbbell(axis, R, a=1.0, m=1.0):
    """Two masses m at (0,0,+-a) and a unit target on the z axis (axis='z') or the
    x axis (axis='x') at distance R from their centre; nleaf = ncrit = 1 puts the
    target in its own group and the pair in its own level-1 cell."""
    tgt = [0.0, 0.0, R] if axis == "z" else [R, 0.0, 0.0]
    pos = np.array([[0.0, 0.0, -a], [0.0, 0.0, a], tgt])
    mass = np.array([m, m, 1.0])
    return pos, mass


def _target_group(t, target_input_index=2):
    perm, _ = t.order()
    s = int(np.nonzero(perm == target_input_index)[0][0])
    g = t.groups()
    return int(np.nonzero((g["first"] <= s) & (s < g["first"] + g["count"]))[0][0])


@pytest.mark.parametrize("axis", ["z", "x"])
def test_dumbbell_far_field_is_quadrupole_accurate(axis):
    a, R, m = 1.0, 30.0, 1.0
    pos, mass = _dumbbell(axis, R, a, m)
    t = oracle.Tree(pos, mass, nleaf=1, ncrit=1)
    g = _target_group(t)
    pc, ppl = t.group_lists(1.0, g)
    c = t.cells()
    # the pair's cell is taken as one multipole
    pair = [i for i in pc if c["count"][i] == 2]
    assert len(pair) == 1 and len(pc) == 1
    acc, pot, _, _ = t.forces(1.0, 0.0)
    if axis == "z":
        exact_a = -m / (R - a) ** 2 - m / (R + a) ** 2
        exact_p = -m / (R - a) - m / (R + a)
        got_a = acc[2, 2]
        mono = -2 * m / R ** 2
        assert abs(acc[2, 0]) < 1e-15 and abs(acc[2, 1]) < 1e-15
    else:
        exact_a = -2 * m * R / (R * R + a * a) ** 1.5
        exact_p = -2 * m / np.sqrt(R * R + a * a)
        got_a = acc[2, 0]
        mono = -2 * m / R ** 2
        assert abs(acc[2, 1]) < 1e-15 and abs(acc[2, 2]) < 1e-15
    # quadrupole truncation error is O((a/R)^4) ~ 6e-6; the monopole alone is off
    # by O((a/R)^2) ~ 3e-3
    assert abs(got_a - exact_a) / abs(exact_a) < 2e-5
    assert abs(pot[2] - exact_p) / abs(exact_p) < 2e-5
    assert abs(mono - exact_a) / abs(exact_a) > 1e-3


def test_mac_threshold_matches_eq1_geometry():
    # z dumbbell: pair cell at level 1 has side l = L/2, geometric centre
    # lo + l/2 per axis, centre of mass at the origin, distance to the target d = R.
    a, R = 1.0, 30.0
    pos, mass = _dumbbell("z", R, a)
    t = oracle.Tree(pos, mass, nleaf=1, ncrit=1)
    g = _target_group(t)
    L = R + a
    l = L / 2
    centre = np.array([0.0, 0.0, -a]) + 0.5 * l
    delta = np.linalg.norm(centre)
    theta_star = l / (R - delta)          # d = l/theta + delta
    pair = int(np.nonzero(t.cells()["count"] == 2)[0][0])
    for theta, want in ((theta_star * 1.01, True), (theta_star * 0.99, False)):
        pc, _ = t.group_lists(theta, g)
        assert (pair in pc) == want
    # the same through the single-pair opening test
    r2, _ = t.rcrit(theta_star * 1.01)
    assert t.mac_accept(g, pair, r2[pair])
    r2, _ = t.rcrit(theta_star * 0.99)
    assert not t.mac_accept(g, pair, r2[pair])


@pytest.mark.parametrize("n", [2, 17, 300, 512])
def test_tiny_theta_reduces_to_direct_summation(n):
    pos, _, m = workloads.plummer(n, 11)
    t = oracle.Tree(pos, m, 16, 64)
    npp, npc = t.walk_counts(1e-6)
    assert np.all(npc == 0) and np.all(npp == n)
    acc, pot, _, _ = t.forces(1e-6, 0.01)
    ad, pd = oracle.direct(pos, m, 0.01)
    assert np.allclose(acc, ad, rtol=1e-12, atol=1e-12 * np.abs(ad).max())
    assert np.allclose(pot, pd, rtol=1e-12, atol=0)


def test_two_body_closed_form():
    pos, _, m = workloads.two_body(sep=0.7, m1=0.3, m2=1.1)
    t = oracle.Tree(pos, m)
    for eps in (0.0, 0.05):
        acc, pot, _, _ = t.forces(0.5, eps)
        e = float(np.float32(eps))     # the softening length is a float32 parameter
        s = 0.7 ** 2 + e * e
        assert acc[0, 0] == pytest.approx(1.1 * 0.7 / s ** 1.5, rel=1e-15)
        assert acc[1, 0] == pytest.approx(-0.3 * 0.7 / s ** 1.5, rel=1e-15)
        assert pot[0] == pytest.approx(-1.1 / np.sqrt(s), rel=1e-15)
        assert np.all(acc[:, 1:] == 0)


def test_direct_sum_conserves_momentum():
    pos, _, m = workloads.clustered(700, 2)
    acc, _ = oracle.direct(pos, m, 0.001)
    f = (m[:, None] * acc).sum(axis=0)
    scale = (m * np.linalg.norm(acc, axis=1)).sum()
    assert np.all(np.abs(f) <= 1e-13 * scale)


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.75, 1.0])
@pytest.mark.parametrize("name", ["plummer", "clustered", "cube"])
def test_walk_lists_cover_every_particle_once(theta, name):
    gen = {"plummer": workloads.plummer, "clustered": workloads.clustered,
           "cube": workloads.uniform_cube}[name]
    pos, _, m = gen(2500, 6)
    t = oracle.Tree(pos, m, 16, 64)
    c = t.cells()
    npp, npc = t.walk_counts(theta)
    for g in range(0, t.ngroups, max(1, t.ngroups // 40)):
        pc, ppl = t.group_lists(theta, g)
        assert len(pc) == npc[g]
        assert c["count"][ppl].sum() == npp[g]
        assert c["count"][pc].sum() + npp[g] == t.n
        assert np.all(c["is_leaf"][ppl] == 1)


@pytest.mark.parametrize("theta", [0.4, 0.75])
def test_walk_lists_equal_brute_force_enumeration(theta):
    # c is in the cell list iff it is accepted and every strict ancestor is
    # opened; a leaf is in the particle list iff it and all ancestors are opened.
    pos, _, m = workloads.plummer(600, 7)
    t = oracle.Tree(pos, m, 8, 32)
    c = t.cells()
    r2, _ = t.rcrit(theta)
    for g in range(0, t.ngroups, 3):
        acc_cell = np.array([t.mac_accept(g, i, r2[i]) for i in range(t.ncells)])
        opened_path = np.zeros(t.ncells, bool)   # all strict ancestors opened
        opened_path[0] = True
        for i in range(1, t.ncells):             # parents precede children
            p = c["parent"][i]
            opened_path[i] = opened_path[p] and not acc_cell[p]
        want_pc = np.nonzero(opened_path & acc_cell)[0]
        want_pp = np.nonzero(opened_path & ~acc_cell & (c["is_leaf"] == 1))[0]
        pc, ppl = t.group_lists(theta, g)
        assert np.array_equal(pc, want_pc)
        assert np.array_equal(ppl, want_pp)


def test_own_particles_are_never_in_an_accepted_cell():
    # d <= l sqrt(3)/2 + delta < l/theta + delta for theta <= 1 when the cell holds
    # a particle of the group, so every target meets its own leaf in the p-p list.
    pos, _, m = workloads.plummer(3000, 8)
    t = oracle.Tree(pos, m)
    c = t.cells()
    g = t.groups()
    for gi in range(0, t.ngroups, 7):
        pc, _ = t.group_lists(1.0, gi)
        s, e = g["first"][gi], g["first"][gi] + g["count"][gi]
        for i in pc:
            assert c["first"][i] + c["count"][i] <= s or c["first"][i] >= e


def test_tree_error_against_direct_summation_plummer_4096():
    # Eq. (2) at the small workload (theta = 0.5, eps = 0.01): the paper reports
    # only plots; the bounds here are the acceptance bounds used for the GPU path.
    pos, _, m = workloads.plummer(4096, 1)
    t = oracle.Tree(pos, m)
    acc, _, _, _ = t.forces(0.5, 0.01)
    ad, _ = oracle.direct(pos, m, 0.01)
    err = np.linalg.norm(acc - ad, axis=1) / np.linalg.norm(ad, axis=1)
    assert np.median(err) < 1e-3 and np.percentile(err, 99) < 1e-2


def test_mac_is_strict():
    # Eq. (1) accepts only when d is larger than l/theta + delta: a cell whose
    # float32 d^2 equals r_crit^2 is opened.  d^2 is formed here from the exported
    # group box and centre of mass in the same float32 order (x, y, then z).
    pos, _, m = workloads.plummer(2000, 12)
    t = oracle.Tree(pos, m)
    g = t.groups()
    mo = t.moments()
    for gi, c in ((3, 17), (10, 5), (25, 40)):
        o = (mo["com"][c] - g["centre"][gi]).astype(np.float32)
        u = np.maximum(np.abs(o) - g["half"][gi], np.float32(0))
        d2 = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]
        assert d2.dtype == np.float32 and d2 > 0
        assert not t.mac_accept(gi, c, d2)
        assert t.mac_accept(gi, c, np.nextafter(d2, np.float32(0)))


def test_threaded_evaluation_equals_the_serial_one():
    # the thread split only partitions the groups (targets): every row is the
    # same computation, bit for bit
    pos, _, m = workloads.plummer(6000, 91)
    t = oracle.Tree(pos, m)
    one = t.forces(0.6, 0.01)
    many = t.forces(0.6, 0.01, threads=5)
    for a, b in zip(one, many):
        assert np.array_equal(a, b)
    sel = np.arange(3, t.ngroups, 7)
    one = t.forces(0.6, 0.01, sel)
    many = t.forces(0.6, 0.01, sel, threads=3)
    for a, b in zip(one, many):
        assert np.array_equal(a, b, equal_nan=True)
    tgt = np.arange(0, 6000, 11)
    d1 = oracle.direct(pos, m, 0.01, tgt)
    d4 = oracle.direct(pos, m, 0.01, tgt, threads=4)
    assert np.array_equal(d1[0], d4[0]) and np.array_equal(d1[1], d4[1])
