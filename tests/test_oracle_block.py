"""Pins of the oracle's block time-steps (Sect. 5: forces only for the particles
due, multipole-only refits in between, a rebuild once the walk has grown).  The
paper gives neither the time-step criterion nor the schedule; the pins check the
readings taken (bh_oracle.c) against closed forms, against the oracle's own
shared-step leapfrog, and against the integrator's order."""

import numpy as np
import pytest

import oracle
import workloads


def test_bins_against_the_closed_form():
    rng = np.random.default_rng(3)
    n = 20000
    acc = (rng.standard_normal((n, 3)) * np.exp(rng.uniform(-6, 6, (n, 1)))).astype(np.float32)
    acc[:5] = 0.0
    dt_max, B, eta, length = 1 / 16, 6, 0.025, 0.01
    bins = oracle.block_bins(acc, dt_max, B, eta, length)
    a = np.linalg.norm(acc.astype(np.float64), axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        x = np.log2(dt_max / np.sqrt(2 * eta * length / a))   # bins needed: ceil(x)
        want = np.clip(np.ceil(x), 0, B).astype(int)
        clear = (a == 0) | (np.abs(x - np.round(x)) > 1e-9)
    want[a == 0] = 0
    assert clear.sum() > n - 10
    assert np.array_equal(bins[clear], want[clear])
    assert np.all(bins[:5] == 0)
    # the bin never decreases as |a| grows
    order = np.argsort(a, kind="stable")
    assert np.all(np.diff(bins[order].astype(int)) >= 0)
    assert set(np.unique(bins)) == set(range(B + 1))


def test_bin_boundary_is_inclusive():
    # dt_max = 1, eta = 1/2, l = 1, |a| = 4: the criterion sqrt(2 eta l / |a|) is
    # exactly 1/2 = dt_max 2^-1, and a step equal to it is taken; a hair more
    # acceleration needs the next bin
    acc = np.array([[4.0, 0, 0], [0, -4.0, 0], [4.0 * (1 + 2.0 ** -20), 0, 0], [0, 0, 3.99]],
                   np.float32)
    assert list(oracle.block_bins(acc, 1.0, 3, 0.5, 1.0)) == [1, 1, 2, 1]


def test_one_level_always_rebuilding_is_the_leapfrog():
    pos, vel, m = workloads.plummer(2000, 41)
    b = oracle.Block(pos, vel, m, 0.6, 0.01)
    p, v = pos.copy(), vel.copy()
    t = oracle.Tree(p, m)
    acc, pot, _, _ = t.forces(0.6, 0.01)
    for _ in range(3):
        rebuilt, _, kicks = b.step(np.zeros(2000, np.uint8), 0, 1 / 64, 0.0)
        oracle.kdk_step(p, v, m, acc, pot, 1 / 64, 0.6, 0.01)
        assert rebuilt and np.all(kicks == 1)
        assert np.array_equal(b.pos, p) and np.array_equal(b.vel, v)
        assert np.array_equal(b.acc, acc) and np.array_equal(b.pot, pot)


def test_coarsest_bin_only_drifts_between_its_kicks():
    # every particle in bin 0 of a 3-level block: nothing is due before the end,
    # so the 8 substeps are one drift and the step is the leapfrog step
    pos, vel, m = workloads.plummer(1500, 42)
    b = oracle.Block(pos, vel, m, 0.6, 0.01)
    p, v = pos.copy(), vel.copy()
    t = oracle.Tree(p, m)
    acc, pot, _, _ = t.forces(0.6, 0.01)
    _, _, kicks = b.step(np.zeros(1500, np.uint8), 3, 1 / 32, 0.0)
    oracle.kdk_step(p, v, m, acc, pot, 1 / 32, 0.6, 0.01)
    assert np.all(kicks == 1)
    assert np.array_equal(b.pos, p) and np.array_equal(b.vel, v)


def test_each_particle_completes_two_to_the_bin_steps():
    pos, vel, m = workloads.clustered(2500, 43)
    rng = np.random.default_rng(44)
    bins = rng.integers(0, 5, 2500).astype(np.uint8)
    b = oracle.Block(pos, vel, m, 0.7, 0.01)
    _, _, kicks = b.step(bins, 4, 1 / 64, 0.0)
    assert np.array_equal(kicks, 1 << bins.astype(np.int64))


def test_finest_bin_equals_shared_steps_of_the_finest_size():
    # theta -> 0 makes the forces the direct sum whatever the tree (refit or
    # rebuild), so all particles in bin B must follow 2^B leapfrog steps of dt/2^B
    pos, vel, m = workloads.plummer(300, 45)
    b = oracle.Block(pos, vel, m, 1e-6, 0.01)
    p, v = pos.copy(), vel.copy()
    acc, pot = oracle.direct(p, m, 0.01)
    b.step(np.full(300, 2, np.uint8), 2, 1 / 16, 0.0)
    for _ in range(4):
        oracle.kdk_step(p, v, m, acc, pot, 1 / 64, 1e-6, 0.01)
    assert np.allclose(b.pos, p, rtol=0, atol=1e-13)
    assert np.allclose(b.vel, v, rtol=0, atol=1e-12)


def _orbit_error(bins, nper, e=0.5, m1=1.0, m2=0.3):
    M = m1 + m2
    rp = 1.0 - e
    vp = np.sqrt(M * (1 + e) / rp)
    pos = np.array([[-m2 / M * rp, 0, 0], [m1 / M * rp, 0, 0]])
    vel = np.array([[0, -m2 / M * vp, 0], [0, m1 / M * vp, 0]])
    mass = np.array([m1, m2])
    b = oracle.Block(pos, vel, mass, 1.0, 0.0, 1, 1)

    def energy():
        T = 0.5 * (mass * (b.vel ** 2).sum(axis=1)).sum()
        return T - m1 * m2 / np.linalg.norm(b.pos[0] - b.pos[1])
    e0 = energy()
    period = 2 * np.pi / np.sqrt(M)
    worst = 0.0
    for _ in range(nper):
        b.step(np.array(bins, np.uint8), 2, period / nper, 0.0)
        worst = max(worst, abs((energy() - e0) / e0))
    return worst


@pytest.mark.parametrize("bins", [(0, 2), (1, 2), (2, 0)])
def test_second_order_with_mixed_bins(bins):
    # an eccentric Kepler orbit over one period: halving the block step divides
    # the largest energy error by 4
    errs = [_orbit_error(bins, n) for n in (64, 128, 256)]
    for a, b in zip(errs, errs[1:]):
        assert 3.6 < a / b < 4.4, errs


def test_rebuild_rule_and_the_walk_it_measures():
    # one level (B = 0): each block step is one force evaluation with every
    # particle due, on the tree refitted to the new positions unless the walk
    # before it had grown past the limit
    pos, vel, m = workloads.plummer(3000, 46)
    b = oracle.Block(pos, vel, m, 0.6, 0.01)
    base0 = b.base
    t0 = oracle.Tree(pos, m)
    npp, npc = t0.walk_counts(0.6)
    assert base0 == (t0.groups()["count"] * (npp + npc)).sum() / 3000
    assert not b.rebuild_next
    zero = np.zeros(3000, np.uint8)
    # a limit that cannot be reached: refitted, and the walk is the refitted tree's
    rebuilt, inter, _ = b.step(zero, 0, 1 / 8, 1e9)
    assert rebuilt == 0 and b.base == base0 and not b.rebuild_next
    t0.refit(b.pos)
    npp, npc = t0.walk_counts(0.6)
    assert inter == (t0.groups()["count"] * (npp + npc)).sum() / 3000
    assert inter > base0        # the refitted cells have grown
    acc, pot, _, _ = t0.forces(0.6, 0.01)
    assert np.array_equal(b.acc, acc) and np.array_equal(b.pot, pot)
    # a limit below the growth: the next evaluation is on a rebuilt tree, whose
    # walk becomes the new base; then the refit again
    c = oracle.Block(pos, vel, m, 0.6, 0.01)
    rebuilt, inter1, _ = c.step(zero, 0, 1 / 8, 1e-9)
    assert rebuilt == 0 and inter1 == inter and c.rebuild_next
    rebuilt, inter2, _ = c.step(zero, 0, 1 / 8, 1e-9)
    assert rebuilt == 1 and not c.rebuild_next
    t1 = oracle.Tree(c.pos, m)
    npp, npc = t1.walk_counts(0.6)
    assert c.base == inter2 == (t1.groups()["count"] * (npp + npc)).sum() / 3000
    acc, pot, _, _ = t1.forces(0.6, 0.01)
    assert np.array_equal(c.acc, acc) and np.array_equal(c.pot, pot)
    rebuilt, _, _ = c.step(zero, 0, 1 / 8, 1e-9)
    assert rebuilt == 0 and c.rebuild_next


def test_growth_zero_rebuilds_before_every_force_evaluation():
    # all particles in the finest of 3 levels: 8 evaluations, 8 rebuilds, and the
    # final forces are those of a fresh tree
    pos, vel, m = workloads.plummer(2000, 47)
    b = oracle.Block(pos, vel, m, 0.6, 0.01)
    rebuilt, inter, kicks = b.step(np.full(2000, 3, np.uint8), 3, 1 / 8, 0.0)
    assert rebuilt == 8 and np.all(kicks == 8) and not b.rebuild_next
    t = oracle.Tree(b.pos, m)
    acc, pot, _, _ = t.forces(0.6, 0.01)
    assert np.array_equal(b.acc, acc) and np.array_equal(b.pot, pot)
    assert b.base == inter


def test_rebuild_threshold_is_one_plus_growth_times_the_base():
    # the same walk judged with the limit just above and just below the growth it
    # measures: kept, then rebuilt before the next evaluation
    pos, vel, m = workloads.plummer(3000, 46)
    zero = np.zeros(3000, np.uint8)
    first = oracle.Block(pos, vel, m, 0.6, 0.01)
    _, inter, _ = first.step(zero, 0, 1 / 8, 1e9)
    grown = inter / first.base - 1.0
    assert 0.0 < grown < 0.5
    for limit, want in ((grown * 1.01, False), (grown * 0.99, True)):
        b = oracle.Block(pos, vel, m, 0.6, 0.01)
        b.step(zero, 0, 1 / 8, limit)
        assert b.rebuild_next == want, (limit, grown)


def test_walks_of_due_groups_compare_with_the_base_of_the_particles_they_cover():
    # two levels, the finest holding a few particles: the substep's walk covers only
    # their groups, and its growth is judged against those particles' base alone
    pos, vel, m = workloads.plummer(3000, 48)
    bins = np.zeros(3000, np.uint8)
    bins[:40] = 1
    # replay the substep by hand: opening kicks, drift half the step, refit, walk
    # the groups holding the 40 particles
    b = oracle.Block(pos, vel, m, 0.6, 0.01)
    t = oracle.Tree(pos, m)
    npp0, npc0 = t.walk_counts(0.6)
    g = t.groups()
    perm, _ = t.order()
    gid = np.repeat(np.arange(g["count"].shape[0]), g["count"])
    pbase = np.zeros(3000, np.int64)
    pbase[perm] = (npp0 + npc0)[gid]
    v = vel + b.acc * (0.5 / 4)                     # opening half kicks (bins 0 and 1)
    v[:40] = vel[:40] + b.acc[:40] * (0.5 / 8)
    p = pos + v * (1 / 8)
    t.refit(p)
    npp, npc = t.walk_counts(0.6)
    walked = np.unique(gid[np.isin(perm, np.arange(40))])
    now = (g["count"][walked] * (npp + npc)[walked]).sum()
    cover = np.isin(gid, walked)
    base_cov = pbase[perm[cover]].sum()
    grown = now / base_cov - 1.0
    assert grown > 0.0
    # the decision at the substep picks the tree of the final evaluation: rebuilt
    # with a limit just below the growth of the covered particles, refitted just
    # above it
    for limit, want in ((grown * 0.99, 1), (grown * 1.01, 0)):
        d = oracle.Block(pos, vel, m, 0.6, 0.01)
        rebuilt, _, _ = d.step(bins, 1, 1 / 4, limit)
        assert rebuilt == want, (limit, grown)


def test_a_walk_that_has_not_grown_is_kept():
    # a block step too short to move anything: the refitted walk equals the base,
    # and with 1 + growth == 1 in float64 only strictly more would rebuild
    pos, vel, m = workloads.plummer(2000, 49)
    b = oracle.Block(pos, vel, m, 0.6, 0.01)
    base = b.base
    rebuilt, inter, _ = b.step(np.zeros(2000, np.uint8), 0, 1e-300, 1e-30)
    assert np.array_equal(b.pos, pos)
    assert rebuilt == 0 and inter == base and not b.rebuild_next


def test_substeps_with_nothing_due_leave_the_decision_alone():
    # every particle in bin 1 of a 2-level block: substeps 1 and 3 only drift; the
    # decision of the walk at substep 2 picks the tree at substep 4, which is then
    # a fresh tree at the final positions
    pos, vel, m = workloads.plummer(2000, 50)
    b = oracle.Block(pos, vel, m, 0.6, 0.01)
    rebuilt, _, kicks = b.step(np.ones(2000, np.uint8), 2, 1 / 8, 1e-9)
    assert rebuilt == 1 and np.all(kicks == 2) and not b.rebuild_next
    t = oracle.Tree(b.pos, m)
    acc, pot, _, _ = t.forces(0.6, 0.01)
    assert np.array_equal(b.acc, acc) and np.array_equal(b.pot, pot)
