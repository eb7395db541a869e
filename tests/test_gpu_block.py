"""GPU tests of block time-steps (bh_block_bins, bh_block_step) against the
oracle's block integrator: bins bit-exact from the same accelerations, one level
with a rebuild every step is the leapfrog step bit for bit, block steps follow
the oracle given the same bins (positions and velocities within the bound the
float32 forces allow, the same rebuild decisions, the same walk measure), the
substeps walk exactly the groups holding due particles, and a batch of clusters
advances as each cluster alone."""

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import say, to_dev

pytestmark = pytest.mark.gpu

ETA, LENGTH = 0.025, 0.01


def _ctx(pos, vel, mass, theta, eps, nleaf=16, ncrit=64, mac=0):
    import paper_1106_1900_amd as bh
    ctx = bh.Context(nleaf=nleaf, ncrit=ncrit)
    ctx.set_mac(mac)
    ctx.build_tree(to_dev(pos), to_dev(mass))
    ctx.set_velocities(to_dev(vel))
    ctx.compute_forces(theta, eps, want=False)
    return ctx


def _state(ctx):
    return [t.cpu().numpy() for t in ctx.get_state()]


def test_bins_equal_the_oracle_bins_of_the_same_accelerations():
    pos, vel, m = workloads.plummer(50_000, 71)
    ctx = _ctx(pos, vel, m, 0.75, 1 / 64)
    for dt_max, B in ((1 / 16, 4), (1 / 4, 7), (1 / 1024, 0)):
        bins, count = ctx.block_bins(dt_max, ETA, LENGTH, B)
        bins = bins.cpu().numpy()
        acc = _state(ctx)[2]
        want = oracle.block_bins(acc, dt_max, B, ETA, LENGTH)
        assert np.array_equal(bins, want), (dt_max, B)
        assert count == list(np.bincount(want, minlength=16))
    ctx.close()


def test_bin_boundary_is_inclusive_on_the_device():
    # two bodies of mass 4 one unit apart, no softening: |a| = 4 exactly, and with
    # dt_max = 1, eta = 1/2, l = 1 the criterion sqrt(2 eta l / |a|) = 1/2 is met
    # with equality by bin 1
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    m = np.array([4.0, 4.0])
    ctx = _ctx(pos, np.zeros((2, 3)), m, 0.75, 0.0)
    acc = _state(ctx)[2]
    assert np.array_equal(np.abs(acc), np.array([[4.0, 0, 0], [4.0, 0, 0]], np.float32)), acc
    bins, count = ctx.block_bins(1.0, 0.5, 1.0, 3)
    assert list(bins.cpu().numpy()) == [1, 1] and count[1] == 2
    ctx.close()


def test_one_level_rebuilding_every_step_is_the_leapfrog():
    pos, vel, m = workloads.plummer(20_000, 72)
    a = _ctx(pos, vel, m, 0.6, 0.01)
    b = _ctx(pos, vel, m, 0.6, 0.01)
    for step in range(3):
        st = a.block_step(1 / 64, ETA, LENGTH, 0, 0.0)
        b.leapfrog_step(1 / 64)
        assert st["rebuilt"] == 1 and st["substeps"] == 1 and st["updates"] == 20_000
        for x, y, name in zip(_state(a), _state(b), ("pos", "vel", "acc", "pot")):
            assert np.array_equal(x, y), (step, name)
    a.close()
    b.close()


@pytest.mark.parametrize("growth,mac", [(0.0, 0), (np.float32(0.02), 0), (np.float32(1e9), 0),
                                        (np.float32(0.02), 1), (np.float32(1e9), 1)])
def test_block_steps_follow_the_oracle(growth, mac):
    n, theta, eps, B, dt_max = 6000, 0.6, 0.01, 3, 1 / 16
    pos, vel, m = workloads.plummer(n, 73)
    ctx = _ctx(pos, vel, m, theta, eps, mac=mac)
    orc = oracle.Block(pos, vel, m, theta, eps, mac=mac)
    say("case block growth", float(growth), "mac", mac)
    for step in range(3):
        bins, _ = ctx.block_bins(dt_max, ETA, LENGTH, B)
        bins = bins.cpu().numpy()
        # the oracle's own bins (float64 forces) differ only at bin edges
        mine = oracle.block_bins(orc.acc.astype(np.float32), dt_max, B, ETA, LENGTH)
        assert np.mean(mine == bins) > 0.99
        st = ctx.block_step(dt_max, ETA, LENGTH, B, float(growth))
        rebuilt, inter, kicks = orc.step(bins, B, dt_max, float(growth))
        say("block step", step, "rebuilds", st["rebuilt"], "oracle", rebuilt)
        assert st["rebuilt"] == rebuilt, (step, st, inter)
        assert st["updates"] == int(kicks.sum())
        assert abs(st["sync_interactions"] - inter) <= 1e-4 * inter
        assert abs(st["base_interactions"] - orc.base) <= 1e-4 * orc.base
        x, v, acc, pot = _state(ctx)
        # float32 forces (within 1e-5 of the sum of term magnitudes) kicked over
        # one block step
        amax = np.abs(orc.acc).max()
        tol_v = 4e-5 * amax * dt_max * (step + 1)
        assert np.abs(v - orc.vel).max() <= tol_v, np.abs(v - orc.vel).max()
        assert np.abs(x - orc.pos).max() <= tol_v * dt_max * (step + 1)
        assert np.all(np.linalg.norm(acc - orc.acc, axis=1) <= 1e-3 * np.linalg.norm(orc.acc, axis=1) + 1e-4 * amax)
    ctx.close()


def test_substeps_walk_exactly_the_groups_holding_due_particles():
    n, B, dt_max = 8000, 3, 1 / 8
    pos, vel, m = workloads.plummer(n, 74)
    ctx = _ctx(pos, vel, m, 0.7, 0.01)
    ex = ctx.export_tree()
    bins, _ = ctx.block_bins(dt_max, ETA, LENGTH, B)
    bins = bins.cpu().numpy()
    gid = np.repeat(np.arange(ex["gfirst"].shape[0]), ex["gcount"])
    pb = bins[ex["perm"]]                      # bins in the tree's (sorted) order
    want = 0
    for s in range(1, 1 << B):
        due = (s % (1 << (B - pb.astype(np.int64)))) == 0
        want += np.unique(gid[due]).shape[0]
    st = ctx.block_step(dt_max, ETA, LENGTH, B, 1e9)   # refitted throughout: the groups stay
    assert st["rebuilt"] == 0
    want += ctx.stats().ngroups                # the final walk of every group
    assert st["walked_groups"] == want
    assert st["updates"] == int((1 << bins.astype(np.int64)).sum())
    ctx.close()


def test_batch_block_step_equals_each_cluster_alone():
    import paper_1106_1900_amd as bh
    parts = []
    for i, (n, th, ep) in enumerate(((5000, 0.6, 0.01), (3000, 0.75, 0.02), (1200, 0.5, 0.01))):
        p, v, mm = workloads.plummer(n, 80 + i)
        parts.append((p, v, mm, dict(n=n, theta=th, eps=ep)))
    pos = np.concatenate([q[0] for q in parts])
    vel = np.concatenate([q[1] for q in parts])
    mass = np.concatenate([q[2] for q in parts])
    ctx = bh.Context()
    ctx.batch_build([q[3] for q in parts], to_dev(pos), to_dev(mass), to_dev(vel))
    ctx.batch_forces(want=False)
    for _ in range(2):
        ctx.block_step(1 / 16, ETA, LENGTH, 2, 0.0)
    got = _state(ctx)
    first = 0
    for p, v, mm, prm in parts:
        one = _ctx(p, v, mm, prm["theta"], prm["eps"])
        for _ in range(2):
            one.block_step(1 / 16, ETA, LENGTH, 2, 0.0)
        for x, y in zip(_state(one), got):
            assert np.array_equal(x, y[first:first + prm["n"]])
        first += prm["n"]
        one.close()
    ctx.close()


def test_block_energy_and_errors():
    import paper_1106_1900_amd as bh
    n = 30_000
    pos, vel, m = workloads.plummer(n, 75)
    ctx = _ctx(pos, vel, m, 0.5, 1 / 64)
    e0 = ctx.energy()[2]
    rebuilds = 0
    for _ in range(8):
        st = ctx.block_step(1 / 32, ETA, 1 / 64, 3, np.float32(0.05))
        rebuilds += st["rebuilt"]
    e = ctx.energy()
    say("block energy drift", (e[2] - e0) / e0, "rebuilds", rebuilds)
    assert abs((e[2] - e0) / e0) < 1e-3
    with pytest.raises(bh.BHError):
        ctx.block_step(0.0, ETA, LENGTH, 3, 0.0)
    with pytest.raises(bh.BHError):
        ctx.block_step(1 / 32, ETA, LENGTH, 16, 0.0)
    ctx.drift(0.0)
    with pytest.raises(bh.BHError):
        ctx.block_step(1 / 32, ETA, LENGTH, 3, 0.0)
    ctx.close()


def test_block_steps_at_full_size():
    # N = 2^20 Plummer, theta 0.75, eps 1/64 (the headline workload): one level with
    # a rebuild before every evaluation is the leapfrog step bit for bit, and a
    # refit-only block step of 5 levels walks exactly the groups holding due particles
    n = 1 << 20
    pos, vel, m = workloads.plummer(n, 2)
    say("case block full size", n)
    a = _ctx(pos, vel, m, 0.75, 1 / 64)
    b = _ctx(pos, vel, m, 0.75, 1 / 64)
    st = a.block_step(1 / 64, ETA, 1 / 64, 0, 0.0)
    b.leapfrog_step(1 / 64)
    assert st["rebuilt"] == 1 and st["updates"] == n
    for x, y in zip(_state(a), _state(b)):
        assert np.array_equal(x, y)
    b.close()
    ex = a.export_tree()
    bins, _ = a.block_bins(1 / 16, 0.01, 1 / 64, 5)
    pb = bins.cpu().numpy()[ex["perm"]]
    gid = np.repeat(np.arange(ex["gfirst"].shape[0]), ex["gcount"])
    want = ex["gfirst"].shape[0]                 # the final walk of every group
    for s in range(1, 32):
        due = (s % (1 << (5 - pb.astype(np.int64)))) == 0
        if due.any():
            want += np.unique(gid[due]).shape[0]
    st = a.block_step(1 / 16, 0.01, 1 / 64, 5, 1e9)
    assert st["rebuilt"] == 0 and st["walked_groups"] == want
    assert st["updates"] == int((1 << bins.cpu().numpy().astype(np.int64)).sum())
    x, v, acc, pot = _state(a)
    assert np.isfinite(x).all() and np.isfinite(acc).all()
    a.close()


def test_pending_rebuild_kept_across_block_steps_and_dropped_by_a_rebuild():
    # one level, a tiny growth limit: the refitted walk of a block step sets the
    # decision, which the next block step acts on; a leapfrog step in between
    # rebuilds the tree and the decision lapses
    pos, vel, m = workloads.plummer(20_000, 76)
    for between in (False, True):
        ctx = _ctx(pos, vel, m, 0.6, 0.01)
        st = ctx.block_step(1 / 16, ETA, LENGTH, 0, np.float32(1e-6))
        assert st["rebuilt"] == 0
        if between:
            ctx.leapfrog_step(1 / 64)
        st = ctx.block_step(1 / 16, ETA, LENGTH, 0, np.float32(1e-6))
        assert st["rebuilt"] == (0 if between else 1), between
        ctx.close()
