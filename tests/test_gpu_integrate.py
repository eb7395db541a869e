"""GPU tests of the leapfrog (Sect. 3.1), the energy sums (Eq. (3)), state copies and
the error paths of the C ABI."""

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import compare_forces, compare_tree, compare_walk, gpu_build, say, to_dev

pytestmark = pytest.mark.gpu


def _state(ctx):
    pos, vel, acc, pot = ctx.get_state()
    return (pos.cpu().numpy(), vel.cpu().numpy(), acc.cpu().numpy().astype(np.float64),
            pot.cpu().numpy().astype(np.float64))


@pytest.mark.parametrize("n,seed,theta,eps,dt", [(4096, 1, 0.5, 0.01, 1 / 128),
                                                 (30_000, 3, 0.75, 1 / 64, 1 / 64)])
def test_leapfrog_steps(n, seed, theta, eps, dt):
    import paper_1106_1900_amd as bh
    say("case leapfrog", n, theta, eps, dt)
    pos, vel, m = workloads.plummer(n, seed)
    ctx = gpu_build(pos, m)
    ctx.set_velocities(to_dev(vel))
    ctx.compute_forces(theta, eps, want=False)
    x0, v0, a0, _ = _state(ctx)
    assert np.array_equal(x0, pos) and np.array_equal(v0, vel)
    h = 0.5 * dt
    for step in range(3):
        ctx.leapfrog_step(dt)
        x1, v1, a1, p1 = _state(ctx)
        # kick-drift-kick in float64 with the accelerations the library used:
        # the same operations in the same order, so bit for bit
        vh = v0 + a0 * h
        assert np.array_equal(x1, x0 + vh * dt), "drift differs"
        assert np.array_equal(v1, vh + a1 * h), "kicks differ"
        # the forces of the step are those of the rebuilt tree at the new positions
        t = oracle.Tree(x1, m)
        ex = ctx.export_tree()
        compare_tree(ex, t)
        compare_walk(ex, t, theta)
        compare_forces(a1.astype(np.float32), p1.astype(np.float32), t, theta, eps)
        x0, v0, a0 = x1, v1, a1
    # energy and momentum sums (Eq. (3)) against the oracle's float64 sums of the
    # same state (another summation order)
    e = ctx.energy()
    eo = oracle.energy(v0, m, p1)
    assert e[0] == pytest.approx(eo[0], rel=1e-12)
    assert e[1] == pytest.approx(eo[1], rel=1e-12)
    assert e[2] == pytest.approx(eo[2], rel=1e-12)
    assert np.allclose(e[3:6], eo[3:6], rtol=0, atol=1e-15 * np.abs(m[:, None] * v0).sum())
    assert e[6] == 0.0    # first call after the build sets E0
    ctx.close()


def test_energy_drift_is_small_and_second_order():
    # N = 4096 Plummer, theta 0.5, eps 0.01: relative energy error over 0.25 time
    # units at dt and dt/2
    pos, vel, m = workloads.plummer(4096, 1)
    errs = []
    for dt in (1 / 64, 1 / 128):
        ctx = gpu_build(pos, m)
        ctx.set_velocities(to_dev(vel))
        ctx.compute_forces(0.5, 0.01, want=False)
        ctx.energy()
        for _ in range(int(round(0.25 / dt))):
            ctx.leapfrog_step(dt)
        errs.append(abs(ctx.energy()[6]))
        ctx.close()
    say("dE", errs)
    assert errs[0] < 1e-4
    assert errs[1] < errs[0]


def test_state_round_trip_and_rebuild():
    pos, vel, m = workloads.plummer(20_000, 8)
    ctx = gpu_build(pos, m)
    rng = np.random.default_rng(9)
    pos2 = pos + 0.01 * rng.standard_normal(pos.shape)
    vel2 = vel + 0.1 * rng.standard_normal(vel.shape)
    ctx.set_state(to_dev(pos2), to_dev(vel2))
    x, v = ctx.get_positions()
    assert np.array_equal(x.cpu().numpy(), pos2) and np.array_equal(v.cpu().numpy(), vel2)
    acc, pot = ctx.compute_forces(0.6, 0.01)
    ex = ctx.export_tree()
    t = oracle.Tree(pos2, m)
    compare_tree(ex, t)
    compare_walk(ex, t, 0.6)
    compare_forces(acc.cpu().numpy(), pot.cpu().numpy(), t, 0.6, 0.01)
    # energy and momentum sums of the replaced state (Eq. (3)): the velocity records
    # written by set_state carry the masses the sums read
    e = ctx.energy()
    eo = oracle.energy(vel2, m, pot.cpu().numpy().astype(np.float64))
    assert e[0] == pytest.approx(eo[0], rel=1e-12)
    assert e[1] == pytest.approx(eo[1], rel=1e-12)
    assert e[2] == pytest.approx(eo[2], rel=1e-12)
    assert np.allclose(e[3:6], eo[3:6], rtol=0, atol=1e-15 * np.abs(m[:, None] * vel2).sum())
    ctx.close()


def test_resume_from_state_continues_bit_for_bit():
    # checkpoint after two steps, continue in a fresh context from the copy
    pos, vel, m = workloads.plummer(10_000, 10)
    a = gpu_build(pos, m)
    a.set_velocities(to_dev(vel))
    a.compute_forces(0.75, 0.01, want=False)
    for _ in range(2):
        a.leapfrog_step(1 / 64)
    x, v = a.get_positions()
    b = gpu_build(x.cpu().numpy(), m)
    b.set_velocities(v)
    b.compute_forces(0.75, 0.01, want=False)
    for _ in range(2):
        a.leapfrog_step(1 / 64)
        b.leapfrog_step(1 / 64)
    xa, va, aa, pa = _state(a)
    xb, vb, ab, pb = _state(b)
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    assert np.array_equal(aa, ab) and np.array_equal(pa, pb)


def test_error_paths():
    import torch

    import paper_1106_1900_amd as bh
    from paper_1106_1900_amd.binding import BH_EINVAL, BH_ESTATE
    pos, vel, m = workloads.plummer(1000, 11)
    ctx = bh.Context()
    with pytest.raises(bh.BHError) as e:
        ctx.compute_forces(0.5, 0.01)
    assert e.value.code == BH_ESTATE
    bad = pos.copy()
    bad[17, 1] = np.nan
    with pytest.raises(bh.BHError) as e:
        ctx.build_tree(to_dev(bad), to_dev(m))
    assert e.value.code == BH_EINVAL
    bad = pos.copy()
    bad[3, 0] = np.inf
    with pytest.raises(bh.BHError) as e:
        ctx.build_tree(to_dev(bad), to_dev(m))
    assert e.value.code == BH_EINVAL
    mm = m.copy()
    mm[5] = 0.0
    with pytest.raises(bh.BHError) as e:
        ctx.build_tree(to_dev(pos), to_dev(mm))
    assert e.value.code == BH_EINVAL
    with pytest.raises(bh.BHError) as e:
        ctx.build_tree(to_dev(pos[:0].copy()), to_dev(m[:0].copy()))
    assert e.value.code == BH_EINVAL
    ctx.build_tree(to_dev(pos), to_dev(m))
    with pytest.raises(bh.BHError) as e:
        ctx.leapfrog_step(0.01)
    assert e.value.code == BH_ESTATE
    for theta, eps in ((0.0, 0.01), (1.5, 0.01), (0.5, -1.0), (float("nan"), 0.01),
                       (0.5, float("inf"))):
        with pytest.raises(bh.BHError) as e:
            ctx.compute_forces(theta, eps)
        assert e.value.code == BH_EINVAL
    # the context still works after the errors
    acc, pot = ctx.compute_forces(0.5, 0.01)
    assert torch.isfinite(acc).all() and torch.isfinite(pot).all()
    ctx.close()


def test_memory_budget_is_enforced():
    import paper_1106_1900_amd as bh
    from paper_1106_1900_amd.binding import BH_ENOMEM
    pos, _, m = workloads.plummer(50_000, 12)
    ctx = bh.Context(hbm_budget_bytes=1 << 20)
    with pytest.raises(bh.BHError) as e:
        ctx.build_tree(to_dev(pos), to_dev(m))
    assert e.value.code == BH_ENOMEM
    ctx.close()
    ctx = bh.Context(hbm_budget_bytes=1 << 30)
    ctx.build_tree(to_dev(pos), to_dev(m))
    assert ctx.stats().device_bytes <= 1 << 30
    ctx.close()


def test_rebuild_orders_equal_keys_by_caller_index():
    # App. A: the split primitive keeps the input order, so equal keys keep
    # caller order.  set_state rebuilds from the particles the context holds;
    # particles moved onto one point (one level-20 key) must come out in caller
    # order whatever their order in the previous tree
    n = 6000
    pos, vel, m = workloads.plummer(n, 12)
    ctx = gpu_build(pos, m)
    perm0 = ctx.export_tree()["perm"]
    rank = np.empty_like(perm0)
    rank[perm0] = np.arange(n)
    new = pos.copy()
    reversed_pairs = 0
    for a in range(0, n - 1, 2):
        b = a + 1
        new[b] = new[a]                      # b joins a on one key
        reversed_pairs += int(rank[b] < rank[a])
    new[n - 100:] = new[n - 101]             # a run of 101 coincident particles
    say("case ties", n, "pairs placed before their partner", reversed_pairs)
    assert reversed_pairs > 1000
    ctx.set_state(to_dev(new), to_dev(vel))
    acc, pot = ctx.compute_forces(0.6, 0.01)
    ex = ctx.export_tree()
    t = oracle.Tree(new, m)
    compare_tree(ex, t)                      # keys, perm (caller order on ties), cells, groups
    compare_walk(ex, t, 0.6)
    compare_forces(acc.cpu().numpy(), pot.cpu().numpy(), t, 0.6, 0.01)
    ctx.close()
