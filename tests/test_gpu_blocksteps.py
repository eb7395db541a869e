"""GPU tests of the between-rebuild operations (Sect. 5: block time-steps need
new forces only for active particles, and between rebuilds it suffices to
recompute the multipole moments): drift without rebuild, multipole-only refit
against the oracle's refit, the active-group walk against the full walk, and a
drift-refit-forces-kick cycle against the oracle."""

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import compare_forces, compare_tree, compare_walk, gpu_build, say, to_dev

pytestmark = pytest.mark.gpu


def _drifted(pos, vel, dt):
    return pos + vel * dt          # the same float64 operations as the device drift


@pytest.mark.parametrize("dt,mac", [(1 / 64, 0), (1 / 8, 0), (1 / 8, 1), (1 / 2, 0), (1 / 2, 1)])
def test_refit_matches_the_oracle_refit(dt, mac):
    # three drifts, then a refit: moments, boxes, the opening geometry of every
    # cell (kept where the particles stayed in their key cell, else the tight
    # box's centre and grown side), counts and forces against the oracle's refit
    import torch
    pos, vel, m = workloads.plummer(30_000, 51)
    theta, eps = 0.6, 0.01
    say("case refit", pos.shape[0], dt, "mac", mac)
    ctx = gpu_build(pos, m, 16, 64)
    ctx.set_mac(mac)
    ctx.set_velocities(to_dev(vel))
    ctx.compute_forces(theta, eps, want=False)
    for _ in range(3):
        ctx.drift(dt)
    x = pos
    for _ in range(3):
        x = _drifted(x, vel, dt)
    gx, _ = ctx.get_positions()
    assert np.array_equal(gx.cpu().numpy(), x)
    ctx.refit()
    acc, pot = ctx.compute_forces(theta, eps)
    torch.cuda.synchronize()
    ex = ctx.export_tree()
    t = oracle.Tree(pos, m, 16, 64, mac=mac)
    t.refit(x)
    compare_tree(ex, t)           # the build's keys and cells, the refit's moments and boxes
    compare_walk(ex, t, theta)
    compare_forces(acc.cpu().numpy(), pot.cpu().numpy(), t, theta, eps)
    ctx.close()


def test_forces_refused_after_a_drift_until_refit():
    from paper_1106_1900_amd.binding import BH_ESTATE

    import paper_1106_1900_amd as bh
    pos, vel, m = workloads.plummer(2000, 52)
    ctx = gpu_build(pos, m)
    ctx.set_velocities(to_dev(vel))
    ctx.compute_forces(0.5, 0.01, want=False)
    ctx.drift(0.01)
    for call in (lambda: ctx.compute_forces(0.5, 0.01),
                 lambda: ctx.compute_forces_active(0.5, 0.01, to_dev(np.ones(2000, np.uint8)))):
        with pytest.raises(bh.BHError) as e:
            call()
        assert e.value.code == BH_ESTATE
    ctx.refit()
    ctx.compute_forces(0.5, 0.01)
    ctx.close()


def _group_of_particles(ex):
    """Caller index -> group index, from the exported groups and sorted order."""
    n = ex["perm"].shape[0]
    g = np.zeros(n, np.int64)
    for k, (f, c) in enumerate(zip(ex["gfirst"], ex["gcount"])):
        g[ex["perm"][f:f + c]] = k
    return g


@pytest.mark.parametrize("frac", [0.001, 0.05, 0.5])
def test_active_walk_equals_the_full_walk_on_active_groups(frac):
    import torch
    pos, _, m = workloads.plummer(50_000, 53)
    n = pos.shape[0]
    say("case active", frac)
    ctx = gpu_build(pos, m)
    a1, p1 = ctx.compute_forces(0.7, 0.01)        # the values inactive particles keep
    a1, p1 = a1.cpu().numpy(), p1.cpu().numpy()
    ref = gpu_build(pos, m)
    a2, p2 = ref.compute_forces(0.5, 0.01)        # full walk at the new opening angle
    a2, p2 = a2.cpu().numpy(), p2.cpu().numpy()
    ex2 = ref.export_tree()
    rng = np.random.default_rng(54)
    active = (rng.uniform(size=n) < frac).astype(np.uint8)
    aa, pa = ctx.compute_forces_active(0.5, 0.01, to_dev(active))
    torch.cuda.synchronize()
    aa, pa = aa.cpu().numpy(), pa.cpu().numpy()
    grp = _group_of_particles(ex2)
    hot = np.zeros(len(ex2["gfirst"]), bool)
    hot[grp[active != 0]] = True
    sel = hot[grp]                                 # particles of groups with an active one
    assert sel.sum() >= active.sum()
    assert np.array_equal(aa[sel], a2[sel]) and np.array_equal(pa[sel], p2[sel])
    assert np.array_equal(aa[~sel], a1[~sel]) and np.array_equal(pa[~sel], p1[~sel])
    ex = ctx.export_tree()
    assert np.array_equal(ex["npp"][hot], ex2["npp"][hot])
    assert np.array_equal(ex["npc"][hot], ex2["npc"][hot])
    ctx.close()
    ref.close()


def test_block_step_cycle_against_the_oracle():
    # one cycle of a two-level scheme: drift everything by dt, refit, new forces for
    # the active half, kick the active particles by dt
    import torch
    pos, vel, m = workloads.plummer(20_000, 55)
    n = pos.shape[0]
    theta, eps, dt = 0.6, 0.01, 1 / 128
    ctx = gpu_build(pos, m)
    ctx.set_velocities(to_dev(vel))
    a0, p0 = ctx.compute_forces(theta, eps)
    a0, p0 = a0.cpu().numpy(), p0.cpu().numpy()
    active = (np.random.default_rng(56).uniform(size=n) < 0.5).astype(np.uint8)
    ctx.drift(dt)
    ctx.refit()
    acc, pot = ctx.compute_forces_active(theta, eps, to_dev(active))
    ctx.kick(dt, to_dev(active))
    torch.cuda.synchronize()
    x1, v1 = [t.cpu().numpy() for t in ctx.get_positions()]
    acc, pot = acc.cpu().numpy(), pot.cpu().numpy()
    xe = _drifted(pos, vel, dt)
    assert np.array_equal(x1, xe)
    t = oracle.Tree(pos, m)
    t.refit(xe)
    ex = ctx.export_tree()
    grp = _group_of_particles(ex)
    hot = np.zeros(len(ex["gfirst"]), bool)
    hot[grp[active != 0]] = True
    sel = hot[grp]
    oa, op, aabs, pabs = t.forces(theta, eps, np.nonzero(hot)[0])
    da = np.linalg.norm(acc[sel].astype(np.float64) - oa[sel], axis=1)
    assert np.all(da <= 1e-5 * aabs[sel])
    assert np.array_equal(acc[~sel], a0[~sel])
    # kicks: active particles with their new accelerations, the others unchanged
    on = active != 0
    assert np.array_equal(v1[on], vel[on] + acc[on].astype(np.float64) * dt)
    assert np.array_equal(v1[~on], vel[~on])
    ctx.close()
