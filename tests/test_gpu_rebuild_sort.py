"""GPU tests of the sort of a rebuild (App. A: keys sorted with equal keys in
caller order).  A single system rebuilt from the particles it holds is sorted
through buckets split at keys of the previous order, each bucket sorted in LDS (or,
when larger than that holds, by stable passes of its own); the order must equal
the oracle's stable sort bit for bit whatever the bucket sizes."""

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import compare_tree, compare_walk, gpu_build, say, to_dev

pytestmark = pytest.mark.gpu


def _order_equal(ctx, pos, m):
    ex = ctx.export_tree()
    perm, key = oracle.Tree(pos, m).order()
    assert np.array_equal(ex["key"], key), "keys differ"
    assert np.array_equal(ex["perm"], perm), "sorted order differs"


def test_plummer_1m_rebuilds_after_steps():
    # the headline system: every leapfrog step rebuilds from the held order
    n = 1 << 20
    pos, vel, m = workloads.plummer(n, 2)
    say("case rebuild-sort plummer-1M")
    ctx = gpu_build(pos, m)
    ctx.set_velocities(to_dev(vel))
    ctx.compute_forces(0.75, 1 / 64, want=False)
    for _ in range(2):
        ctx.leapfrog_step(1 / 64)
    x = ctx.get_state()[0]
    _order_equal(ctx, x.cpu().numpy(), m)
    ctx.close()


@pytest.mark.parametrize("n", [1 << 20, (1 << 20) + 1])
def test_bucket_count_limit(n):
    # 2^20 particles take 256 buckets of 4096 on average; one more takes the
    # radix sort: both rebuilds give the oracle's order
    pos, vel, m = workloads.plummer(n, 9)
    say("case rebuild-sort limit", n)
    ctx = gpu_build(pos, m)
    new = pos + 1e-3 * vel
    ctx.set_state(to_dev(new), to_dev(vel))
    ctx.compute_forces(0.75, 1 / 64, want=False)
    _order_equal(ctx, new, m)
    ctx.close()


@pytest.mark.parametrize("ncoin", [10_000, 16_000])
def test_large_buckets_of_equal_keys(ncoin):
    # ncoin of 30,000 particles moved onto one point: one key, one bucket of 8,192
    # to 12,288 pairs (the largest sorted in LDS) or of more (sorted by the
    # bucket's workgroup through device memory); ties in caller order
    n = 30_000
    pos, vel, m = workloads.plummer(n, 21)
    ctx = gpu_build(pos, m)
    new = pos.copy()
    rng = np.random.default_rng(5)
    sel = rng.choice(n, ncoin, replace=False)
    new[sel] = new[sel[0]]
    say("case rebuild-sort large bucket", ncoin)
    ctx.set_state(to_dev(new), to_dev(vel))
    ctx.compute_forces(0.6, 0.01, want=False)
    ex = ctx.export_tree()
    t = oracle.Tree(new, m)
    compare_tree(ex, t)
    compare_walk(ex, t, 0.6)
    ctx.close()


def test_held_order_unrelated_to_new_keys():
    # positions replaced by a random permutation of themselves: the held order
    # says nothing about the new keys, buckets come out uneven (some above the
    # LDS capacity), the order must still be exact
    n = 200_000
    pos, vel, m = workloads.plummer(n, 33)
    ctx = gpu_build(pos, m)
    rng = np.random.default_rng(8)
    p = rng.permutation(n)
    new = pos[p]
    say("case rebuild-sort random order")
    ctx.set_state(to_dev(new), to_dev(vel))
    ctx.compute_forces(0.75, 1 / 64, want=False)
    _order_equal(ctx, new, m)
    ctx.close()


@pytest.mark.parametrize("n", [2, 3, 65, 4096, 4097, 8193])
def test_small_rebuilds(n):
    # one bucket (n <= 4096) up to three; the bucket sort's padding to a power of two
    pos, vel, m = workloads.plummer(n, 40 + n)
    ctx = gpu_build(pos, m, nleaf=8, ncrit=16)
    new = pos + 0.05 * vel
    say("case rebuild-sort small", n)
    ctx.set_state(to_dev(new), to_dev(vel))
    ctx.compute_forces(0.6, 0.01, want=False)
    ex = ctx.export_tree()
    t = oracle.Tree(new, m, nleaf=8, ncrit=16)
    compare_tree(ex, t)
    ctx.close()
