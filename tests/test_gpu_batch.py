"""GPU tests of batches (K independent clusters in one context): every cluster of
a forest matches the oracle tree of that cluster alone, bit for bit in its
discrete parts; a cluster's forces in a batch are bit-identical to its forces
built alone; the captured step replayed as a graph matches the eager step bit for
bit, replay after replay; per-cluster time steps and energies."""

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import compare_forces, compare_tree, compare_walk, say, split_forest, to_dev

pytestmark = pytest.mark.gpu


def _mixed_batch():
    """Clusters of different shapes, sizes and parameters, including the
    degenerate one-particle and two-particle systems."""
    parts = []
    p, v, m = workloads.plummer(3000, 21)
    parts.append((p, v, m, dict(theta=0.5, eps=0.01, nleaf=16, ncrit=64)))
    p, v, m = workloads.uniform_cube(700, 22)
    parts.append((p, v, m, dict(theta=0.75, eps=0.02, nleaf=8, ncrit=32)))
    p, v, m = workloads.clustered(5000, 23)
    parts.append((p, v, m, dict(theta=0.6, eps=0.005, nleaf=32, ncrit=16)))
    p, v, m = workloads.two_body()
    parts.append((p, v, m, dict(theta=0.9, eps=0.0, nleaf=1, ncrit=1)))
    parts.append((np.array([[0.3, -0.2, 0.1]]), np.zeros((1, 3)), np.array([0.5]),
                  dict(theta=0.7, eps=0.01, nleaf=16, ncrit=64)))
    p, v, m = workloads.plummer(9000, 24)
    parts.append((p, v, m, dict(theta=0.4, eps=0.0, nleaf=16, ncrit=64)))
    # groups of up to 128 particles (the batched configuration's largest size)
    p, v, m = workloads.plummer(6000, 25)
    parts.append((p, v, m, dict(theta=0.75, eps=0.01, nleaf=32, ncrit=128)))
    p, v, m = workloads.clustered(4000, 26)
    parts.append((p, v, m, dict(theta=0.5, eps=0.005, nleaf=8, ncrit=128)))
    return parts


def _concat(parts):
    pos = np.concatenate([q[0] for q in parts])
    vel = np.concatenate([q[1] for q in parts])
    mass = np.concatenate([q[2] for q in parts])
    clusters = [dict(n=q[0].shape[0], **q[3]) for q in parts]
    return pos, vel, mass, clusters


def _batch_ctx(parts, dt=None):
    import paper_1106_1900_amd as bh
    pos, vel, mass, clusters = _concat(parts)
    if dt is not None:
        for q, d in zip(clusters, dt):
            q["dt"] = d
    ctx = bh.Context()
    ctx.batch_build(clusters, to_dev(pos), to_dev(mass), to_dev(vel))
    return ctx, pos, vel, mass, clusters


def test_forest_matches_oracle_per_cluster():
    import torch
    parts = _mixed_batch()
    say("case forest", [q[0].shape[0] for q in parts])
    ctx, pos, vel, mass, clusters = _batch_ctx(parts)
    acc, pot = ctx.batch_forces()
    torch.cuda.synchronize()
    ex = ctx.export_tree()
    st = ctx.stats()
    assert st.nclusters == len(parts)
    sizes = [q["n"] for q in clusters]
    views = split_forest(ex, sizes)
    # the roots of the forest are cells 0..K-1, in cluster order
    assert np.array_equal(ex["level"][:len(parts)], np.zeros(len(parts)))
    assert np.array_equal(ex["first"][:len(parts)], np.cumsum([0] + sizes[:-1]))
    a = acc.cpu().numpy()
    p = pot.cpu().numpy()
    first = 0
    for (cp, _, cm, prm), d in zip(parts, views):
        n = cp.shape[0]
        say("cluster", n, prm)
        t = oracle.Tree(cp, cm, prm["nleaf"], prm["ncrit"])
        compare_tree(d, t)
        compare_walk(d, t, prm["theta"])
        if n > 1:
            compare_forces(a[first:first + n], p[first:first + n], t, prm["theta"], prm["eps"])
        else:
            assert np.all(a[first] == 0.0) and p[first] == 0.0
        first += n
    assert sum(int(v.shape[0]) for v in (d["gfirst"] for d in views)) == st.ngroups
    ctx.close()


def test_cluster_in_batch_equals_cluster_alone():
    import paper_1106_1900_amd as bh
    import torch
    parts = _mixed_batch()
    ctx, pos, vel, mass, clusters = _batch_ctx(parts)
    acc, pot = ctx.batch_forces()
    torch.cuda.synchronize()
    a = acc.cpu().numpy()
    p = pot.cpu().numpy()
    first = 0
    for cp, cv, cm, prm in parts:
        n = cp.shape[0]
        one = bh.Context(nleaf=prm["nleaf"], ncrit=prm["ncrit"])
        one.build_tree(to_dev(cp), to_dev(cm))
        a1, p1 = one.compute_forces(prm["theta"], prm["eps"])
        assert np.array_equal(a1.cpu().numpy(), a[first:first + n]), ("acc", n, prm)
        assert np.array_equal(p1.cpu().numpy(), p[first:first + n]), ("pot", n, prm)
        one.close()
        first += n
    ctx.close()


def _state(ctx):
    x, v, a, p = ctx.get_state()
    return [t.cpu().numpy() for t in (x, v, a, p)]


def test_graph_replays_match_eager_steps():
    # the same batch advanced by eager steps and by graph replays, compared after
    # every step, with synchronisations and other work between the replays
    parts = _mixed_batch()
    dt = 1 / 128
    g, *_ = _batch_ctx(parts, dt=[dt] * len(parts))
    e, *_ = _batch_ctx(parts, dt=[dt] * len(parts))
    g.batch_forces(want=False)
    e.batch_forces(want=False)
    for step in range(5):
        g.batch_run(1)
        e.leapfrog_step(dt)
        sg, se = _state(g), _state(e)
        for a, b, name in zip(sg, se, ("pos", "vel", "acc", "pot")):
            assert np.array_equal(a, b), ("replay", step, name)
        eg, ee = g.batch_energy(), e.batch_energy()
        assert np.array_equal(eg, ee)
    assert g.stats().graph_launches == 5
    # several replays in one call
    g.batch_run(3)
    for _ in range(3):
        e.leapfrog_step(dt)
    for a, b in zip(_state(g), _state(e)):
        assert np.array_equal(a, b)
    g.close()
    e.close()


def test_per_cluster_time_steps():
    # cluster k advances with its own dt; dt = 0 leaves positions and velocities
    # bit for bit and recomputes that cluster's forces
    import paper_1106_1900_amd as bh
    parts = _mixed_batch()
    dts = [1 / 64, 0.0, 1 / 256, 1 / 32, 1 / 128, 0.0]
    ctx, pos, vel, mass, clusters = _batch_ctx(parts, dt=dts)
    ctx.batch_forces(want=False)
    x0, v0, a0, _ = _state(ctx)
    ctx.batch_run(1)
    x1, v1, a1, p1 = _state(ctx)
    first = 0
    for (cp, cv, cm, prm), dt in zip(parts, dts):
        n = cp.shape[0]
        s = slice(first, first + n)
        h = 0.5 * dt
        vh = v0[s] + a0[s].astype(np.float64) * h
        assert np.array_equal(x1[s], x0[s] + vh * dt)
        assert np.array_equal(v1[s], vh + a1[s].astype(np.float64) * h)
        if dt == 0.0:
            assert np.array_equal(x1[s], cp)
            one = bh.Context(nleaf=prm["nleaf"], ncrit=prm["ncrit"])
            one.build_tree(to_dev(cp), to_dev(cm))
            oa, op = one.compute_forces(prm["theta"], prm["eps"])
            assert np.array_equal(oa.cpu().numpy(), a1[s])
            assert np.array_equal(op.cpu().numpy(), p1[s])
            one.close()
        first += n
    # per-cluster energies against float64 sums of the state
    en = ctx.batch_energy()
    first = 0
    for k, (cp, _, cm, _) in enumerate(parts):
        n = cp.shape[0]
        s = slice(first, first + n)
        T = 0.5 * np.sum(cm * np.sum(v1[s] * v1[s], axis=1))
        W = 0.5 * np.sum(cm * p1[s].astype(np.float64))
        assert en[k, 0] == pytest.approx(T, rel=1e-12, abs=1e-300)
        assert en[k, 1] == pytest.approx(W, rel=1e-12, abs=1e-300)
        assert en[k, 6] == 0.0
        first += n
    tot = ctx.energy()
    assert tot[0] == pytest.approx(en[:, 0].sum(), rel=1e-12)
    ctx.close()


def test_batch_errors():
    import paper_1106_1900_amd as bh
    from paper_1106_1900_amd.binding import BH_EINVAL, BH_ESTATE
    parts = _mixed_batch()[:2]
    pos, vel, mass, clusters = _concat(parts)
    ctx = bh.Context()
    with pytest.raises(bh.BHError) as e:
        ctx.batch_run(1)
    assert e.value.code == BH_ESTATE
    for bad in (dict(theta=0.0), dict(theta=1.5), dict(eps=-1.0), dict(nleaf=65),
                dict(ncrit=-1), dict(dt=float("inf"))):
        cl = [dict(q) for q in clusters]
        cl[1].update(bad)
        with pytest.raises(bh.BHError) as e:
            ctx.batch_build(cl, to_dev(pos), to_dev(mass), to_dev(vel))
        assert e.value.code == BH_EINVAL, bad
    ctx.batch_build(clusters, to_dev(pos), to_dev(mass), to_dev(vel))
    with pytest.raises(bh.BHError) as e:
        ctx.batch_run(1)
    assert e.value.code == BH_ESTATE
    cl = [dict(q) for q in clusters]
    cl[0]["nleaf"] = 8
    with pytest.raises(bh.BHError) as e:
        ctx.batch_set_params(cl)
    assert e.value.code == BH_EINVAL
    cl = [dict(q, theta=0.3, dt=1 / 64) for q in clusters]
    ctx.batch_set_params(cl)
    ctx.batch_forces(want=False)
    ctx.batch_run(2)
    assert np.all(np.isfinite(ctx.batch_energy()))
    ctx.close()


def test_autotune_table_and_tuned_build():
    # two classes of cluster (log2 n = 10 and 12 at theta 0.75, plus theta 0.5);
    # the table holds one entry per class with candidates from the grid, and a
    # batch loaded with nleaf = ncrit = 0 takes the tuned values, checked against
    # the oracle tree built with them
    import paper_1106_1900_amd as bh
    import torch
    parts = []
    for i, (n, theta) in enumerate([(1100, 0.75), (1500, 0.75), (4500, 0.75), (6000, 0.75),
                                    (1300, 0.5)]):
        p, v, m = workloads.plummer(n, 40 + i)
        parts.append((p, v, m, dict(theta=theta, eps=0.01, nleaf=16, ncrit=64)))
    pos, vel, mass, clusters = _concat(parts)
    ctx = bh.Context()
    ctx.batch_build(clusters, to_dev(pos), to_dev(mass), to_dev(vel))
    tab = ctx.autotune(reps=2)
    say("tuning", tab)
    got = sorted((t["log2n"], round(t["theta"], 6)) for t in tab)
    assert got == [(10, 0.5), (10, 0.75), (12, 0.75)]
    for t in tab:
        assert t["nleaf"] in (8, 16, 32) and t["ncrit"] in (16, 32, 64)
        assert 0 < t["ms"] <= t["ms_default"]
    zero = [dict(q, nleaf=0, ncrit=0) for q in clusters]
    for c in (ctx, None):
        if c is None:
            c = bh.Context()
            c.set_tuning(tab)
        c.batch_build(zero, to_dev(pos), to_dev(mass), to_dev(vel))
        c.batch_forces(want=False)
        torch.cuda.synchronize()
        views = split_forest(c.export_tree(), [q["n"] for q in clusters])
        for (cp, _, cm, prm), d in zip(parts, views):
            t = [e for e in tab if e["log2n"] == int(np.log2(cp.shape[0]))
                 and abs(e["theta"] - prm["theta"]) < 1e-6][0]
            tree = oracle.Tree(cp, cm, t["nleaf"], t["ncrit"])
            compare_tree(d, tree)
            compare_walk(d, tree, prm["theta"])
        c.close()


def test_batch_512_full_size_sampled_clusters():
    # the full batched workload (512 clusters, 8.8 M particles) through the
    # captured step with dt = 0 (rebuild and forces at the same positions), as the
    # bench runs it; sampled clusters against their oracle trees, and properties
    # of the whole forest
    import paper_1106_1900_amd as bh
    import torch
    cl = workloads.cluster_batch(512, 4)
    sizes = [q["n"] for q in cl]
    say("case batch512", sum(sizes))
    table = [dict(n=q["n"], theta=q["theta"], eps=q["eps"], dt=0.0) for q in cl]
    ctx = bh.Context()
    ctx.batch_build(table, to_dev(np.concatenate([q["pos"] for q in cl])),
                    to_dev(np.concatenate([q["mass"] for q in cl])),
                    to_dev(np.concatenate([q["vel"] for q in cl])))
    ctx.batch_forces(want=False)
    ctx.batch_run(2)
    x, v, a, p = [t.cpu().numpy() for t in ctx.get_state()]
    torch.cuda.synchronize()
    ex = ctx.export_tree()
    K = len(cl)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    assert np.array_equal(ex["level"][:K], np.zeros(K)) and np.array_equal(ex["first"][:K], starts)
    assert np.array_equal(ex["count"][:K], sizes)
    # groups partition every cluster's range and never cross a cluster boundary
    gend = ex["gfirst"] + ex["gcount"]
    assert np.array_equal(ex["gfirst"][1:], gend[:-1]) and gend[-1] == sum(sizes)
    assert np.all(np.searchsorted(starts, ex["gfirst"], "right") ==
                  np.searchsorted(starts, gend - 1, "right"))
    rng = np.random.default_rng(44)
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes))} |
                  set(rng.choice(K, 4, replace=False).tolist()))
    views = split_forest(ex, sizes, pick)
    for c, d in zip(pick, views):
        q = cl[c]
        s = slice(int(starts[c]), int(starts[c] + q["n"]))
        assert np.array_equal(x[s], q["pos"])     # dt = 0 leaves positions as they are
        say("cluster", c, q["n"])
        t = oracle.Tree(q["pos"], q["mass"])
        compare_tree(d, t)
        compare_walk(d, t, q["theta"])
        compare_forces(a[s], p[s], t, q["theta"], q["eps"])
    ctx.close()


def test_replayed_step_after_a_refit_walks_the_rebuilt_tree():
    # a replayed step rebuilds the tree: a refit before it (a block step that
    # only refits) must not leave the next force call with the refitted cells'
    # geometry (the opening radii and counts of the rebuilt tree's own cells)
    import paper_1106_1900_amd as bh
    pos, vel, m = workloads.plummer(20_000, 25)
    theta, eps = 0.6, 0.01
    ctx = bh.Context()
    ctx.build_tree(to_dev(pos), to_dev(m))
    ctx.set_velocities(to_dev(vel))
    ctx.compute_forces(theta, eps, want=False)
    ctx.batch_set_params([dict(n=20_000, theta=theta, eps=eps, dt=1 / 64)])
    ctx.batch_run(2)                         # captures the step of both buffer parities
    assert ctx.stats().graph_captures == 2
    st = ctx.block_step(1 / 16, 0.025, 0.01, 2, 1e9)
    assert st["rebuilt"] == 0                # refitted throughout
    ctx.batch_run(1)                         # a replay, no new capture
    assert ctx.stats().graph_captures == 2
    acc, pot = ctx.compute_forces(theta, eps)
    x, _ = ctx.get_positions()
    t = oracle.Tree(x.cpu().numpy(), m)
    ex = ctx.export_tree()
    compare_tree(ex, t)
    compare_walk(ex, t, theta)
    compare_forces(acc.cpu().numpy(), pot.cpu().numpy(), t, theta, eps)
    ctx.close()
