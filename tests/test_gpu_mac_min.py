"""GPU parity of the minimum-distance opening test (the alternative of Sect. 3.3):
the HIP walk with BH_MAC_MIN_DIST against the oracle tree with mac=1, bit for bit
in the opening radii and interaction counts, within the stated tolerances in the
forces; the test per cluster in a batch, through graph replays and through the
serving loop; switching the test back and forth."""

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import compare_forces, compare_tree, compare_walk, say, split_forest, to_dev

pytestmark = pytest.mark.gpu


def _ctx(pos, mass, nleaf=16, ncrit=64, mac=1):
    import paper_1106_1900_amd as bh
    ctx = bh.Context(nleaf=nleaf, ncrit=ncrit)
    ctx.set_mac(mac)
    ctx.build_tree(to_dev(pos), to_dev(mass))
    return ctx


def _check(pos, mass, theta, eps, nleaf=16, ncrit=64, label="", groups=None):
    import torch
    say("case min-mac", label, "n", pos.shape[0], "theta", theta, "eps", eps, nleaf, ncrit)
    ctx = _ctx(pos, mass, nleaf, ncrit)
    acc, pot = ctx.compute_forces(theta, eps)
    torch.cuda.synchronize()
    ex = ctx.export_tree()
    t = oracle.Tree(pos, mass, nleaf, ncrit, mac=1)
    compare_tree(ex, t)
    compare_walk(ex, t, theta)
    compare_forces(acc.cpu().numpy(), pot.cpu().numpy(), t, theta, eps, groups)
    st = ctx.stats()
    ctx.close()
    return ex, t, st


@pytest.mark.parametrize("name,n,seed,theta,eps,nleaf,ncrit", [
    ("plummer", 4096, 1, 0.5, 0.01, 16, 64),
    ("plummer", 30000, 51, 0.75, 1 / 64, 16, 64),
    ("clustered", 20000, 52, 0.75, 0.005, 8, 32),
    ("cube", 5000, 53, 0.4, 0.0, 16, 16),
    ("plummer", 3000, 54, 1.0, 0.01, 32, 64),
])
def test_min_mac_matches_oracle(name, n, seed, theta, eps, nleaf, ncrit):
    gen = {"plummer": workloads.plummer, "clustered": workloads.clustered,
           "cube": workloads.uniform_cube}[name]
    pos, _, m = gen(n, seed)
    _check(pos, m, theta, eps, nleaf, ncrit, label=name)


@pytest.mark.parametrize("n", [1, 2, 17, 65])
def test_min_mac_tiny_systems(n):
    pos, _, m = workloads.plummer(n, 55)
    if n == 1:
        import torch
        ctx = _ctx(pos, m)
        acc, pot = ctx.compute_forces(0.5, 0.01)
        torch.cuda.synchronize()
        assert np.all(acc.cpu().numpy() == 0) and np.all(pot.cpu().numpy() == 0)
        ctx.close()
        return
    _check(pos, m, 0.5, 0.01, label="tiny")


def test_min_mac_plummer_1m_full_size():
    # the headline workload with the minimum-distance test: tree and all counts
    # bit-exact, forces on a seeded sample of groups
    n = 1 << 20
    pos, _, m = workloads.plummer(n, 2)
    rng = np.random.default_rng(17)
    t = oracle.Tree(pos, m, mac=1)
    groups = np.sort(rng.choice(t.ngroups, 200, replace=False))
    del t
    _check(pos, m, 0.75, 1 / 64, label="plummer-1M", groups=groups)


def test_switching_the_test_back_and_forth():
    import torch
    import paper_1106_1900_amd as bh
    pos, _, m = workloads.plummer(8000, 56)
    ctx = _ctx(pos, m, mac=bh.MAC_EQ1)
    a0, p0 = [x.cpu().numpy() for x in ctx.compute_forces(0.6, 0.01)]
    ctx.set_mac(bh.MAC_MIN_DIST)
    a1, p1 = ctx.compute_forces(0.6, 0.01)
    torch.cuda.synchronize()
    t1 = oracle.Tree(pos, m, mac=1)
    compare_walk(ctx.export_tree(), t1, 0.6)
    compare_forces(a1.cpu().numpy(), p1.cpu().numpy(), t1, 0.6, 0.01)
    ctx.set_mac(bh.MAC_EQ1)
    a2, p2 = [x.cpu().numpy() for x in ctx.compute_forces(0.6, 0.01)]
    assert np.array_equal(a0, a2) and np.array_equal(p0, p2)
    compare_walk(ctx.export_tree(), oracle.Tree(pos, m), 0.6)
    with pytest.raises(bh.BHError):
        ctx.set_mac(2)
    ctx.close()


def _mixed():
    parts = []
    p, v, m = workloads.plummer(6000, 57)
    parts.append((p, v, m, dict(theta=0.6, eps=0.01, nleaf=16, ncrit=64, mac=1)))
    p, v, m = workloads.plummer(4000, 58)
    parts.append((p, v, m, dict(theta=0.6, eps=0.01, nleaf=16, ncrit=64, mac=0)))
    p, v, m = workloads.clustered(3000, 59)
    parts.append((p, v, m, dict(theta=0.8, eps=0.0, nleaf=8, ncrit=32, mac=1)))
    return parts


def test_mixed_tests_in_one_batch():
    import torch
    import paper_1106_1900_amd as bh
    parts = _mixed()
    pos = np.concatenate([q[0] for q in parts])
    vel = np.concatenate([q[1] for q in parts])
    mass = np.concatenate([q[2] for q in parts])
    clusters = [dict(n=q[0].shape[0], dt=1 / 128, **q[3]) for q in parts]
    ctx = bh.Context()
    ctx.batch_build(clusters, to_dev(pos), to_dev(mass), to_dev(vel))
    acc, pot = ctx.batch_forces()
    torch.cuda.synchronize()
    views = split_forest(ctx.export_tree(), [q["n"] for q in clusters])
    a, p = acc.cpu().numpy(), pot.cpu().numpy()
    first = 0
    for (cp, _, cm, prm), d in zip(parts, views):
        n = cp.shape[0]
        say("cluster", n, prm)
        t = oracle.Tree(cp, cm, prm["nleaf"], prm["ncrit"], mac=prm["mac"])
        compare_tree(d, t)
        compare_walk(d, t, prm["theta"])
        compare_forces(a[first:first + n], p[first:first + n], t, prm["theta"], prm["eps"])
        first += n
    # graph replays against eager steps of an identical batch
    e = bh.Context()
    e.batch_build(clusters, to_dev(pos), to_dev(mass), to_dev(vel))
    e.batch_forces(want=False)
    for step in range(3):
        ctx.batch_run(1)
        e.leapfrog_step(1 / 128)
        for x, y in zip(ctx.get_state(), e.get_state()):
            assert np.array_equal(x.cpu().numpy(), y.cpu().numpy()), ("replay", step)
    bad = [dict(q) for q in clusters]
    bad[1]["mac"] = 5
    with pytest.raises(bh.BHError):
        e.batch_set_params(bad)
    ctx.close()
    e.close()


def test_min_mac_error_and_cost_against_eq1():
    # Sect. 3.3: at the same theta the minimum-distance test costs more
    # interactions and gives a smaller acceleration error than Eq. (1)
    import torch
    pos, _, m = workloads.plummer(4096, 1)
    ad, _ = oracle.direct(pos, m, 0.01)
    res = []
    for mac in (0, 1):
        ctx = _ctx(pos, m, mac=mac)
        acc, _ = ctx.compute_forces(0.75, 0.01)
        torch.cuda.synchronize()
        st = ctx.stats()
        a = acc.cpu().numpy().astype(np.float64)
        err = np.linalg.norm(a - ad, axis=1) / np.linalg.norm(ad, axis=1)
        res.append((st.sum_npp + st.sum_npc, np.median(err), np.percentile(err, 99)))
        ctx.close()
    say("eq1 vs min-dist (interactions, median, p99):", res)
    assert res[1][0] > res[0][0]
    assert res[1][1] < res[0][1] and res[1][2] < res[0][2]


def test_served_request_with_min_mac_equals_alone():
    import torch
    import paper_1106_1900_amd as bh
    reqs = []
    for i, (n, mac) in enumerate(((5000, 1), (3000, 0), (2000, 1))):
        p, v, m = workloads.plummer(n, 60 + i)
        reqs.append(dict(pos=p, vel=v, mass=m, theta=0.6, eps=0.01, dt=1 / 128, nsteps=2, mac=mac))
    srv = bh.Server(1 << 30, max_requests=8)
    outs, tickets = [], []
    for q in reqs:
        n = q["pos"].shape[0]
        o = (torch.empty((n, 3), dtype=torch.float64, device="cuda"),
             torch.empty((n, 3), dtype=torch.float64, device="cuda"),
             torch.empty((n, 3), dtype=torch.float32, device="cuda"),
             torch.empty((n,), dtype=torch.float32, device="cuda"))
        tickets.append(srv.submit(to_dev(q["pos"]), to_dev(q["mass"]), to_dev(q["vel"]), q["theta"],
                                  q["eps"], q["dt"], q["nsteps"], out_pos=o[0], out_vel=o[1],
                                  out_acc=o[2], out_pot=o[3], mac=q["mac"]))
        outs.append(o)
    it = 0
    while any(srv.poll(t)["state"] < 2 for t in tickets):
        srv.step()
        it += 1
        assert it < 50
    torch.cuda.synchronize()
    for q, o, t in zip(reqs, outs, tickets):
        assert srv.poll(t)["state"] == 2
        ctx = _ctx(q["pos"], q["mass"], mac=q["mac"])
        ctx.set_velocities(to_dev(q["vel"]))
        ctx.compute_forces(q["theta"], q["eps"], want=False)
        for _ in range(q["nsteps"]):
            ctx.leapfrog_step(q["dt"])
        ref = [x.cpu().numpy() for x in ctx.get_state()]
        for a, b in zip(ref, o):
            assert np.array_equal(a, b.cpu().numpy()), ("served", q["pos"].shape[0], q["mac"])
        ctx.close()
    srv.close()
