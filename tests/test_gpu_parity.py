"""GPU parity: the HIP path through the C ABI against the oracle on the same seeded
inputs.  Keys, sorted order, cells, groups, centres of mass, opening radii and
interaction counts must be identical; forces must agree within the stated
tolerances (tests/gpu_helpers.py)."""

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import (compare_forces, compare_tree, compare_walk, gpu_build, host_threads, say,
                         to_dev)

pytestmark = pytest.mark.gpu


def _case(name, n, seed):
    if name == "plummer":
        return workloads.plummer(n, seed)
    if name == "clustered":
        return workloads.clustered(n, seed)
    if name == "line":
        return workloads.on_a_line(n, seed)
    if name == "cube":
        return workloads.uniform_cube(n, seed)
    if name == "coincident":
        return workloads.coincident(n)
    if name == "lattice":
        return workloads.lattice(int(round(n ** (1 / 3))))
    raise KeyError(name)


def _full_check(pos, mass, theta, eps, nleaf=16, ncrit=64, label=""):
    import torch
    say("case", label, "n", pos.shape[0], "theta", theta, "eps", eps, "nleaf", nleaf, "ncrit", ncrit)
    ctx = gpu_build(pos, mass, nleaf, ncrit)
    acc, pot = ctx.compute_forces(theta, eps)
    torch.cuda.synchronize()
    ex = ctx.export_tree()
    t = oracle.Tree(pos, mass, nleaf, ncrit)
    compare_tree(ex, t)
    compare_walk(ex, t, theta)
    compare_forces(acc.cpu().numpy(), pot.cpu().numpy(), t, theta, eps)
    ctx.close()
    return ex, t


def test_plummer_4096_small_workload():
    # theta 0.5, eps 0.01, leaf 16, group 64, and the error bound vs direct sum
    pos, _, m = workloads.plummer(4096, 1)
    _full_check(pos, m, 0.5, 0.01, label="plummer-4096")
    import torch
    ctx = gpu_build(pos, m)
    acc, _ = ctx.compute_forces(0.5, 0.01)
    ad, _ = oracle.direct(pos, m, 0.01)
    a = acc.cpu().numpy().astype(np.float64)
    err = np.linalg.norm(a - ad, axis=1) / np.linalg.norm(ad, axis=1)
    say("plummer-4096 vs direct: median", np.median(err), "p99", np.percentile(err, 99))
    assert np.median(err) <= 1e-3 and np.percentile(err, 99) <= 1e-2


@pytest.mark.parametrize("name,n,seed,theta,eps", [
    ("plummer", 100_003, 21, 0.75, 1 / 64),     # many tiles and a ragged tail
    ("clustered", 20_000, 22, 0.5, 1e-3),
    ("line", 5_000, 23, 0.6, 0.01),
    ("cube", 30_001, 24, 0.9, 0.0),             # eps = 0
    ("lattice", 4_096, 0, 0.5, 0.05),           # ties in the opening test geometry
    ("coincident", 1_000, 0, 0.5, 0.01),        # one chain down to a 1000-particle leaf
])
def test_structured_inputs(name, n, seed, theta, eps):
    pos, _, m = _case(name, n, seed)
    _full_check(pos, m, theta, eps, label=name)


@pytest.mark.parametrize("nleaf,ncrit", [(8, 32), (32, 64), (1, 1), (16, 16), (4, 64),
                                         # groups of 65..128 particles: two per lane
                                         (16, 128), (32, 128), (64, 100), (8, 65)])
def test_leaf_and_group_sizes(nleaf, ncrit):
    pos, _, m = workloads.plummer(8_191, 5)
    _full_check(pos, m, 0.6, 0.02, nleaf, ncrit, label="sizes")


def test_large_leaf_cut_into_groups_of_128():
    # 1000 coincident particles: one level-20 leaf cut into runs of 128
    pos, _, m = workloads.coincident(1_000)
    _full_check(pos, m, 0.5, 0.01, 16, 128, label="coincident-128")


@pytest.mark.parametrize("n", [1, 2, 3, 16, 17, 64, 65, 257])
def test_tiny_systems(n):
    pos, _, m = workloads.plummer(n, 100 + n)
    _full_check(pos, m, 0.5, 0.01, label="tiny")


def test_two_body_closed_form():
    import torch
    pos, _, m = workloads.two_body(sep=0.7, m1=0.3, m2=1.1)
    ctx = gpu_build(pos, m)
    acc, pot = ctx.compute_forces(0.5, 0.05)
    a = acc.cpu().numpy()
    e = np.float32(0.05)
    s = 0.7 ** 2 + float(e) ** 2
    assert a[0, 0] == pytest.approx(1.1 * 0.7 / s ** 1.5, rel=1e-6)
    assert a[1, 0] == pytest.approx(-0.3 * 0.7 / s ** 1.5, rel=1e-6)
    assert pot.cpu().numpy()[0] == pytest.approx(-1.1 / np.sqrt(s), rel=1e-6)


def test_tiny_theta_is_direct_summation():
    pos, _, m = workloads.plummer(700, 30)
    ex, t = _full_check(pos, m, 1e-6, 0.01, label="theta->0")
    assert np.all(ex["npc"] == 0) and np.all(ex["npp"] == 700)


def test_repeat_runs_are_bitwise_identical():
    import torch
    pos, _, m = workloads.plummer(50_000, 31)
    outs = []
    for _ in range(2):
        ctx = gpu_build(pos, m)
        acc, pot = ctx.compute_forces(0.75, 0.01)
        outs.append((acc.cpu().numpy(), pot.cpu().numpy()))
        ctx.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_plummer_1m_full_size():
    # the headline workload: N = 2^20, theta 0.75, eps 1/64.  Tree and all counts
    # bit-exact; the forces of every particle against the oracle's (evaluated on
    # the host's cores).
    import torch
    n = 1 << 20
    pos, _, m = workloads.plummer(n, 2)
    say("case plummer-1M")
    ctx = gpu_build(pos, m)
    acc, pot = ctx.compute_forces(0.75, 1 / 64)
    torch.cuda.synchronize()
    ex = ctx.export_tree()
    t = oracle.Tree(pos, m)
    compare_tree(ex, t)
    compare_walk(ex, t, 0.75)
    say("oracle forces of all", t.ngroups, "groups on", host_threads(), "threads")
    compare_forces(acc.cpu().numpy(), pot.cpu().numpy(), t, 0.75, 1 / 64, threads=host_threads())


def test_small_opening_angle_deep_stack():
    # theta = 0.15 opens many nodes per level: long interaction lists and a deep
    # walk stack
    pos, _, m = workloads.plummer(60_000, 41)
    _full_check(pos, m, 0.15, 0.01, label="theta-0.15")


def test_galaxy_4m_full_size():
    # three-component galaxy, N = 4,194,304, theta 0.4, eps 0.02: tree and all
    # counts bit-exact, forces on sampled groups against the oracle, and the error
    # against float64 direct summation on seeded targets
    import torch
    pos, _, m = workloads.galaxy(seed=3)
    say("case galaxy-4M")
    ctx = gpu_build(pos, m)
    acc, pot = ctx.compute_forces(0.4, 0.02)
    torch.cuda.synchronize()
    ex = ctx.export_tree()
    t = oracle.Tree(pos, m)
    compare_tree(ex, t)
    compare_walk(ex, t, 0.4)
    rng = np.random.default_rng(13)
    groups = np.sort(rng.choice(t.ngroups, 4000, replace=False))
    a = acc.cpu().numpy()
    compare_forces(a, pot.cpu().numpy(), t, 0.4, 0.02, groups, threads=host_threads())
    tgt = np.sort(rng.choice(pos.shape[0], 1024, replace=False))
    ad, _ = oracle.direct(pos, m, 0.02, tgt, threads=host_threads())
    err = np.linalg.norm(a[tgt].astype(np.float64) - ad, axis=1) / np.linalg.norm(ad, axis=1)
    say("galaxy-4M vs direct: median", np.median(err), "p99", np.percentile(err, 99))
    assert np.median(err) <= 1e-3 and np.percentile(err, 99) <= 1e-2
    ctx.close()
