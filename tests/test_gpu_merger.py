"""GPU tests on the two-galaxy encounter (240,002 bodies, the particle numbers of
the paper's merger test, eps = 0.1): the tree, opening radii and interaction
counts bit for bit against the oracle, forces on sampled groups within the stated
tolerances, and a few graph-replayed leapfrog steps against the oracle's
leapfrog within the bound the float32 forces allow."""

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import compare_forces, compare_tree, compare_walk, say, to_dev

pytestmark = pytest.mark.gpu

EPS, DT = 0.1, 1 / 64


@pytest.mark.parametrize("theta", [0.75, 0.5])
def test_merger_tree_counts_and_forces(theta):
    import torch
    import paper_1106_1900_amd as bh
    pos, vel, m = workloads.merger()
    say("case merger theta", theta)
    ctx = bh.Context()
    ctx.build_tree(to_dev(pos), to_dev(m))
    acc, pot = ctx.compute_forces(theta, EPS)
    torch.cuda.synchronize()
    ex = ctx.export_tree()
    t = oracle.Tree(pos, m)
    compare_tree(ex, t)
    compare_walk(ex, t, theta)
    rng = np.random.default_rng(19)
    groups = np.sort(rng.choice(t.ngroups, 150, replace=False))
    # the black holes' groups too
    perm, _ = t.order()
    g = t.groups()
    for i in workloads.black_holes(pos.shape[0]):
        s = int(np.nonzero(perm == i)[0][0])
        groups = np.union1d(groups, np.nonzero((g["first"] <= s) & (s < g["first"] + g["count"]))[0])
    compare_forces(acc.cpu().numpy(), pot.cpu().numpy(), t, theta, EPS, groups)
    ctx.close()


def test_merger_steps_follow_the_oracle_leapfrog():
    import torch
    import paper_1106_1900_amd as bh
    pos, vel, m = workloads.merger()
    n = pos.shape[0]
    theta, steps = 0.75, 3
    ctx = bh.Context()
    ctx.batch_build([dict(n=n, theta=theta, eps=EPS, dt=DT)], to_dev(pos), to_dev(m), to_dev(vel))
    ctx.batch_forces(want=False)
    e0 = ctx.batch_energy()[0]
    ctx.batch_run(steps)
    x, v, a, _ = [t.cpu().numpy() for t in ctx.get_state()]
    e1 = ctx.batch_energy()[0]
    p, u = pos.copy(), vel.copy()
    t = oracle.Tree(p, m)
    oa, op, _, _ = t.forces(theta, EPS)
    for _ in range(steps):
        oracle.kdk_step(p, u, m, oa, op, DT, theta, EPS)
    amax = np.abs(oa).max()
    tol_v = 4e-5 * amax * DT * steps
    say("merger steps: max |dv|", np.abs(v - u).max(), "bound", tol_v)
    assert np.abs(v - u).max() <= tol_v
    assert np.abs(x - p).max() <= tol_v * DT * steps
    # the energy change over the steps agrees with the oracle's
    ek = 0.5 * (m * (u * u).sum(axis=1)).sum() + 0.5 * (m * op).sum()
    tt = oracle.Tree(pos, m)
    _, op0, _, _ = tt.forces(theta, EPS)
    ek0 = 0.5 * (m * (vel * vel).sum(axis=1)).sum() + 0.5 * (m * op0).sum()
    say("merger dE/E gpu", (e1[2] - e0[2]) / e0[2], "oracle", (ek - ek0) / ek0)
    assert abs((e1[2] - e0[2]) - (ek - ek0)) <= 1e-6 * abs(ek0)
    ctx.close()
