"""bh_forces_static (the entry point that allocates no device memory) against the
existing path it stands for, bh_build_tree + bh_compute_forces on a context with
the same leaf and group sizes: the same kernels run on the same tree, so the
accelerations and potentials must be identical, call after call, whatever the
previous call left in the library's array.  The first call is also checked
against the oracle's tree forces at the parity bar of the other GPU tests."""

import numpy as np
import pytest

import oracle
import workloads

from gpu_helpers import TOL_ABS_TERMS, say, to_dev

pytestmark = pytest.mark.gpu


def _context_forces(pos, mass, theta, eps):
    import torch
    import paper_1106_1900_amd as bh
    with bh.Context(nleaf=16, ncrit=64) as ctx:
        ctx.build_tree(to_dev(pos), to_dev(mass))
        acc, pot = ctx.compute_forces(theta, eps)
        torch.cuda.synchronize()
        return acc.cpu().numpy(), pot.cpu().numpy()


def _static_forces(pos, mass, theta, eps):
    import torch
    import paper_1106_1900_amd as bh
    acc, pot = bh.forces_static(to_dev(pos), to_dev(mass), theta, eps)
    torch.cuda.synchronize()
    return acc.cpu().numpy(), pot.cpu().numpy()


def test_static_calls_equal_the_context_path():
    import paper_1106_1900_amd as bh
    # a larger call, then a smaller one (the array keeps the first call's
    # contents), then the largest allowed and a ragged tiny one
    cases = [(20000, 11, 0.75, 0.01), (5000, 12, 0.5, 0.02), (bh.STATIC_MAX_N, 13, 0.75, 1.0 / 64),
             (17, 14, 0.5, 0.01)]
    for i, (n, seed, theta, eps) in enumerate(cases):
        say("static forces: n=%d seed=%d theta=%g eps=%g" % (n, seed, theta, eps))
        pos, _, mass = workloads.plummer(n, seed)
        sa, sp = _static_forces(pos, mass, theta, eps)
        ca, cp = _context_forces(pos, mass, theta, eps)
        assert np.array_equal(sa, ca), "accelerations differ (n=%d)" % n
        assert np.array_equal(sp, cp), "potentials differ (n=%d)" % n
        if i == 0:
            t = oracle.Tree(pos, mass, 16, 64)
            oa, _, aabs, _ = t.forces(theta, eps)
            err = np.linalg.norm(sa.astype(np.float64) - oa, axis=1)
            assert np.all(err <= TOL_ABS_TERMS * aabs)


def test_static_rejects_bad_arguments():
    import torch
    import paper_1106_1900_amd as bh
    n = bh.STATIC_MAX_N + 1
    pos = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    mass = torch.ones((n,), dtype=torch.float64, device="cuda")
    with pytest.raises(bh.BHError) as e:
        bh.forces_static(pos, mass, 0.75, 0.01)
    assert e.value.code == -1 and "BH_STATIC_MAX_N" in str(e.value)
    pos, _, mass = workloads.plummer(100, 15)
    with pytest.raises(bh.BHError) as e:
        bh.forces_static(to_dev(pos), to_dev(mass), 1.5, 0.01)
    assert e.value.code == -1
    # a non-finite coordinate is found on the device and reported by the call
    pos[7, 1] = np.nan
    with pytest.raises(bh.BHError) as e:
        bh.forces_static(to_dev(pos), to_dev(mass), 0.75, 0.01)
    assert e.value.code == -1 and "non-finite" in str(e.value)
    # and the next good call is unaffected
    pos, _, mass = workloads.plummer(3000, 16)
    sa, sp = _static_forces(pos, mass, 0.75, 0.01)
    ca, cp = _context_forces(pos, mass, 0.75, 0.01)
    assert np.array_equal(sa, ca) and np.array_equal(sp, cp)
