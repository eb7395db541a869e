"""The float64 direct summation that bench.py uses as the reference of its force
errors (Sect. 4.2.1, Eq. (2)) against the oracle's direct summation: the same
sums in another order, so equal to a few float64 roundings."""

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("maker,n,eps", [("plummer", 1 << 16, 1.0 / 64), ("hernquist", 20_000, 0.01),
                                         ("clustered", 3000, 0.001)])
def test_bench_direct_sum_equals_the_oracle_direct_sum(maker, n, eps):
    import bench
    if maker == "plummer":
        pos, _, m = workloads.plummer(n, 61)
    elif maker == "hernquist":
        pos, _, m = workloads.hernquist(n, 62)
    else:
        pos, _, m = workloads.clustered(n, 63)
    say("case direct", maker, n, eps)
    tgt = np.sort(np.random.default_rng(64).choice(n, 300, replace=False))
    got = bench.direct_fp64(pos, m, eps, tgt)
    want, _ = oracle.direct(pos, m, eps, tgt)
    scale = np.linalg.norm(want, axis=1).max()
    assert np.all(np.abs(got - want) <= 1e-12 * scale + 1e-300), float(np.abs(got - want).max() / scale)
