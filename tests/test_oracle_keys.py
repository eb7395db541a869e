"""Pins of the oracle's integer map, Morton keys and stable sort (App. A, App. B)."""

import numpy as np
import pytest

import oracle
from conftest import golden_path


def _read_dilate_example():
    rows = []
    for line in open(golden_path("dilate_example.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        rows.append((parts[0], "".join(parts[1:])))
    return rows


def test_paper_dilate_example():
    # App. B: 0100111011 -> 000 001 000 000 001 001 001 000 001 001.  A key made
    # from an x coordinate alone is exactly the dilation of x.
    (src, dst), = _read_dilate_example()
    q = int(src, 2)
    assert oracle.interleave(q, 0, 0) == int(dst, 2)
    # y and z land one and two bits higher
    assert oracle.interleave(0, q, 0) == int(dst, 2) << 1
    assert oracle.interleave(0, 0, q) == int(dst, 2) << 2


def test_all_10bit_inputs_spread_to_every_third_bit():
    # brute force over every 10-bit input: the spread value has popcount equal to
    # the input's, only bits at multiples of 3, and reading those bits back in
    # order recovers the input.
    for v in range(1024):
        k = oracle.interleave(v, 0, 0)
        assert bin(k).count("1") == bin(v).count("1")
        assert k & ~int("001" * 20, 2) == 0
        back = int("".join(bin(k)[2:].zfill(60)[2::3]), 2)
        assert back == v


def test_key_prefix_is_cell_membership():
    # Two points share the level-l key prefix iff their integer coordinates agree
    # in the top l bits on every axis (same octree cell at level l).
    rng = np.random.default_rng(0)
    for _ in range(3000):
        a = rng.integers(0, 1 << 20, 3)
        b = a.copy()
        lvl = int(rng.integers(0, 21))
        # perturb b below the level-lvl resolution on a random axis, sometimes above
        ax = int(rng.integers(0, 3))
        bit = int(rng.integers(0, 20))
        b[ax] ^= (1 << bit)
        ka = oracle.interleave(*[int(x) for x in a])
        kb = oracle.interleave(*[int(x) for x in b])
        same_key = (ka >> (3 * (20 - lvl))) == (kb >> (3 * (20 - lvl)))
        same_cell = all((int(a[k]) >> (20 - lvl)) == (int(b[k]) >> (20 - lvl)) for k in range(3))
        assert same_key == same_cell


def test_keys_are_injective_and_60_bit():
    rng = np.random.default_rng(1)
    q = np.unique(rng.integers(0, 1 << 20, (20000, 3)), axis=0)
    ks = {oracle.interleave(*map(int, row)) for row in q}
    assert len(ks) == q.shape[0]
    assert max(ks) < (1 << 60)


def test_domain_and_integer_map_hand_cases():
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [0.5, 0.25, 0.75]])
    lo, L, scale = oracle.domain(pos)
    assert np.all(lo == 0.0) and L == 1.0 and scale == 2.0 ** 20
    key, q = oracle.keys(pos)
    assert q[0].tolist() == [0, 0, 0]
    assert q[1].tolist() == [2 ** 20 - 1] * 3          # top corner clamps
    assert q[2].tolist() == [2 ** 19, 2 ** 18, 3 * 2 ** 18]
    # the cube side is the largest extent; shorter axes are not stretched
    pos2 = np.array([[-2.0, 5.0, 1.0], [2.0, 6.0, 1.0]])
    lo2, L2, s2 = oracle.domain(pos2)
    assert lo2.tolist() == [-2.0, 5.0, 1.0] and L2 == 4.0
    _, q2 = oracle.keys(pos2)
    assert q2[1].tolist() == [2 ** 20 - 1, 2 ** 18, 0]
    # all points equal: side 1
    _, L3, _ = oracle.domain(np.ones((5, 3)))
    assert L3 == 1.0


def test_domain_rejects_non_finite():
    pos = np.zeros((4, 3))
    pos[2, 1] = np.nan
    with pytest.raises(ValueError):
        oracle.domain(pos)


def test_argsort_is_stable_ascending():
    rng = np.random.default_rng(2)
    for n in (1, 2, 7, 1000, 4097):
        key = rng.integers(0, 50, n).astype(np.uint64) << np.uint64(40)
        perm = oracle.argsort(key)
        assert np.array_equal(perm, np.argsort(key, kind="stable"))
