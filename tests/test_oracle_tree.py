"""Pins of the oracle's tree (Sect. 2.1), groups (Sect. 2.2) and moments (Sect. 3.2)."""

import numpy as np
import pytest

import oracle
import workloads


def _sets(name, n, seed=0):
    if name == "plummer":
        return workloads.plummer(n, seed)
    if name == "clustered":
        return workloads.clustered(n, seed)
    if name == "line":
        return workloads.on_a_line(n, seed)
    if name == "cube":
        return workloads.uniform_cube(n, seed)
    raise KeyError(name)


CASES = [("plummer", 3000), ("clustered", 2000), ("line", 700), ("cube", 1500)]


def check_tree_invariants(t):
    c = t.cells()
    perm, key = t.order()
    n = t.n
    lev, first, count = c["level"].astype(int), c["first"], c["count"]
    # (level, prefix) order, root first
    assert lev[0] == 0 and first[0] == 0 and count[0] == n and c["parent"][0] == -1
    order = np.lexsort((c["prefix"], lev))
    assert np.array_equal(order, np.arange(t.ncells))
    # prefix is the key prefix of every particle in the cell
    for i in range(t.ncells):
        sh = np.uint64(3 * (20 - lev[i]))
        ks = key[first[i]:first[i] + count[i]] >> sh
        assert np.all(ks == c["prefix"][i])
    leaf = c["is_leaf"].astype(bool)
    # leaf rule and node rule
    assert np.all(count[leaf & (lev < 20)] <= t.nleaf)
    assert np.all(count[~leaf] > t.nleaf)
    assert np.all(lev[~leaf] < 20)
    # children contiguous, partition their parent's range in order, one level down
    for p in np.nonzero(~leaf)[0]:
        ch0, nc = c["child"][p], c["nchild"][p]
        assert 1 <= nc <= 8
        ch = np.arange(ch0, ch0 + nc)
        assert np.all(c["parent"][ch] == p)
        assert np.all(lev[ch] == lev[p] + 1)
        assert first[ch[0]] == first[p]
        assert np.all(first[ch[1:]] == first[ch[:-1]] + count[ch[:-1]])
        assert first[ch[-1]] + count[ch[-1]] == first[p] + count[p]
        assert np.all(c["prefix"][ch] >> np.uint64(3) == c["prefix"][p])
        assert len(set(c["prefix"][ch].tolist())) == nc
    assert np.all(c["child"][leaf] == -1) and np.all(c["nchild"][leaf] == 0)
    # every particle is in exactly one leaf
    cover = np.zeros(n, int)
    for i in np.nonzero(leaf)[0]:
        cover[first[i]:first[i] + count[i]] += 1
    assert np.all(cover == 1)
    # sorted order is the stable key order
    key_in, _ = oracle.keys(t.pos)
    assert np.array_equal(perm, np.argsort(key_in, kind="stable"))


@pytest.mark.parametrize("name,n", CASES)
def test_tree_invariants(name, n):
    pos, _, m = _sets(name, n)
    for nleaf, ncrit in ((16, 64), (1, 1), (8, 32), (32, 128)):
        check_tree_invariants(oracle.Tree(pos, m, nleaf, ncrit))


def _recursive_octree(q, nleaf):
    """Independent top-down subdivision by integer geometry (no keys): returns a
    list of (level, sorted tuple of input indices, is_leaf) in level order and,
    within a level, in Morton (child-index) order."""
    per_level = [[] for _ in range(21)]

    def rec(level, corner, idx):
        leaf = len(idx) <= nleaf or level == 20
        per_level[level].append((level, tuple(sorted(idx.tolist())), leaf))
        if leaf:
            return
        sh = 20 - level - 1
        sub = q[idx] >> sh
        for o in range(8):
            cc = np.array([2 * corner[0] + (o & 1), 2 * corner[1] + ((o >> 1) & 1),
                           2 * corner[2] + ((o >> 2) & 1)])
            sel = idx[np.all(sub == cc, axis=1)]
            if sel.size:
                rec(level + 1, cc, sel)

    rec(0, np.zeros(3, dtype=np.int64), np.arange(q.shape[0]))
    return [c for lvl in per_level for c in lvl]


@pytest.mark.parametrize("name,n", [("plummer", 300), ("clustered", 250), ("line", 120),
                                    ("cube", 200)])
@pytest.mark.parametrize("nleaf", [1, 4, 16])
def test_tree_equals_recursive_subdivision(name, n, nleaf):
    pos, _, m = _sets(name, n, seed=3)
    t = oracle.Tree(pos, m, nleaf, 64)
    _, q = oracle.keys(pos)
    ref = _recursive_octree(q.astype(np.int64), nleaf)
    c = t.cells()
    perm, _ = t.order()
    got = [(int(c["level"][i]),
            tuple(sorted(perm[c["first"][i]:c["first"][i] + c["count"][i]].tolist())),
            bool(c["is_leaf"][i])) for i in range(t.ncells)]
    assert got == ref


def test_hand_case_eight_octants():
    pos = np.array([[x, y, z] for z in (0.25, 0.75) for y in (0.25, 0.75) for x in (0.25, 0.75)])
    t = oracle.Tree(pos, np.ones(8), nleaf=1, ncrit=1)
    c = t.cells()
    assert t.ncells == 9
    assert c["level"].tolist() == [0] + [1] * 8
    assert c["is_leaf"].tolist() == [0] + [1] * 8
    assert c["nchild"][0] == 8 and c["child"][0] == 1
    # children in Morton order: x bit lowest, then y, then z -> input order here
    perm, _ = t.order()
    assert perm.tolist() == list(range(8))
    assert c["prefix"][1:].tolist() == list(range(8))


def test_hand_case_coincident_chain():
    pos, _, m = workloads.coincident(100)
    t = oracle.Tree(pos, m, nleaf=16, ncrit=64)
    c = t.cells()
    assert t.ncells == 21 and t.depth == 20
    assert c["level"].tolist() == list(range(21))
    assert c["is_leaf"].tolist() == [0] * 20 + [1]
    assert np.all(c["count"] == 100)
    g = t.groups()
    # a 100-particle deepest leaf is cut into groups of 64 and 36
    assert g["first"].tolist() == [0, 64] and g["count"].tolist() == [64, 36]


def test_small_set_is_one_leaf():
    pos, _, m = workloads.plummer(16, 5)
    t = oracle.Tree(pos, m, nleaf=16, ncrit=64)
    assert t.ncells == 1 and t.cells()["is_leaf"][0] == 1
    assert t.ngroups == 1


@pytest.mark.parametrize("name,n", CASES)
@pytest.mark.parametrize("ncrit", [1, 16, 64, 100])
def test_groups_partition_and_maximality(name, n, ncrit):
    pos, _, m = _sets(name, n, seed=4)
    t = oracle.Tree(pos, m, 16, ncrit)
    g = t.groups()
    c = t.cells()
    first, count = g["first"], g["count"]
    assert first[0] == 0 and np.all(first[1:] == first[:-1] + count[:-1])
    assert first[-1] + count[-1] == t.n
    assert np.all(count >= 1) and np.all(count <= ncrit)
    # each group is a maximal cell (count <= ncrit, parent > ncrit) or a chunk of
    # a leaf larger than ncrit
    # (a chain of single-child cells shares one range, so look at all of them)
    cells_of = {}
    for i, (f, k) in enumerate(zip(c["first"], c["count"])):
        cells_of.setdefault((int(f), int(k)), []).append(i)
    for f, k in zip(first, count):
        cand = cells_of.get((int(f), int(k)), [])
        if any(i == 0 or c["count"][c["parent"][i]] > ncrit for i in cand):
            continue
        # must lie inside a leaf holding more than ncrit particles
        inside = [j for j in np.nonzero(c["is_leaf"])[0]
                  if c["first"][j] <= f and f + k <= c["first"][j] + c["count"][j]]
        assert len(inside) == 1 and c["count"][inside[0]] > ncrit
        assert (f - c["first"][inside[0]]) % ncrit == 0
    # boxes are the tight boxes of the sorted particles
    perm, _ = t.order()
    xs = t.pos[perm]
    for gi in range(0, t.ngroups, max(1, t.ngroups // 50)):
        p = xs[first[gi]:first[gi] + count[gi]]
        lo, hi = p.min(axis=0), p.max(axis=0)
        assert np.array_equal(g["centre"][gi], 0.5 * (lo + hi))
        assert np.array_equal(g["half"][gi], (0.5 * (hi - lo)).astype(np.float32))


@pytest.mark.parametrize("name,n", CASES)
def test_moments_against_direct_sums(name, n):
    pos, _, m = _sets(name, n, seed=5)
    t = oracle.Tree(pos, m, 16, 64)
    mo = t.moments()
    c = t.cells()
    perm, _ = t.order()
    xs, ms = t.pos[perm], t.mass[perm]
    idx = np.unique(np.concatenate([[0], np.linspace(0, t.ncells - 1, 60).astype(int)]))
    for i in idx:
        sl = slice(c["first"][i], c["first"][i] + c["count"][i])
        M = ms[sl].sum()
        com = (ms[sl, None] * xs[sl]).sum(axis=0) / M
        d = xs[sl] - com
        S = np.einsum("i,ij,ik->jk", ms[sl], d, d)
        assert mo["mass"][i] == pytest.approx(M, rel=1e-14)
        scale = np.abs(xs[sl]).max() + 1e-300
        assert np.all(np.abs(mo["com"][i] - com) <= 1e-13 * scale)
        Sg = mo["S"][i]
        Sm = np.array([[Sg[0], Sg[3], Sg[4]], [Sg[3], Sg[1], Sg[5]], [Sg[4], Sg[5], Sg[2]]])
        assert np.all(np.abs(Sm - S) <= 1e-12 * (np.abs(S).max() + M * scale * scale * 1e-3))


@pytest.mark.parametrize("shape", ["cube_corners", "octahedron"])
def test_symmetric_sets_have_isotropic_second_moment(shape):
    # For these sets S is a multiple of the identity, so the traceless quadrupole
    # 3S - tr(S) I vanishes (cube corners and regular octahedron).
    if shape == "cube_corners":
        pts = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], float)
    else:
        pts = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                       float)
    t = oracle.Tree(pts, np.full(len(pts), 0.25), nleaf=16, ncrit=64)
    S = t.moments()["S"][0]
    Sm = np.array([[S[0], S[3], S[4]], [S[3], S[1], S[5]], [S[4], S[5], S[2]]])
    Q = 3 * Sm - np.trace(Sm) * np.eye(3)
    assert np.abs(Q).max() < 1e-14
    assert np.trace(Sm) > 0


def test_rcrit_geometry_hand_case():
    # two points spanning [0,1]^3: the root has side 1, centre (0.5,0.5,0.5)
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])
    t = oracle.Tree(pos, np.array([1.0, 3.0]), nleaf=16, ncrit=64)
    r2, centre = t.rcrit(0.5)
    assert centre[0].tolist() == [0.5, 0.5, 0.5]
    com = t.moments()["com"][0]
    assert np.allclose(com, [0.75, 0.75, 0.75], rtol=0, atol=1e-15)
    delta = np.sqrt(3 * 0.25 ** 2)
    assert r2[0] == np.float32((1.0 / 0.5 + delta) ** 2)
