"""Shared pieces of the GPU parity tests: running the HIP path through the C ABI
and comparing its tree, counts and forces with the oracle."""

import sys

import numpy as np

import oracle

# float32 interactions against the float64 oracle on the same interaction lists:
# each interaction carries O(1e-7) relative rounding (offsets, rsqrt, products)
# and the tile sums are compensated, so the error of a particle's total is a
# small multiple of 1e-7 of the sum of the magnitudes of its terms.  1e-5 of that
# sum leaves a factor ~50 of headroom; the median relative error of |a| must be
# far below the tree's own truncation error.
TOL_ABS_TERMS = 1e-5
TOL_MEDIAN_REL = 1e-6


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_build(pos, mass, nleaf=16, ncrit=64):
    import paper_1106_1900_amd as bh
    ctx = bh.Context(nleaf=nleaf, ncrit=ncrit)
    ctx.build_tree(to_dev(pos), to_dev(mass))
    return ctx


def compare_tree(ex, t):
    """Bit-exact comparison of the exported GPU tree with the oracle tree."""
    perm, key = t.order()
    assert np.array_equal(ex["key"], key), "keys differ"
    assert np.array_equal(ex["perm"], perm), "sorted order differs"
    c = t.cells()
    assert ex["level"].shape[0] == t.ncells, ("cell count", ex["level"].shape[0], t.ncells)
    for k in ("level", "prefix", "first", "count", "is_leaf", "parent", "child", "nchild"):
        assert np.array_equal(ex[k], c[k]), "cell field %s differs" % k
    g = t.groups()
    assert ex["gfirst"].shape[0] == t.ngroups, ("group count", ex["gfirst"].shape[0], t.ngroups)
    assert np.array_equal(ex["gfirst"], g["first"])
    assert np.array_equal(ex["gcount"], g["count"])
    assert np.array_equal(ex["gcentre"], g["centre"]), "group centres differ"
    assert np.array_equal(ex["ghalf"], g["half"]), "group half-sizes differ"
    mo = t.moments()
    assert np.array_equal(ex["mass"], mo["mass"]), "cell masses differ"
    assert np.array_equal(ex["com"], mo["com"]), "centres of mass differ"
    scale = np.abs(mo["S"]).max(axis=1, keepdims=True) + 1e-300
    assert np.all(np.abs(ex["S"] - mo["S"]) <= 1e-12 * scale), "second moments differ"


def compare_walk(ex, t, theta):
    r2, _ = t.rcrit(theta)
    assert np.array_equal(ex["rcrit2"], r2), "opening radii differ"
    npp, npc = t.walk_counts(theta)
    assert np.array_equal(ex["npp"], npp), "particle-particle counts differ"
    assert np.array_equal(ex["npc"], npc), "particle-cell counts differ"


def host_threads():
    """Host threads for the oracle's evaluations (the cores this process may use,
    at most 16)."""
    import os
    try:
        k = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        k = os.cpu_count() or 1
    return max(1, min(16, k))


def compare_forces(acc, pot, t, theta, eps, groups=None, threads=1):
    """GPU float32 forces against the float64 oracle on the same lists."""
    oa, op, aabs, pabs = t.forces(theta, eps, groups, threads=threads)
    sel = ~np.isnan(op)
    acc = acc[sel].astype(np.float64)
    pot = pot[sel].astype(np.float64)
    oa, op, aabs, pabs = oa[sel], op[sel], aabs[sel], pabs[sel]
    da = np.linalg.norm(acc - oa, axis=1)
    assert np.all(np.isfinite(acc)) and np.all(np.isfinite(pot))
    bad = da > TOL_ABS_TERMS * aabs
    assert not bad.any(), ("acc", int(bad.sum()), float((da / aabs).max()))
    dp = np.abs(pot - op)
    badp = dp > TOL_ABS_TERMS * pabs
    assert not badp.any(), ("pot", int(badp.sum()), float((dp / pabs).max()))
    na = np.linalg.norm(oa, axis=1)
    nz = na > 0
    if nz.any():
        med = float(np.median(da[nz] / na[nz]))
        assert med <= TOL_MEDIAN_REL, ("median relative", med)
    return float((da / np.maximum(aabs, 1e-300)).max())


def split_forest(ex, sizes, selected=None):
    """Per-cluster views of a batch's exported forest: particle, cell and group
    indices renumbered from 0 within each cluster (cells keep their relative
    order, which is (level, key prefix) order within the cluster).  selected:
    indices of the clusters to return (default all)."""
    out = []
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    for c in (range(len(sizes)) if selected is None else selected):
        lo, hi = int(starts[c]), int(starts[c] + sizes[c])
        cm = (ex["first"] >= lo) & (ex["first"] < hi)
        idx = np.nonzero(cm)[0]
        local = np.full(ex["first"].shape[0], -1, np.int64)
        local[idx] = np.arange(idx.shape[0])
        d = {"key": ex["key"][lo:hi], "perm": ex["perm"][lo:hi] - lo}
        for k in ("level", "prefix", "count", "is_leaf", "nchild", "mass", "com", "S", "rcrit2"):
            d[k] = ex[k][idx]
        d["first"] = ex["first"][idx] - lo
        for k in ("parent", "child"):
            v = ex[k][idx]
            d[k] = np.where(v < 0, -1, local[np.maximum(v, 0)])
        gm = (ex["gfirst"] >= lo) & (ex["gfirst"] < hi)
        d["gfirst"] = ex["gfirst"][gm] - lo
        for k in ("gcount", "gcentre", "ghalf", "npp", "npc"):
            d[k] = ex[k][gm]
        out.append(d)
    return out
