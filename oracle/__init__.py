"""CPU oracle for the sparse-octree Barnes-Hut tree-code (Bedorf, Gaburov &
Portegies Zwart, arXiv:1106.1900): a plain single-threaded float64 C library
(``bh_oracle.c``) and this ctypes wrapper.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It shares no code with the HIP
library; the two meet only through the arrays of the ``workloads`` generators.

What each function follows in the paper:

* ``domain``/``keys``/``interleave`` - App. B (integer map and Morton key).
* ``argsort`` - App. A (stable radix sort = stable ascending order of keys).
* ``Tree`` - Sect. 2.1 (level-by-level cells, links), Sect. 2.2 (groups),
  Sect. 3.2 (float64 monopole and quadrupole moments).
* ``Tree.rcrit``/``Tree.mac_accept`` - Sect. 3.3, Eq. (1); with ``mac=1`` the
  minimum-distance test that Sect. 3.3 names as the alternative (Salmon & Warren
  1994): the group's box must be farther than l/theta from the cell's cube.
* ``Tree.walk_counts``/``Tree.group_lists``/``Tree.forces`` - Sect. 2.2
  breadth-first group walk with float64 evaluation.
* ``direct`` - the direct-summation reference of Sect. 4.2.1 (Eq. (2)).
* ``kdk_step`` - Sect. 3.1 leapfrog; ``energy`` - Eq. (3) ingredients.
* ``block_bins``/``Block`` - block time-steps motivated in Sect. 5 (forces only
  for the particles due, multipole-only refits in between, a rebuild once the
  walk has grown); the criterion and schedule are readings (bh_oracle.c).
"""

import ctypes
from concurrent.futures import ThreadPoolExecutor
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bh_oracle.c")
_LIB = os.path.join(_HERE, "_bh_oracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

_lib = None


def build(force=True):
    """Compile the oracle with gcc (no fused multiply-add)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], cwd=_HERE)
    os.replace(tmp, _LIB)
    return _LIB


def _P(t):
    return ctypes.POINTER(t)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    L = ctypes.CDLL(_LIB)
    d, f, i64, u64, u32, u8, i32 = (ctypes.c_double, ctypes.c_float, ctypes.c_int64,
                                    ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint8,
                                    ctypes.c_int32)
    vp = ctypes.c_void_p
    sig = {
        "orc_interleave": (u64, [u32, u32, u32]),
        "orc_domain": (ctypes.c_int, [vp, i64, vp, vp, vp]),
        "orc_keys": (None, [vp, i64, vp, d, vp, vp]),
        "orc_argsort": (ctypes.c_int, [vp, i64, vp]),
        "orc_build": (vp, [vp, vp, i64, ctypes.c_int, ctypes.c_int]),
        "orc_free": (None, [vp]),
        "orc_n": (i64, [vp]),
        "orc_ncells": (i64, [vp]),
        "orc_ngroups": (i64, [vp]),
        "orc_depth": (ctypes.c_int, [vp]),
        "orc_get_domain": (None, [vp, vp, vp, vp]),
        "orc_get_order": (None, [vp, vp, vp]),
        "orc_get_cells": (None, [vp] + [vp] * 8),
        "orc_get_groups": (None, [vp, vp, vp, vp, vp]),
        "orc_get_moments": (None, [vp, vp, vp, vp]),
        "orc_rcrit": (None, [vp, f, vp, vp]),
        "orc_mac_accept": (ctypes.c_int, [vp, i64, i64, f]),
        "orc_mac_accept_min": (ctypes.c_int, [vp, i64, i64, f]),
        "orc_set_mac": (None, [vp, ctypes.c_int]),
        "orc_get_mac": (ctypes.c_int, [vp]),
        "orc_walk_counts": (ctypes.c_int, [vp, f, vp, vp]),
        "orc_group_lists": (i64, [vp, f, i64, vp, i64, vp, i64, vp]),
        "orc_forces": (ctypes.c_int, [vp, f, f, vp, i64, vp, vp, vp, vp]),
        "orc_refit": (ctypes.c_int, [vp, vp]),
        "orc_direct": (None, [vp, vp, i64, f, vp, i64, vp, vp]),
        "orc_kdk_step": (ctypes.c_int, [vp, vp, vp, i64, vp, vp, d, f, f,
                                        ctypes.c_int, ctypes.c_int]),
        "orc_energy": (None, [vp, vp, vp, i64, vp]),
        "orc_block_bins": (None, [vp, i64, d, ctypes.c_int, d, d, vp]),
        "orc_block_new": (vp, [vp, vp, vp, i64, vp, vp, f, f, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int]),
        "orc_block_free": (None, [vp]),
        "orc_block_base": (d, [vp]),
        "orc_block_rebuild_next": (ctypes.c_int, [vp]),
        "orc_block_step": (ctypes.c_int, [vp, vp, ctypes.c_int, d, d, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    del i32, u8
    _lib = L
    return L


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


def interleave(qx, qy, qz):
    return int(lib().orc_interleave(qx, qy, qz))


def domain(pos):
    pos = _f64(pos)
    lo = np.zeros(3)
    L = ctypes.c_double()
    scale = ctypes.c_double()
    st = lib().orc_domain(_ptr(pos), pos.shape[0], _ptr(lo), ctypes.byref(L), ctypes.byref(scale))
    if st:
        raise ValueError("non-finite coordinate")
    return lo, L.value, scale.value


def keys(pos):
    """Keys and integer coordinates of every point, input order."""
    pos = _f64(pos)
    lo, L, scale = domain(pos)
    n = pos.shape[0]
    key = np.zeros(n, dtype=np.uint64)
    q = np.zeros((n, 3), dtype=np.uint32)
    lib().orc_keys(_ptr(pos), n, _ptr(lo), scale, _ptr(key), _ptr(q))
    return key, q


def argsort(key):
    key = np.ascontiguousarray(key, dtype=np.uint64)
    perm = np.zeros(key.shape[0], dtype=np.int64)
    if lib().orc_argsort(_ptr(key), key.shape[0], _ptr(perm)):
        raise MemoryError
    return perm


class Tree:
    """The canonical tree of a particle set (Sect. 2.1-2.2, 3.2)."""

    def __init__(self, pos, mass, nleaf=16, ncrit=64, mac=0):
        self.pos = _f64(pos)
        self.mass = _f64(mass)
        n = self.pos.shape[0]
        if self.pos.shape != (n, 3) or self.mass.shape != (n,):
            raise ValueError("pos must be (n, 3), mass (n,)")
        self.n = n
        self.nleaf = nleaf
        self.ncrit = ncrit
        h = lib().orc_build(_ptr(self.pos), _ptr(self.mass), n, nleaf, ncrit)
        if not h:
            raise ValueError("oracle build failed (bad input or out of memory)")
        self._h = ctypes.c_void_p(h)
        L = lib()
        self.ncells = int(L.orc_ncells(self._h))
        self.ngroups = int(L.orc_ngroups(self._h))
        self.depth = int(L.orc_depth(self._h))
        L.orc_set_mac(self._h, int(mac))
        self.mac = int(L.orc_get_mac(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    def refit(self, pos):
        """Multipole-only update (Sect. 5): same cells, groups, keys and domain;
        moments and group boxes recomputed from the new positions (input order)."""
        p = _f64(pos)
        if p.shape != (self.n, 3):
            raise ValueError("pos must be (n, 3)")
        if lib().orc_refit(self._h, _ptr(p)) != 0:
            raise ValueError("non-finite coordinate")
        self.pos = p

    def domain(self):
        lo = np.zeros(3)
        L = ctypes.c_double()
        s = ctypes.c_double()
        lib().orc_get_domain(self._h, _ptr(lo), ctypes.byref(L), ctypes.byref(s))
        return lo, L.value, s.value

    def order(self):
        perm = np.zeros(self.n, dtype=np.int64)
        key = np.zeros(self.n, dtype=np.uint64)
        lib().orc_get_order(self._h, _ptr(perm), _ptr(key))
        return perm, key

    def cells(self):
        c = self.ncells
        out = dict(
            level=np.zeros(c, np.uint8), prefix=np.zeros(c, np.uint64),
            first=np.zeros(c, np.int64), count=np.zeros(c, np.int64),
            is_leaf=np.zeros(c, np.uint8), parent=np.zeros(c, np.int64),
            child=np.zeros(c, np.int64), nchild=np.zeros(c, np.int32))
        lib().orc_get_cells(self._h, *[_ptr(out[k]) for k in
                                       ("level", "prefix", "first", "count", "is_leaf",
                                        "parent", "child", "nchild")])
        return out

    def groups(self):
        g = self.ngroups
        out = dict(first=np.zeros(g, np.int64), count=np.zeros(g, np.int64),
                   centre=np.zeros((g, 3)), half=np.zeros((g, 3), np.float32))
        lib().orc_get_groups(self._h, _ptr(out["first"]), _ptr(out["count"]),
                             _ptr(out["centre"]), _ptr(out["half"]))
        return out

    def moments(self):
        c = self.ncells
        out = dict(mass=np.zeros(c), com=np.zeros((c, 3)), S=np.zeros((c, 6)))
        lib().orc_get_moments(self._h, _ptr(out["mass"]), _ptr(out["com"]), _ptr(out["S"]))
        return out

    def rcrit(self, theta):
        r2 = np.zeros(self.ncells, np.float32)
        centre = np.zeros((self.ncells, 3))
        lib().orc_rcrit(self._h, float(theta), _ptr(r2), _ptr(centre))
        return r2, centre

    def mac_accept(self, g, c, rcrit2_c):
        f = lib().orc_mac_accept_min if self.mac else lib().orc_mac_accept
        return bool(f(self._h, int(g), int(c), float(rcrit2_c)))

    def walk_counts(self, theta):
        npp = np.zeros(self.ngroups, np.int64)
        npc = np.zeros(self.ngroups, np.int64)
        if lib().orc_walk_counts(self._h, float(theta), _ptr(npp), _ptr(npc)):
            raise MemoryError
        return npp, npc

    def group_lists(self, theta, g):
        cap = self.ncells
        pc = np.zeros(cap, np.int64)
        pp = np.zeros(cap, np.int64)
        npl = ctypes.c_int64()
        r = lib().orc_group_lists(self._h, float(theta), int(g), _ptr(pc), cap, _ptr(pp), cap,
                                  ctypes.byref(npl))
        if r < 0:
            raise RuntimeError("group_lists failed")
        return pc[:r].copy(), pp[:npl.value].copy()

    def forces(self, theta, eps, groups=None, threads=1):
        """float64 tree forces, input order; rows of unselected groups are NaN.
        threads > 1: the groups are split over that many host threads (the C
        evaluation reads the tree only and writes the rows of its own groups)."""
        n = self.n
        acc = np.full((n, 3), np.nan)
        pot = np.full(n, np.nan)
        aabs = np.full(n, np.nan)
        pabs = np.full(n, np.nan)
        if groups is None:
            garr = np.arange(self.ngroups, dtype=np.int64) if threads > 1 else None
        else:
            garr = np.ascontiguousarray(groups, dtype=np.int64)

        def run(sel):
            gp, ng = (None, 0) if sel is None else (_ptr(sel), sel.shape[0])
            return lib().orc_forces(self._h, float(theta), float(eps), gp, ng, _ptr(acc),
                                    _ptr(pot), _ptr(aabs), _ptr(pabs))

        if threads <= 1 or garr is None or garr.shape[0] < 2:
            sts = [run(garr)]
        else:
            # round-robin runs of 16 groups: neighbouring groups cost alike
            runs = [garr[i:i + 16] for i in range(0, garr.shape[0], 16)]
            parts = [np.ascontiguousarray(np.concatenate(runs[k::threads]))
                     for k in range(min(threads, len(runs)))]
            with ThreadPoolExecutor(len(parts)) as ex:
                sts = list(ex.map(run, parts))
        for st in sts:
            if st:
                raise RuntimeError("oracle forces failed (%d)" % st)
        return acc, pot, aabs, pabs


def direct(pos, mass, eps, targets=None, threads=1):
    """float64 direct summation on the given targets (all if None); threads > 1
    splits the targets over that many host threads."""
    pos = _f64(pos)
    mass = _f64(mass)
    n = pos.shape[0]
    tgt = np.arange(n, dtype=np.int64) if targets is None else np.ascontiguousarray(
        targets, dtype=np.int64)
    acc = np.zeros((tgt.shape[0], 3))
    pot = np.zeros(tgt.shape[0])

    def run(k0, k1):
        lib().orc_direct(_ptr(pos), _ptr(mass), n, float(eps), _ptr(tgt[k0:]), k1 - k0,
                         _ptr(acc[k0:]), _ptr(pot[k0:]))

    if threads <= 1 or tgt.shape[0] < 2:
        run(0, tgt.shape[0])
    else:
        b = np.linspace(0, tgt.shape[0], min(threads, tgt.shape[0]) + 1).astype(np.int64)
        with ThreadPoolExecutor(len(b) - 1) as ex:
            list(ex.map(lambda k: run(int(b[k]), int(b[k + 1])), range(len(b) - 1)))
    return acc, pot


def kdk_step(pos, vel, mass, acc, pot, dt, theta, eps, nleaf=16, ncrit=64):
    """One kick-drift-kick step in place (float64 arrays, input order)."""
    for a in (pos, vel, acc, pot):
        if a.dtype != np.float64 or not a.flags.c_contiguous:
            raise ValueError("state arrays must be contiguous float64")
    mass = _f64(mass)
    st = lib().orc_kdk_step(_ptr(pos), _ptr(vel), _ptr(mass), pos.shape[0], _ptr(acc),
                            _ptr(pot), float(dt), float(theta), float(eps), nleaf, ncrit)
    if st:
        raise RuntimeError("oracle kdk failed (%d)" % st)


def energy(vel, mass, pot):
    vel = _f64(vel)
    mass = _f64(mass)
    pot = _f64(pot)
    out = np.zeros(6)
    lib().orc_energy(_ptr(vel), _ptr(mass), _ptr(pot), mass.shape[0], _ptr(out))
    return out


def block_bins(acc, dt_max, max_level, eta, length):
    """Power-of-two time-step bins from float32 accelerations [n, 3]."""
    a = np.ascontiguousarray(acc, dtype=np.float32)
    n = a.shape[0]
    bins = np.zeros(n, np.uint8)
    lib().orc_block_bins(_ptr(a), n, float(dt_max), int(max_level), float(eta), float(length),
                         _ptr(bins))
    return bins


class Block:
    """A system advanced by block time-steps (float64, caller order).  pos, vel,
    acc, pot are numpy arrays updated in place."""

    def __init__(self, pos, vel, mass, theta, eps, nleaf=16, ncrit=64, mac=0):
        self.pos = _f64(pos).copy()
        self.vel = _f64(vel).copy()
        self.mass = _f64(mass).copy()
        n = self.pos.shape[0]
        self.n = n
        self.acc = np.zeros((n, 3))
        self.pot = np.zeros(n)
        h = lib().orc_block_new(_ptr(self.pos), _ptr(self.vel), _ptr(self.mass), n,
                                _ptr(self.acc), _ptr(self.pot), float(theta), float(eps),
                                int(nleaf), int(ncrit), int(mac))
        if not h:
            raise ValueError("oracle block system failed")
        self._h = ctypes.c_void_p(h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_block_free(h)

    @property
    def base(self):
        """Mean over the particles of their base (interactions of their group in
        the last walk covering them on a freshly built tree)."""
        return float(lib().orc_block_base(self._h))

    @property
    def rebuild_next(self):
        """True if the next force evaluation will be on a rebuilt tree."""
        return bool(lib().orc_block_rebuild_next(self._h))

    def step(self, bins, max_level, dt_max, growth):
        """One block step; returns (rebuilds during the step, interactions per
        particle of the final walk, completed steps per particle)."""
        b = np.ascontiguousarray(bins, dtype=np.uint8)
        rebuilt = ctypes.c_int()
        inter = ctypes.c_double()
        kicks = np.zeros(self.n, np.int64)
        st = lib().orc_block_step(self._h, _ptr(b), int(max_level), float(dt_max), float(growth),
                                  ctypes.byref(rebuilt), ctypes.byref(inter), _ptr(kicks))
        if st:
            raise ValueError("oracle block step failed (%d)" % st)
        return int(rebuilt.value), float(inter.value), kicks
