"""ctypes binding of libbh (include/bh.h).  Argument marshalling only: every step
of the method runs in the HIP kernels of the library.  Tensors passed in must be
contiguous CUDA (HIP) tensors of the stated dtype on the context's device; work is
enqueued on the current torch stream at context creation.
"""

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
HEADER = os.path.join(_ROOT, "include", "bh.h")

BH_OK, BH_EINVAL, BH_ENOMEM, BH_EDEVICE, BH_ESTATE = 0, -1, -2, -3, -4
MAC_EQ1, MAC_MIN_DIST = 0, 1     # opening tests (BH_MAC_EQ1, BH_MAC_MIN_DIST)
_NAMES = {BH_EINVAL: "EINVAL", BH_ENOMEM: "ENOMEM", BH_EDEVICE: "EDEVICE", BH_ESTATE: "ESTATE"}


class BHError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_NAMES.get(code, "?"), code, msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("nleaf", ctypes.c_int32), ("ncrit", ctypes.c_int32),
                ("max_n", ctypes.c_int64), ("hbm_budget_bytes", ctypes.c_int64),
                ("max_clusters", ctypes.c_int64)]


class Cluster(ctypes.Structure):
    """One cluster of a batch (bh_cluster)."""
    _fields_ = [("n", ctypes.c_int64), ("theta", ctypes.c_float), ("eps", ctypes.c_float),
                ("dt", ctypes.c_double), ("nleaf", ctypes.c_int32), ("ncrit", ctypes.c_int32),
                ("mac", ctypes.c_int32), ("pad", ctypes.c_int32)]


class BlockParams(ctypes.Structure):
    """bh_block_params: block time-steps."""
    _fields_ = [("dt_max", ctypes.c_double), ("eta", ctypes.c_double), ("length", ctypes.c_double),
                ("max_level", ctypes.c_int32), ("growth", ctypes.c_float)]


class BlockStats(ctypes.Structure):
    _fields_ = [("substeps", ctypes.c_int64), ("rebuilt", ctypes.c_int64),
                ("updates", ctypes.c_int64), ("walked_groups", ctypes.c_int64),
                ("sync_interactions", ctypes.c_double), ("base_interactions", ctypes.c_double),
                ("bin_count", ctypes.c_int64 * 16)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "bin_count"}
        d["bin_count"] = list(self.bin_count)
        return d


class TuneEntry(ctypes.Structure):
    _fields_ = [("log2n", ctypes.c_int32), ("theta", ctypes.c_float), ("nleaf", ctypes.c_int32),
                ("ncrit", ctypes.c_int32), ("ms", ctypes.c_double), ("ms_default", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("ncells", ctypes.c_int64), ("nleaves", ctypes.c_int64),
                ("ngroups", ctypes.c_int64), ("depth", ctypes.c_int32),
                ("lanes_per_group_max", ctypes.c_int32), ("sum_npp", ctypes.c_int64),
                ("sum_npc", ctypes.c_int64), ("ms_keys", ctypes.c_double),
                ("ms_sort", ctypes.c_double), ("ms_move", ctypes.c_double),
                ("ms_tree", ctypes.c_double), ("ms_moments", ctypes.c_double),
                ("ms_walk", ctypes.c_double), ("device_bytes", ctypes.c_int64),
                ("ms_walk_kernel", ctypes.c_double), ("walk_kernel_ms_total", ctypes.c_double),
                ("walk_kernel_launches", ctypes.c_int64), ("total_npp", ctypes.c_int64),
                ("total_npc", ctypes.c_int64), ("nclusters", ctypes.c_int64),
                ("graph_launches", ctypes.c_int64),
                ("graph_captures", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p


class TreeHost(ctypes.Structure):
    _fields_ = [(k, _vp) for k in ("key", "perm", "level", "prefix", "first", "count", "is_leaf",
                                   "parent", "child", "nchild", "mass", "com", "S", "rcrit2",
                                   "gfirst", "gcount", "gcentre", "ghalf", "npp", "npc")]


_lib = None


def library_path():
    return os.environ.get("BH_LIBRARY", os.path.join(_HERE, "libbh.so"))


def declared_functions():
    """Names of the functions include/bh.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(bh_\w+)\s*\(", text, re.M)))


def load_library():
    """Load libbh.so (built by ``python -m paper_1106_1900_amd.build``).  Raises if
    it is missing: there is no other implementation to fall back on."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError("libbh.so not built (%s); run python -m paper_1106_1900_amd.build" % path)
    L = ctypes.CDLL(path)
    i32, i64, f32, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_float, ctypes.c_double
    sig = {
        "bh_default_params": (i32, [ctypes.POINTER(Params)]),
        "bh_create": (i32, [ctypes.POINTER(_vp), ctypes.POINTER(Params), _vp]),
        "bh_destroy": (i32, [_vp]),
        "bh_build_tree": (i32, [_vp, _vp, _vp, i64]),
        "bh_set_velocities": (i32, [_vp, _vp]),
        "bh_set_mac": (i32, [_vp, i32]),
        "bh_compute_forces": (i32, [_vp, f32, f32, _vp, _vp]),
        "bh_leapfrog_step": (i32, [_vp, f64]),
        "bh_get_state": (i32, [_vp, _vp, _vp, _vp, _vp]),
        "bh_set_state": (i32, [_vp, _vp, _vp]),
        "bh_energy": (i32, [_vp, _vp]),
        "bh_stats_get": (i32, [_vp, ctypes.POINTER(Stats)]),
        "bh_export_tree": (i32, [_vp, ctypes.POINTER(TreeHost)]),
        "bh_drift": (i32, [_vp, f64]),
        "bh_kick": (i32, [_vp, f64, _vp]),
        "bh_refit": (i32, [_vp]),
        "bh_compute_forces_active": (i32, [_vp, f32, f32, _vp, _vp, _vp]),
        "bh_block_bins": (i32, [_vp, ctypes.POINTER(BlockParams), _vp, _vp]),
        "bh_block_step": (i32, [_vp, ctypes.POINTER(BlockParams), ctypes.POINTER(BlockStats)]),
        "bh_batch_build": (i32, [_vp, ctypes.POINTER(Cluster), i64, _vp, _vp, _vp]),
        "bh_batch_set_params": (i32, [_vp, ctypes.POINTER(Cluster), i64]),
        "bh_batch_forces": (i32, [_vp, _vp, _vp]),
        "bh_batch_run": (i32, [_vp, ctypes.c_int32]),
        "bh_batch_energy": (i32, [_vp, _vp]),
        "bh_autotune": (i32, [_vp, ctypes.c_int32, ctypes.POINTER(TuneEntry), i64,
                              ctypes.POINTER(i64)]),
        "bh_set_tuning": (i32, [_vp, ctypes.POINTER(TuneEntry), i64]),
        "bh_last_error": (ctypes.c_char_p, [_vp]),
        "bh_forces_static": (i32, [_vp, _vp, i64, f32, f32, _vp, _vp, _vp]),
        "bh_forces_static_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _dev_ptr(t, dtype, shape=None, name="tensor"):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s" % (name, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, shape, tuple(t.shape)))
    return _vp(t.data_ptr())


STATIC_MAX_N = 32768     # BH_STATIC_MAX_N


def forces_static(pos, mass, theta, eps, acc=None, pot=None, stream=None):
    """bh_forces_static: build and walk of one particle set (n <= STATIC_MAX_N)
    without any device allocation by the library.  pos (n, 3) and mass (n,) are
    float64 device tensors; acc (n, 3) and pot (n,) float32 device tensors are
    allocated here (by torch) unless given.  Synchronous.  Returns (acc, pot)."""
    import torch
    L = load_library()
    n = int(mass.shape[0])
    p = _dev_ptr(pos, torch.float64, (n, 3), "pos")
    m = _dev_ptr(mass, torch.float64, (n,), "mass")
    if acc is None:
        acc = torch.empty((n, 3), dtype=torch.float32, device=pos.device)
    if pot is None:
        pot = torch.empty((n,), dtype=torch.float32, device=pos.device)
    a = _dev_ptr(acc, torch.float32, (n, 3), "acc")
    q = _dev_ptr(pot, torch.float32, (n,), "pot")
    if stream is None:
        stream = torch.cuda.current_stream()
    st = L.bh_forces_static(p, m, n, float(theta), float(eps), a, q, _vp(stream.cuda_stream))
    if st:
        raise BHError(st, L.bh_forces_static_error().decode())
    return acc, pot


class Context:
    """One particle system on the device (bh_ctx)."""

    def __init__(self, nleaf=16, ncrit=64, max_n=0, hbm_budget_bytes=0, stream=None,
                 max_clusters=0):
        import torch
        self._L = load_library()
        p = Params(nleaf, ncrit, max_n, hbm_budget_bytes, max_clusters)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = _vp()
        st = self._L.bh_create(ctypes.byref(h), ctypes.byref(p), _vp(stream.cuda_stream))
        if st:
            raise BHError(st, "bh_create failed")
        self._h = h
        self.n = 0
        self.nleaf = nleaf
        self.ncrit = ncrit

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.bh_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, st):
        if st:
            raise BHError(st, self._L.bh_last_error(self._h).decode())

    # --- the method -------------------------------------------------------
    def build_tree(self, pos, mass):
        import torch
        n = int(pos.shape[0]) if pos.dim() == 2 else 0
        pp = _dev_ptr(pos, torch.float64, (n, 3), "pos")
        mp = _dev_ptr(mass, torch.float64, (n,), "mass")
        self._keep = (pos, mass)
        self._check(self._L.bh_build_tree(self._h, pp, mp, n))
        self._keep = None
        self.n = n
        self.k = 1

    # --- between rebuilds ---------------------------------------------------
    def drift(self, dt):
        self._check(self._L.bh_drift(self._h, float(dt)))

    def kick(self, dt, active=None):
        import torch
        self._check(self._L.bh_kick(self._h, float(dt),
                                    _dev_ptr(active, torch.uint8, (self.n,), "active")))

    def refit(self):
        self._check(self._L.bh_refit(self._h))

    def compute_forces_active(self, theta, eps, active, acc=None, pot=None, want=True):
        """Forces of the groups holding active particles (uint8 [n] device mask,
        caller order); the others keep their last values."""
        import torch
        if want and acc is None:
            acc = torch.empty((self.n, 3), dtype=torch.float32, device=self._device())
        if want and pot is None:
            pot = torch.empty((self.n,), dtype=torch.float32, device=self._device())
        self._check(self._L.bh_compute_forces_active(
            self._h, float(theta), float(eps), _dev_ptr(active, torch.uint8, (self.n,), "active"),
            _dev_ptr(acc, torch.float32, (self.n, 3), "acc"),
            _dev_ptr(pot, torch.float32, (self.n,), "pot")))
        return acc, pot

    # --- block time-steps ---------------------------------------------------
    @staticmethod
    def _block_params(dt_max, eta, length, max_level, growth):
        return BlockParams(float(dt_max), float(eta), float(length), int(max_level), float(growth))

    def block_bins(self, dt_max, eta, length, max_level, growth=0.0):
        """Bins (uint8 [n] device tensor, caller order) the next block step would
        use, and the particles per bin."""
        import torch
        bins = torch.empty((self.n,), dtype=torch.uint8, device=self._device())
        count = (ctypes.c_int64 * 16)()
        p = self._block_params(dt_max, eta, length, max_level, growth)
        self._check(self._L.bh_block_bins(self._h, ctypes.byref(p), _vp(bins.data_ptr()), count))
        return bins, list(count)

    def block_step(self, dt_max, eta, length, max_level, growth):
        """One block step; returns its statistics (bh_block_stats as a dict)."""
        p = self._block_params(dt_max, eta, length, max_level, growth)
        st = BlockStats()
        self._check(self._L.bh_block_step(self._h, ctypes.byref(p), ctypes.byref(st)))
        return st.as_dict()

    # --- batches ------------------------------------------------------------
    @staticmethod
    def _table(clusters):
        """clusters: sequence of dicts with n, theta, eps and optional dt, nleaf,
        ncrit (0: the context's), mac (MAC_EQ1 or MAC_MIN_DIST)."""
        arr = (Cluster * len(clusters))()
        for a, q in zip(arr, clusters):
            a.n = int(q["n"])
            a.theta = float(q["theta"])
            a.eps = float(q["eps"])
            a.dt = float(q.get("dt", 0.0))
            a.nleaf = int(q.get("nleaf", 0))
            a.ncrit = int(q.get("ncrit", 0))
            a.mac = int(q.get("mac", MAC_EQ1))
        return arr

    def batch_build(self, clusters, pos, mass, vel=None):
        """Load clusters (concatenated pos [N,3], mass [N], vel [N,3] or None)."""
        import torch
        n = int(sum(int(q["n"]) for q in clusters))
        tab = self._table(clusters)
        pp = _dev_ptr(pos, torch.float64, (n, 3), "pos")
        mp = _dev_ptr(mass, torch.float64, (n,), "mass")
        vp = _dev_ptr(vel, torch.float64, (n, 3), "vel")
        self._keep = (pos, mass, vel)
        self._check(self._L.bh_batch_build(self._h, tab, len(clusters), pp, mp, vp))
        self._keep = None
        self.n = n
        self.k = len(clusters)

    def batch_set_params(self, clusters):
        self._check(self._L.bh_batch_set_params(self._h, self._table(clusters), len(clusters)))

    def batch_forces(self, acc=None, pot=None, want=True):
        import torch
        if want and acc is None:
            acc = torch.empty((self.n, 3), dtype=torch.float32, device=self._device())
        if want and pot is None:
            pot = torch.empty((self.n,), dtype=torch.float32, device=self._device())
        ap = _dev_ptr(acc, torch.float32, (self.n, 3), "acc")
        pp = _dev_ptr(pot, torch.float32, (self.n,), "pot")
        self._check(self._L.bh_batch_forces(self._h, ap, pp))
        return acc, pot

    def batch_run(self, nsteps):
        self._check(self._L.bh_batch_run(self._h, int(nsteps)))

    def batch_energy(self):
        out = np.zeros((self.k, 7))
        self._check(self._L.bh_batch_energy(self._h, out.ctypes.data_as(_vp)))
        return out

    def autotune(self, reps=3):
        """Tune (nleaf, ncrit) per class (floor(log2 n), theta) of the loaded batch;
        returns the table (list of dicts) the context now holds."""
        cap = 64
        arr = (TuneEntry * cap)()
        cnt = ctypes.c_int64()
        self._check(self._L.bh_autotune(self._h, int(reps), arr, cap, ctypes.byref(cnt)))
        return [arr[i].as_dict() for i in range(min(cap, cnt.value))]

    def set_tuning(self, table):
        arr = (TuneEntry * max(1, len(table)))()
        for a, t in zip(arr, table):
            for k, _ in TuneEntry._fields_:
                setattr(a, k, t[k])
        self._check(self._L.bh_set_tuning(self._h, arr, len(table)))

    def set_mac(self, mac):
        """Opening test of every loaded cluster and of later bh_build_tree loads."""
        self._check(self._L.bh_set_mac(self._h, int(mac)))

    def set_velocities(self, vel):
        import torch
        self._check(self._L.bh_set_velocities(self._h, _dev_ptr(vel, torch.float64, (self.n, 3),
                                                                "vel")))

    def compute_forces(self, theta, eps, acc=None, pot=None, want=True):
        """Accelerations [n,3] and potentials [n] (float32, caller order)."""
        import torch
        if want and acc is None:
            acc = torch.empty((self.n, 3), dtype=torch.float32, device=self._device())
        if want and pot is None:
            pot = torch.empty((self.n,), dtype=torch.float32, device=self._device())
        ap = _dev_ptr(acc, torch.float32, (self.n, 3), "acc")
        pp = _dev_ptr(pot, torch.float32, (self.n,), "pot")
        self._check(self._L.bh_compute_forces(self._h, float(theta), float(eps), ap, pp))
        return acc, pot

    def leapfrog_step(self, dt):
        self._check(self._L.bh_leapfrog_step(self._h, float(dt)))

    def get_state(self, pos=None, vel=None, acc=None, pot=None):
        """Positions, velocities, accelerations and potentials in caller order.
        With no arguments all four are returned in new tensors; otherwise only the
        given caller-owned tensors are written (the others are skipped)."""
        import torch
        if pos is None and vel is None and acc is None and pot is None:
            dev = self._device()
            pos = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
            vel = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
            acc = torch.empty((self.n, 3), dtype=torch.float32, device=dev)
            pot = torch.empty((self.n,), dtype=torch.float32, device=dev)
        n = self.n
        self._check(self._L.bh_get_state(self._h, _dev_ptr(pos, torch.float64, (n, 3), "pos"),
                                         _dev_ptr(vel, torch.float64, (n, 3), "vel"),
                                         _dev_ptr(acc, torch.float32, (n, 3), "acc"),
                                         _dev_ptr(pot, torch.float32, (n,), "pot")))
        return pos, vel, acc, pot

    def get_positions(self):
        import torch
        dev = self._device()
        pos = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
        vel = torch.empty((self.n, 3), dtype=torch.float64, device=dev)
        self._check(self._L.bh_get_state(self._h, _vp(pos.data_ptr()), _vp(vel.data_ptr()),
                                         None, None))
        return pos, vel

    def set_state(self, pos, vel):
        import torch
        self._check(self._L.bh_set_state(self._h, _dev_ptr(pos, torch.float64, (self.n, 3), "pos"),
                                         _dev_ptr(vel, torch.float64, (self.n, 3), "vel")))

    def energy(self):
        out = np.zeros(7)
        self._check(self._L.bh_energy(self._h, out.ctypes.data_as(_vp)))
        return out

    def stats(self):
        s = Stats()
        self._check(self._L.bh_stats_get(self._h, ctypes.byref(s)))
        return s

    def export_tree(self):
        """Host copies of keys, sorted order, cells, moments, groups and counts."""
        s = self.stats()
        n, nc, ng = s.n, s.ncells, s.ngroups
        out = dict(
            key=np.zeros(n, np.uint64), perm=np.zeros(n, np.int64),
            level=np.zeros(nc, np.uint8), prefix=np.zeros(nc, np.uint64),
            first=np.zeros(nc, np.int64), count=np.zeros(nc, np.int64),
            is_leaf=np.zeros(nc, np.uint8), parent=np.zeros(nc, np.int64),
            child=np.zeros(nc, np.int64), nchild=np.zeros(nc, np.int32),
            mass=np.zeros(nc), com=np.zeros((nc, 3)), S=np.zeros((nc, 6)),
            rcrit2=np.zeros(nc, np.float32),
            gfirst=np.zeros(ng, np.int64), gcount=np.zeros(ng, np.int64),
            gcentre=np.zeros((ng, 3)), ghalf=np.zeros((ng, 3), np.float32),
            npp=np.zeros(ng, np.int64), npc=np.zeros(ng, np.int64))
        th = TreeHost(**{k: v.ctypes.data_as(_vp) for k, v in out.items()})
        self._check(self._L.bh_export_tree(self._h, ctypes.byref(th)))
        return out

    def _device(self):
        import torch
        return torch.device("cuda", torch.cuda.current_device())


class ServerParams(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_requests", ctypes.c_int64),
                ("nleaf", ctypes.c_int32), ("ncrit", ctypes.c_int32),
                ("min_nleaf", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("max_resident", ctypes.c_int64)]


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("pos", _vp), ("mass", _vp), ("vel", _vp),
                ("theta", ctypes.c_float), ("eps", ctypes.c_float), ("dt", ctypes.c_double),
                ("nsteps", ctypes.c_int32), ("nleaf", ctypes.c_int32), ("ncrit", ctypes.c_int32),
                ("mac", ctypes.c_int32), ("arrival", ctypes.c_double), ("out_pos", _vp),
                ("out_vel", _vp), ("out_acc", _vp), ("out_pot", _vp)]


class RequestStatus(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("units_done", ctypes.c_int32),
                ("arrival", ctypes.c_double), ("admitted", ctypes.c_double),
                ("completed", ctypes.c_double), ("energy", ctypes.c_double * 7)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "admitted", "completed", "rejected",
                                              "queued", "resident_requests", "resident_particles",
                                              "capacity_particles", "iterations",
                                              "particle_evals")] + \
               [(k, ctypes.c_double) for k in ("busy_seconds", "latency_p50", "latency_p99",
                                               "latency_max", "queue_wait_p50", "queue_wait_p99")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3


def _server_sigs(L):
    i32, i64 = ctypes.c_int, ctypes.c_int64
    sig = {
        "bh_server_create": (i32, [ctypes.POINTER(_vp), ctypes.POINTER(ServerParams), _vp]),
        "bh_server_destroy": (i32, [_vp]),
        "bh_server_submit": (i32, [_vp, ctypes.POINTER(Request), ctypes.POINTER(i64)]),
        "bh_server_step": (i32, [_vp, ctypes.POINTER(i64)]),
        "bh_server_poll": (i32, [_vp, i64, ctypes.POINTER(RequestStatus)]),
        "bh_server_release": (i32, [_vp, i64]),
        "bh_server_stats_get": (i32, [_vp, ctypes.POINTER(ServerStats)]),
        "bh_server_now": (i32, [_vp, ctypes.POINTER(ctypes.c_double)]),
        "bh_server_set_tuning": (i32, [_vp, ctypes.POINTER(TuneEntry), i64]),
        "bh_server_last_error": (ctypes.c_char_p, [_vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args


class Server:
    """The serving loop (bh_server): requests of one system each, admitted by the
    memory budget and advanced together one unit per iteration."""

    def __init__(self, hbm_budget_bytes, max_requests=256, nleaf=16, ncrit=64, min_nleaf=0,
                 stream=None, max_resident=0):
        import torch
        self._L = load_library()
        _server_sigs(self._L)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        p = ServerParams(int(hbm_budget_bytes), int(max_requests), int(nleaf), int(ncrit),
                         int(min_nleaf), 0, int(max_resident))
        h = _vp()
        st = self._L.bh_server_create(ctypes.byref(h), ctypes.byref(p), _vp(stream.cuda_stream))
        if st:
            raise BHError(st, "bh_server_create failed")
        self._h = h
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.bh_server_destroy(self._h)
        self._h = None
        self._keep = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st:
            raise BHError(st, self._L.bh_server_last_error(self._h).decode())

    def now(self):
        t = ctypes.c_double()
        self._check(self._L.bh_server_now(self._h, ctypes.byref(t)))
        return t.value

    def submit(self, pos, mass, vel=None, theta=0.75, eps=0.01, dt=1.0 / 128, nsteps=10,
               nleaf=0, ncrit=0, arrival=-1.0, out_pos=None, out_vel=None, out_acc=None,
               out_pot=None, mac=0):
        """Queue a request; the tensors are kept alive until it is done."""
        import torch
        n = int(pos.shape[0])
        r = Request()
        r.n = n
        r.pos = _dev_ptr(pos, torch.float64, (n, 3), "pos")
        r.mass = _dev_ptr(mass, torch.float64, (n,), "mass")
        r.vel = _dev_ptr(vel, torch.float64, (n, 3), "vel")
        r.theta, r.eps, r.dt, r.nsteps = float(theta), float(eps), float(dt), int(nsteps)
        r.nleaf, r.ncrit, r.arrival, r.mac = int(nleaf), int(ncrit), float(arrival), int(mac)
        r.out_pos = _dev_ptr(out_pos, torch.float64, (n, 3), "out_pos")
        r.out_vel = _dev_ptr(out_vel, torch.float64, (n, 3), "out_vel")
        r.out_acc = _dev_ptr(out_acc, torch.float32, (n, 3), "out_acc")
        r.out_pot = _dev_ptr(out_pot, torch.float32, (n,), "out_pot")
        t = ctypes.c_int64()
        self._check(self._L.bh_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = (pos, mass, vel, out_pos, out_vel, out_acc, out_pot)
        return t.value

    def set_tuning(self, table):
        arr = (TuneEntry * max(1, len(table)))()
        for a, t in zip(arr, table):
            for k, _ in TuneEntry._fields_:
                setattr(a, k, t[k])
        self._check(self._L.bh_server_set_tuning(self._h, arr, len(table)))

    def step(self):
        k = ctypes.c_int64()
        self._check(self._L.bh_server_step(self._h, ctypes.byref(k)))
        return k.value

    def poll(self, ticket):
        s = RequestStatus()
        self._check(self._L.bh_server_poll(self._h, int(ticket), ctypes.byref(s)))
        if s.state in (REQ_DONE, REQ_FAILED):
            self._keep.pop(int(ticket), None)
        return {"state": s.state, "units_done": s.units_done, "arrival": s.arrival,
                "admitted": s.admitted, "completed": s.completed, "energy": list(s.energy)}

    def release(self, ticket):
        """Drop the record of a finished request (later polls of it fail)."""
        self._check(self._L.bh_server_release(self._h, int(ticket)))
        self._keep.pop(int(ticket), None)

    def stats(self):
        s = ServerStats()
        self._check(self._L.bh_server_stats_get(self._h, ctypes.byref(s)))
        return s.as_dict()
