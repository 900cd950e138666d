"""Python binding of libljmd (include/ljmd.h): argument marshalling only.

Every step of the computation runs in the HIP kernels of libljmd.so. PyTorch, when it has a
GPU, only supplies device memory (its caching allocator, through the allocator callbacks
of ljmd_config) and the stream the library enqueues on. If the shared library is missing
this module raises instead of falling back to anything else.
"""

from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libljmd.so")
# the same sources built with the device checks of LJMD_DEBUG_CHECKS (build_lib, debug=True),
# loaded instead when the environment sets LJMD_DEBUG_CHECKS=1
LIB_DEBUG_PATH = os.path.join(HERE, "libljmd_debug.so")

LJMD_OK = 0
LJMD_E_INVAL = -1
LJMD_E_NOMEM = -2
LJMD_E_DEVICE = -3
LJMD_E_BOX = -4
LJMD_E_NONFINITE = -5
LJMD_E_STATE = -6
LJMD_E_CAPACITY = -7
LJMD_FP64 = 0
LJMD_MIXED = 1
LJMD_MAX_TYPES = 16

_ERRNAMES = {LJMD_E_INVAL: "INVAL", LJMD_E_NOMEM: "NOMEM", LJMD_E_DEVICE: "DEVICE",
             LJMD_E_BOX: "BOX", LJMD_E_NONFINITE: "NONFINITE", LJMD_E_STATE: "STATE",
             LJMD_E_CAPACITY: "CAPACITY"}

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class LjmdConfig(C.Structure):
    _fields_ = [("box", C.c_double * 3), ("ntypes", C.c_int32), ("dt", C.c_double),
                ("skin", C.c_double), ("precision", C.c_int32), ("nlist_capacity", C.c_int32),
                ("threads_per_particle", C.c_int32), ("block_size", C.c_int32),
                ("graph_steps", C.c_int32), ("stream", C.c_void_p), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("alloc_ctx", C.c_void_p)]


class LjmdStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("rebuilds", C.c_int64), ("max_neighbors", C.c_int32),
                ("nlist_capacity", C.c_int32), ("overflow_retries", C.c_int64),
                ("threads_per_particle", C.c_int32), ("block_size", C.c_int32),
                ("ncell", C.c_int32 * 3), ("graph_steps", C.c_int32),
                ("device_bytes", C.c_int64), ("list_entries", C.c_int64)]


class LjmdBatchConfig(C.Structure):
    _fields_ = [("budget_bytes", C.c_int64), ("max_slots", C.c_int32), ("precision", C.c_int32),
                ("dt", C.c_double), ("skin", C.c_double), ("block_steps", C.c_int32),
                ("threads_per_particle", C.c_int32), ("block_size", C.c_int32),
                ("nlist_capacity", C.c_int32), ("stream", C.c_void_p), ("alloc", ALLOC_FN),
                ("free", FREE_FN), ("alloc_ctx", C.c_void_p)]


class LjmdReplicaSpec(C.Structure):
    _fields_ = [("box", C.c_double * 3), ("n", C.c_int64), ("pos", C.POINTER(C.c_double)),
                ("vel", C.POINTER(C.c_double)), ("type", C.POINTER(C.c_int32)),
                ("ntypes", C.c_int32), ("eps", C.POINTER(C.c_double)),
                ("sigma", C.POINTER(C.c_double)), ("r_cut", C.POINTER(C.c_double)),
                ("nsteps", C.c_int64)]


class LjmdBatchStats(C.Structure):
    _fields_ = [("resident", C.c_int32), ("running", C.c_int32), ("blocks", C.c_int64),
                ("overflow_reruns", C.c_int64), ("rebuilds", C.c_int64),
                ("nlist_capacity", C.c_int32), ("threads_per_particle", C.c_int32),
                ("block_size", C.c_int32), ("tile_capacity", C.c_int32),
                ("device_bytes", C.c_int64), ("used_bytes", C.c_int64),
                ("budget_bytes", C.c_int64)]


class LjmdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"LJMD_E_{_ERRNAMES.get(code, code)} ({code}): {msg}")
        self.code = code


_lib = None

class LjmdTuningEntry(C.Structure):
    _fields_ = [("precision", C.c_int32), ("multi_type", C.c_int32), ("size_bucket", C.c_int32),
                ("threads_per_particle", C.c_int32), ("block_size", C.c_int32)]


EXPORTED = [
    "ljmd_system_create", "ljmd_system_destroy", "ljmd_pair_lj_set", "ljmd_pair_set",
    "ljmd_step",
    "ljmd_get_forces", "ljmd_get_energy", "ljmd_get_virial", "ljmd_get_per_particle",
    "ljmd_get_state", "ljmd_set_state", "ljmd_get_neighbor_pairs", "ljmd_get_neighbor_list",
    "ljmd_get_stats", "ljmd_set_nlist", "ljmd_set_pair_shift", "ljmd_set_nvt", "ljmd_set_nve", "ljmd_get_thermostat",
    "ljmd_set_thermostat", "ljmd_negate_velocities", "ljmd_set_thermo", "ljmd_get_thermo",
    "ljmd_set_kernel_timing", "ljmd_kernel_time", "ljmd_kernel_durations", "ljmd_last_error", "ljmd_version",
    "ljmd_batch_create", "ljmd_batch_destroy", "ljmd_batch_footprint", "ljmd_batch_admit",
    "ljmd_batch_run_block", "ljmd_batch_poll", "ljmd_batch_read", "ljmd_batch_slot_steps",
    "ljmd_batch_slot_status", "ljmd_batch_read_noalloc",
    "ljmd_batch_release", "ljmd_batch_get_stats", "ljmd_tuning_get", "ljmd_tuning_set",
]


def load(path: str | None = None):
    """Load libljmd.so (libljmd_debug.so when LJMD_DEBUG_CHECKS=1); raises if it has not been
    built. A process keeps the first library it loads."""
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = LIB_DEBUG_PATH if os.environ.get("LJMD_DEBUG_CHECKS") == "1" else LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1308_5587_amd.build_lib.build()")
    lib = C.CDLL(path)
    vp, dp, ip, lp = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    sig = {
        "ljmd_system_create": ([C.POINTER(LjmdConfig), C.c_int64, dp, dp, ip, dp, C.POINTER(vp)], C.c_int),
        "ljmd_system_destroy": ([vp], None),
        "ljmd_pair_lj_set": ([vp, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double], C.c_int),
        "ljmd_pair_set": ([vp, C.c_int32, C.c_int32, C.c_int32, dp, C.c_int32, C.c_double],
                          C.c_int),
        "ljmd_step": ([vp, C.c_int64], C.c_int),
        "ljmd_get_forces": ([vp, dp], C.c_int),
        "ljmd_get_energy": ([vp, dp, dp], C.c_int),
        "ljmd_get_virial": ([vp, dp], C.c_int),
        "ljmd_get_per_particle": ([vp, dp, dp], C.c_int),
        "ljmd_get_state": ([vp, dp, dp, ip, lp], C.c_int),
        "ljmd_set_state": ([vp, dp, dp, ip, lp], C.c_int),
        "ljmd_get_neighbor_pairs": ([vp, lp, ip, dp], C.c_int),
        "ljmd_get_neighbor_list": ([vp, ip, lp, ip, dp], C.c_int),
        "ljmd_get_stats": ([vp, C.POINTER(LjmdStats)], C.c_int),
        "ljmd_set_nlist": ([vp, C.c_int32], C.c_int),
        "ljmd_set_pair_shift": ([vp, C.c_int32], C.c_int),
        "ljmd_set_nvt": ([vp, C.c_double, C.c_double], C.c_int),
        "ljmd_set_nve": ([vp], C.c_int),
        "ljmd_get_thermostat": ([vp, dp, dp, dp], C.c_int),
        "ljmd_set_thermostat": ([vp, C.c_double, C.c_double], C.c_int),
        "ljmd_set_thermo": ([vp, C.c_int32, C.c_int32], C.c_int),
        "ljmd_get_thermo": ([vp, dp, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
        "ljmd_negate_velocities": ([vp], C.c_int),
        "ljmd_set_kernel_timing": ([vp, C.c_int32], C.c_int),
        "ljmd_kernel_time": ([vp, lp, dp], C.c_int),
        "ljmd_kernel_durations": ([vp, C.c_int32, lp, C.POINTER(C.c_float)], C.c_int),
        "ljmd_last_error": ([], C.c_char_p),
        "ljmd_version": ([], C.c_char_p),
        "ljmd_batch_create": ([C.POINTER(LjmdBatchConfig), C.POINTER(vp)], C.c_int),
        "ljmd_batch_destroy": ([vp], None),
        "ljmd_batch_footprint": ([vp, C.POINTER(LjmdReplicaSpec), lp], C.c_int),
        "ljmd_batch_admit": ([vp, C.POINTER(LjmdReplicaSpec), ip], C.c_int),
        "ljmd_batch_run_block": ([vp], C.c_int),
        "ljmd_batch_poll": ([vp, ip, ip], C.c_int),
        "ljmd_batch_read": ([vp, C.c_int32, dp, dp, dp, dp, dp], C.c_int),
        "ljmd_batch_read_noalloc": ([vp, C.c_int32, dp, dp, dp, dp, dp], C.c_int),
        "ljmd_batch_slot_steps": ([vp, C.c_int32, lp], C.c_int),
        "ljmd_batch_slot_status": ([vp, C.c_int32, ip], C.c_int),
        "ljmd_batch_release": ([vp, C.c_int32], C.c_int),
        "ljmd_batch_get_stats": ([vp, C.POINTER(LjmdBatchStats)], C.c_int),
        "ljmd_tuning_get": ([C.POINTER(LjmdTuningEntry), C.c_int32, ip], C.c_int),
        "ljmd_tuning_set": ([C.POINTER(LjmdTuningEntry), C.c_int32], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc):
    if rc != LJMD_OK:
        raise LjmdError(rc, _lib.ljmd_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _torch_cuda():
    try:
        import torch
    except Exception:
        return None
    try:
        if torch.cuda.is_available():
            return torch
    except Exception:
        return None
    return None


class _TorchAllocator:
    """ljmd allocator callbacks backed by torch's caching allocator."""

    def __init__(self, torch, device):
        self.torch = torch
        self.device = device

        def _alloc(nbytes, stream, ctx):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                              stream or 0))
            except Exception:
                return None

        def _free(ptr, nbytes, stream, ctx):
            try:
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:
                pass

        self.alloc = ALLOC_FN(_alloc)
        self.free = FREE_FN(_free)


class System:
    """One LJ system on the GPU (ljmd_system). Arrays in and out are numpy, tag order."""

    def __init__(self, box, pos, vel, types, ntypes=None, pairs=(), dt=0.005, skin=0.4,
                 precision="fp64", mass=None, nlist_capacity=0, threads_per_particle=0,
                 block_size=0, graph_steps=0, stream=None, torch_memory=True):
        lib = load()
        self._lib = lib
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3)
        typ = np.ascontiguousarray(types, dtype=np.int32).reshape(-1)
        self.n = pos.shape[0]
        if ntypes is None:
            ntypes = int(typ.max()) + 1 if self.n else 1
        cfg = LjmdConfig()
        for a in range(3):
            cfg.box[a] = float(np.asarray(box, dtype=np.float64).reshape(3)[a])
        cfg.ntypes = int(ntypes)
        cfg.dt = float(dt)
        cfg.skin = float(skin)
        cfg.precision = {"fp64": LJMD_FP64, "mixed": LJMD_MIXED}[precision]
        cfg.nlist_capacity = int(nlist_capacity)
        cfg.threads_per_particle = int(threads_per_particle)
        cfg.block_size = int(block_size)
        cfg.graph_steps = int(graph_steps)
        self._alloc = None
        torch = _torch_cuda()
        if torch is not None:
            dev = torch.cuda.current_device()
            if stream is None:
                stream = torch.cuda.current_stream(dev).cuda_stream
            if torch_memory:
                self._alloc = _TorchAllocator(torch, dev)
                cfg.alloc = self._alloc.alloc
                cfg.free = self._alloc.free
        cfg.stream = stream if stream else None
        self._cfg = cfg
        m = None if mass is None else np.ascontiguousarray(mass, dtype=np.float64)
        h = C.c_void_p()
        _check(lib.ljmd_system_create(C.byref(cfg), self.n, _dp(pos), _dp(vel), _ip(typ),
                                      None if m is None else _dp(m), C.byref(h)))
        self._h = h
        for (a, b, eps, sig, rc) in pairs:
            self.pair_lj_set(a, b, eps, sig, rc)

    @classmethod
    def from_spec(cls, spec, **kw):
        return cls(spec.box, spec.pos, spec.vel, spec.type, spec.ntypes, spec.pairs, **kw)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.ljmd_system_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pair_lj_set(self, a, b, epsilon, sigma, r_cut):
        _check(self._lib.ljmd_pair_lj_set(self._h, int(a), int(b), float(epsilon), float(sigma),
                                          float(r_cut)))

    PAIR_FORMS = {"lj": 0, "mie": 1, "gauss": 2, "yukawa": 3, "wca": 4}

    def pair_set(self, a, b, form, params, r_cut):
        """Pair (a, b) of another form: 'mie' (eps, sigma, n, m), 'gauss' (eps, sigma),
        'yukawa' (eps, kappa), 'wca' (eps, sigma; r_cut 0) or 'lj' (eps, sigma)."""
        p = np.ascontiguousarray(params, dtype=np.float64)
        _check(self._lib.ljmd_pair_set(self._h, a, b, self.PAIR_FORMS[form], _dp(p), len(p),
                                       float(r_cut)))

    def step(self, nsteps=1):
        _check(self._lib.ljmd_step(self._h, int(nsteps)))

    def forces(self):
        out = np.empty((self.n, 3))
        _check(self._lib.ljmd_get_forces(self._h, _dp(out)))
        return out

    def energy(self):
        u = np.zeros(1)
        k = np.zeros(1)
        _check(self._lib.ljmd_get_energy(self._h, _dp(u), _dp(k)))
        return float(u[0]), float(k[0])

    def virial(self):
        out = np.empty(6)
        _check(self._lib.ljmd_get_virial(self._h, _dp(out)))
        return out

    def per_particle(self):
        u = np.empty(self.n)
        w = np.empty((self.n, 6))
        _check(self._lib.ljmd_get_per_particle(self._h, _dp(u), _dp(w)))
        return u, w

    def state(self):
        pos = np.empty((self.n, 3))
        vel = np.empty((self.n, 3))
        img = np.empty((self.n, 3), dtype=np.int32)
        st = C.c_int64(0)
        _check(self._lib.ljmd_get_state(self._h, _dp(pos), _dp(vel), _ip(img), C.byref(st)))
        return pos, vel, img, int(st.value)

    def set_state(self, pos, vel, img=None, step=None):
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3)
        im = None if img is None else np.ascontiguousarray(img, dtype=np.int32).reshape(-1, 3)
        st = None if step is None else C.byref(C.c_int64(int(step)))
        _check(self._lib.ljmd_set_state(self._h, _dp(pos), _dp(vel),
                                        None if im is None else _ip(im), st))

    def neighbor_pairs(self):
        cnt = C.c_int64(0)
        _check(self._lib.ljmd_get_neighbor_pairs(self._h, C.byref(cnt), None, None))
        out = np.empty((cnt.value, 2), dtype=np.int32)
        xb = np.empty((self.n, 3))
        _check(self._lib.ljmd_get_neighbor_pairs(self._h, C.byref(cnt), _ip(out), _dp(xb)))
        return out, xb

    NLIST_METHODS = {"cell": 0, "tree": 1}

    def set_nlist(self, method):
        """Neighbour-list method: 'cell' (default) or 'tree' (one BVH per type)."""
        _check(self._lib.ljmd_set_nlist(self._h, self.NLIST_METHODS[method]))

    SHIFT_MODES = {"energy": 0, "force": 1}

    def set_pair_shift(self, mode):
        """Truncation of every pair form at r_cut: 'energy' (default; energy shifted to 0,
        force not) or 'force' (shifted force: both vanish at r_cut)."""
        _check(self._lib.ljmd_set_pair_shift(self._h, self.SHIFT_MODES[mode]))

    def set_nvt(self, kT, tau):
        """NVT at kT with thermostat time constant tau (float('inf'): zero coupling)."""
        _check(self._lib.ljmd_set_nvt(self._h, float(kT), float(tau)))

    def set_nve(self):
        _check(self._lib.ljmd_set_nve(self._h))

    def thermostat(self):
        """(xi, eta, thermostat energy Q xi^2/2 + N_f kT eta)."""
        out = np.zeros(3)
        _check(self._lib.ljmd_get_thermostat(self._h, _dp(out[0:1]), _dp(out[1:2]),
                                             _dp(out[2:3])))
        return float(out[0]), float(out[1]), float(out[2])

    def set_thermostat(self, xi, eta):
        _check(self._lib.ljmd_set_thermostat(self._h, float(xi), float(eta)))

    def negate_velocities(self):
        _check(self._lib.ljmd_negate_velocities(self._h))

    THERMO_COLUMNS = ("step", "K", "U", "E", "T", "P", "Wxx", "Wxy", "Wxz", "Wyy", "Wyz", "Wzz")

    def set_thermo(self, period, capacity=1024):
        """Sample (step, K, U, E, T, P, W) every `period` steps into a device ring of
        `capacity` rows (period 0: off)."""
        _check(self._lib.ljmd_set_thermo(self._h, int(period), int(capacity)))

    def thermo(self, max_rows=None):
        """The latest samples, oldest first: an array of rows with THERMO_COLUMNS."""
        n = C.c_int32(0)
        _check(self._lib.ljmd_get_thermo(self._h, None, 0, C.byref(n)))
        k = n.value if max_rows is None else min(n.value, int(max_rows))
        out = np.zeros((k, len(self.THERMO_COLUMNS)))
        if k:
            _check(self._lib.ljmd_get_thermo(self._h, _dp(out), k, C.byref(n)))
        return out[: n.value]

    def neighbor_list(self):
        """The full list: (counts[n], neighbours[total]) with rows in tag order and each
        row's entries in stored order, plus the build positions."""
        tot = C.c_int64(0)
        counts = np.empty(self.n, dtype=np.int32)
        _check(self._lib.ljmd_get_neighbor_list(self._h, _ip(counts), C.byref(tot), None, None))
        nb = np.empty(max(1, tot.value), dtype=np.int32)
        xb = np.empty((self.n, 3))
        _check(self._lib.ljmd_get_neighbor_list(self._h, _ip(counts), C.byref(tot), _ip(nb),
                                                _dp(xb)))
        return counts, nb[:tot.value], xb

    def stats(self):
        st = LjmdStats()
        _check(self._lib.ljmd_get_stats(self._h, C.byref(st)))
        return {f: (list(getattr(st, f)) if f == "ncell" else getattr(st, f))
                for f, _ in LjmdStats._fields_}

    def set_kernel_timing(self, on=True):
        _check(self._lib.ljmd_set_kernel_timing(self._h, 1 if on else 0))

    KERNEL_KINDS = ("step", "bin", "scan", "scatter", "gather", "nlist")

    def kernel_durations(self):
        """Per-launch durations (ms) recorded while kernel timing was on, by kernel kind."""
        out = {}
        for k, name in enumerate(self.KERNEL_KINDS):
            cnt = C.c_int64(0)
            _check(self._lib.ljmd_kernel_durations(self._h, k, C.byref(cnt), None))
            buf = np.empty(max(1, cnt.value), dtype=np.float32)
            _check(self._lib.ljmd_kernel_durations(self._h, k, C.byref(cnt),
                                                    buf.ctypes.data_as(C.POINTER(C.c_float))))
            out[name] = buf[:cnt.value].astype(np.float64)
        return out

    def kernel_time(self):
        n = C.c_int64(0)
        ms = C.c_double(0.0)
        _check(self._lib.ljmd_kernel_time(self._h, C.byref(n), C.byref(ms)))
        return int(n.value), float(ms.value)


def pair_tables(ntypes, pairs):
    """(eps, sigma, r_cut) as symmetric ntypes x ntypes float64 tables from a list of
    (a, b, epsilon, sigma, r_cut); unlisted pairs get r_cut = 0 (no interaction)."""
    eps = np.zeros((ntypes, ntypes))
    sig = np.ones((ntypes, ntypes))
    rc = np.zeros((ntypes, ntypes))
    for (a, b, e, sg, r) in pairs:
        for (i, j) in ((a, b), (b, a)):
            eps[i, j], sig[i, j], rc[i, j] = e, sg, r
    return eps, sig, rc


class _ReplicaRequest:
    """A replica spec in C layout; owns the arrays it points to."""

    def __init__(self, spec, nsteps):
        self.pos = np.ascontiguousarray(spec.pos, dtype=np.float64).reshape(-1, 3)
        self.vel = np.ascontiguousarray(spec.vel, dtype=np.float64).reshape(-1, 3)
        self.typ = np.ascontiguousarray(spec.type, dtype=np.int32).reshape(-1)
        self.eps, self.sig, self.rc = (np.ascontiguousarray(t) for t in
                                       pair_tables(int(spec.ntypes), spec.pairs))
        c = LjmdReplicaSpec()
        for a in range(3):
            c.box[a] = float(np.asarray(spec.box, dtype=np.float64).reshape(3)[a])
        c.n = self.pos.shape[0]
        c.pos = _dp(self.pos)
        c.vel = _dp(self.vel)
        c.type = _ip(self.typ)
        c.ntypes = int(spec.ntypes)
        c.eps = _dp(self.eps)
        c.sigma = _dp(self.sig)
        c.r_cut = _dp(self.rc)
        c.nsteps = int(nsteps)
        self.c = c


class Batch:
    """Many independent LJ replicas on the GPU (ljmd_batch): admit, run blocks, poll, read,
    release. Arrays in and out are numpy, tag order."""

    def __init__(self, budget_bytes, max_slots, precision="mixed", dt=0.005, skin=0.4,
                 block_steps=100, threads_per_particle=0, block_size=0, nlist_capacity=0,
                 stream=None, torch_memory=True):
        lib = load()
        self._lib = lib
        cfg = LjmdBatchConfig()
        cfg.budget_bytes = int(budget_bytes)
        cfg.max_slots = int(max_slots)
        cfg.precision = {"fp64": LJMD_FP64, "mixed": LJMD_MIXED}[precision]
        cfg.dt = float(dt)
        cfg.skin = float(skin)
        cfg.block_steps = int(block_steps)
        cfg.threads_per_particle = int(threads_per_particle)
        cfg.block_size = int(block_size)
        cfg.nlist_capacity = int(nlist_capacity)
        self._alloc = None
        torch = _torch_cuda()
        if torch is not None:
            dev = torch.cuda.current_device()
            if stream is None:
                stream = torch.cuda.current_stream(dev).cuda_stream
            if torch_memory:
                self._alloc = _TorchAllocator(torch, dev)
                cfg.alloc = self._alloc.alloc
                cfg.free = self._alloc.free
        cfg.stream = stream if stream else None
        self._cfg = cfg
        self.max_slots = int(max_slots)
        self.block_steps = int(block_steps) if block_steps else 100
        self._n = {}
        h = C.c_void_p()
        _check(lib.ljmd_batch_create(C.byref(cfg), C.byref(h)))
        self._h = h

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.ljmd_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def footprint(self, spec, nsteps=1):
        req = _ReplicaRequest(spec, nsteps)
        out = C.c_int64(0)
        _check(self._lib.ljmd_batch_footprint(self._h, C.byref(req.c), C.byref(out)))
        return int(out.value)

    def admit(self, spec, nsteps):
        """Admit a replica for nsteps steps; returns its slot. Raises LjmdError (code
        LJMD_E_CAPACITY when no slot or budget is free)."""
        req = _ReplicaRequest(spec, nsteps)
        slot = C.c_int32(-1)
        _check(self._lib.ljmd_batch_admit(self._h, C.byref(req.c), C.byref(slot)))
        self._n[int(slot.value)] = req.pos.shape[0]
        return int(slot.value)

    def run_block(self):
        _check(self._lib.ljmd_batch_run_block(self._h))

    def poll(self):
        out = np.empty(self.max_slots, dtype=np.int32)
        k = C.c_int32(0)
        _check(self._lib.ljmd_batch_poll(self._h, _ip(out), C.byref(k)))
        return [int(v) for v in out[:k.value]]

    def slot_status(self, slot):
        """LJMD_OK, or the status the replica in `slot` was retired with."""
        out = C.c_int32(0)
        _check(self._lib.ljmd_batch_slot_status(self._h, int(slot), C.byref(out)))
        return int(out.value)

    def slot_steps(self, slot):
        out = C.c_int64(0)
        _check(self._lib.ljmd_batch_slot_steps(self._h, int(slot), C.byref(out)))
        return int(out.value)

    def read(self, slot, energy=True, noalloc=False):
        """Results of a finished slot; noalloc reads through ljmd_batch_read_noalloc (no device
        allocation; replicas of at most 349,525 particles)."""
        n = max(1, self._n.get(int(slot), 0))  # an unknown slot gets LJMD_E_STATE below
        pos = np.empty((n, 3))
        vel = np.empty((n, 3))
        f = np.empty((n, 3))
        e = np.zeros(2)
        w = np.zeros(6)
        fn = self._lib.ljmd_batch_read_noalloc if noalloc else self._lib.ljmd_batch_read
        _check(fn(self._h, int(slot), _dp(pos), _dp(vel), _dp(f),
                  _dp(e) if energy else None, _dp(w) if energy else None))
        out = {"pos": pos, "vel": vel, "forces": f}
        if energy:
            out.update(potential=float(e[0]), kinetic=float(e[1]), virial=w)
        return out

    def stats(self):
        st = LjmdBatchStats()
        _check(self._lib.ljmd_batch_get_stats(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in LjmdBatchStats._fields_}

    def release(self, slot):
        _check(self._lib.ljmd_batch_release(self._h, int(slot)))
        self._n.pop(int(slot), None)


def version():
    return load().ljmd_version().decode()


_TUNING_FIELDS = ("precision", "multi_type", "size_bucket", "threads_per_particle", "block_size")


def tuning_table():
    """The process-wide tuning table of single systems, as a list of dicts ordered by key
    (precision, multi_type, size_bucket) with the chosen threads_per_particle and
    block_size."""
    lib = load()
    n = C.c_int32(0)
    _check(lib.ljmd_tuning_get(None, 0, C.byref(n)))
    buf = (LjmdTuningEntry * max(1, n.value))()
    _check(lib.ljmd_tuning_get(buf, n.value, C.byref(n)))
    return [{f: int(getattr(buf[k], f)) for f in _TUNING_FIELDS} for k in range(n.value)]


def set_tuning(entries):
    """Preload (freeze) tuning choices: systems created afterwards whose key is given take
    the stored lanes per particle and workgroup size without timing runs."""
    lib = load()
    entries = list(entries)
    buf = (LjmdTuningEntry * max(1, len(entries)))()
    for k, e in enumerate(entries):
        for f in _TUNING_FIELDS:
            setattr(buf[k], f, int(e[f]))
    _check(lib.ljmd_tuning_set(buf, len(entries)))


def save_tuning(path):
    """Write the tuning table to a JSON file."""
    with open(path, "w") as f:
        json.dump({"ljmd_tuning": tuning_table()}, f, indent=1)


def load_tuning(path):
    """Preload the tuning table from a JSON file written by save_tuning."""
    with open(path) as f:
        set_tuning(json.load(f)["ljmd_tuning"])
