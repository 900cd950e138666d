"""CPU FP64 oracle for the Lennard-Jones MD hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
package. The product library never loads it, and it imports nothing from the product
package: the two share no code. ``oracle_md.c`` states the definitions it computes; this
module only compiles that file with gcc and marshals numpy arrays through ctypes.

Parity status: every function is pinned by CPU tests against O(N^2) brute force, closed
forms, lattice sums and conservation laws (see the tests directory); none is "parity
unpinned".
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle_md.c")
_LIB = os.path.join(_HERE, "liboracle_md.so")
# Test-only override: the mutation test points this at a deliberately broken build of the
# oracle to show that the pins catch it.
_LIB_OVERRIDE = os.environ.get("LJMD_ORACLE_LIB_OVERRIDE")

ORC_OK = 0
ORC_ERRORS = {-1: "invalid argument", -2: "out of memory", -4: "box too small",
              -5: "non-finite force", -6: "pair table incomplete"}


_NATIVE_LIB = os.path.join(_HERE, "liboracle_md_native.so")
# Flags of every build: optimised, no FMA contraction, no fast-math (the arithmetic is the
# definitions' as written). The native build adds -march=native for timing on the host it
# runs on; it is compiled there, on first use.
_FLAGS = ["-O3", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = True, native: bool = False) -> str:
    """Compile the oracle with gcc."""
    out = _NATIVE_LIB if native else _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp"
        cmd = ["gcc", *_FLAGS, *(["-march=native"] if native else []), "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


def build_flags(native: bool = False) -> str:
    return " ".join(["gcc", *_FLAGS, *(["-march=native"] if native else [])])


_lib = None
_use_native = False


def use_native_build():
    """Load the -march=native build (compiled on this host) instead of the portable one; only
    before the first oracle system of the process is created. Used for CPU timing."""
    global _use_native
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    _use_native = True


def _load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            lib = C.CDLL(_LIB_OVERRIDE)
        elif _use_native:
            lib = C.CDLL(build(force=True, native=True))
        else:
            build(force=False)
            lib = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        lp = C.POINTER(C.c_int64)
        lib.oracle_create.restype = C.c_void_p
        lib.oracle_create.argtypes = [C.c_int64, dp, dp, dp, ip, dp, C.c_int32, C.c_double,
                                      C.c_double]
        lib.oracle_destroy.argtypes = [C.c_void_p]
        lib.oracle_set_pair.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_double,
                                        C.c_double, C.c_double]
        lib.oracle_compute.argtypes = [C.c_void_p]
        lib.oracle_rebuild.argtypes = [C.c_void_p]
        lib.oracle_step.argtypes = [C.c_void_p, C.c_int64]
        lib.oracle_get_forces.argtypes = [C.c_void_p, dp]
        lib.oracle_get_energy.argtypes = [C.c_void_p, dp, dp]
        lib.oracle_get_virial.argtypes = [C.c_void_p, dp]
        lib.oracle_get_per_particle.argtypes = [C.c_void_p, dp, dp]
        lib.oracle_get_state.argtypes = [C.c_void_p, dp, dp, ip, lp]
        lib.oracle_get_pairs.argtypes = [C.c_void_p, lp, ip, dp]
        lib.oracle_get_counters.argtypes = [C.c_void_p, lp, lp]
        lib.oracle_set_nvt.argtypes = [C.c_void_p, C.c_double, C.c_double]
        lib.oracle_set_pair_style.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, dp,
                                              C.c_double]
        lib.oracle_set_nve.argtypes = [C.c_void_p]
        lib.oracle_get_thermostat.argtypes = [C.c_void_p, dp, dp, dp]
        lib.oracle_set_thermostat.argtypes = [C.c_void_p, C.c_double, C.c_double]
        lib.oracle_negate_velocities.argtypes = [C.c_void_p]
        lib.oracle_set_shift_mode.argtypes = [C.c_void_p, C.c_int32]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class OracleError(RuntimeError):
    pass


def _check(rc):
    if rc != ORC_OK:
        raise OracleError(f"oracle status {rc}: {ORC_ERRORS.get(rc, 'unknown')}")


class OracleSystem:
    """FP64 CPU reference system. Arrays are in input (tag) order."""

    def __init__(self, box, pos, vel, types, ntypes, pairs, dt=0.005, skin=0.4, mass=None):
        lib = _load()
        self._box = np.ascontiguousarray(box, dtype=np.float64).reshape(3)
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3)
        typ = np.ascontiguousarray(types, dtype=np.int32).reshape(-1)
        self.n = pos.shape[0]
        m = None if mass is None else np.ascontiguousarray(mass, dtype=np.float64)
        h = lib.oracle_create(self.n, _dp(self._box), _dp(pos), _dp(vel), _ip(typ),
                              None if m is None else _dp(m), int(ntypes), float(dt),
                              float(skin))
        if not h:
            raise OracleError("oracle_create rejected its arguments")
        self._h = h
        self._lib = lib
        for (a, b, eps, sig, rc) in pairs:
            self.set_pair(a, b, eps, sig, rc)

    @classmethod
    def from_spec(cls, spec, dt=0.005, skin=0.4):
        return cls(spec.box, spec.pos, spec.vel, spec.type, spec.ntypes, spec.pairs, dt, skin)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.oracle_destroy(h)
            self._h = None

    def set_pair(self, a, b, eps, sig, rc):
        _check(self._lib.oracle_set_pair(self._h, a, b, eps, sig, rc))

    def compute(self):
        _check(self._lib.oracle_compute(self._h))

    def rebuild(self):
        _check(self._lib.oracle_rebuild(self._h))

    def step(self, n):
        _check(self._lib.oracle_step(self._h, int(n)))

    def forces(self):
        out = np.empty((self.n, 3))
        _check(self._lib.oracle_get_forces(self._h, _dp(out)))
        return out

    def energy(self):
        u = np.zeros(1)
        k = np.zeros(1)
        _check(self._lib.oracle_get_energy(self._h, _dp(u), _dp(k)))
        return float(u[0]), float(k[0])

    def virial(self):
        out = np.empty(6)
        _check(self._lib.oracle_get_virial(self._h, _dp(out)))
        return out

    def per_particle(self):
        u = np.empty(self.n)
        w = np.empty((self.n, 6))
        _check(self._lib.oracle_get_per_particle(self._h, _dp(u), _dp(w)))
        return u, w

    def state(self):
        pos = np.empty((self.n, 3))
        vel = np.empty((self.n, 3))
        img = np.empty((self.n, 3), dtype=np.int32)
        st = C.c_int64(0)
        _check(self._lib.oracle_get_state(self._h, _dp(pos), _dp(vel), _ip(img), C.byref(st)))
        return pos, vel, img, int(st.value)

    def pairs(self):
        """Current half list as an (M, 2) int32 array of (i < j) pairs, plus the build
        positions."""
        cnt = C.c_int64(0)
        _check(self._lib.oracle_get_pairs(self._h, C.byref(cnt), None, None))
        out = np.empty((cnt.value, 2), dtype=np.int32)
        xb = np.empty((self.n, 3))
        _check(self._lib.oracle_get_pairs(self._h, C.byref(cnt), _ip(out), _dp(xb)))
        return out, xb

    STYLES = {"lj": 0, "mie": 1, "gauss": 2, "yukawa": 3}

    def set_pair_style(self, a, b, style, params, rc):
        """A pair of another form: 'mie' (eps, sigma, n, m), 'gauss' (eps, sigma),
        'yukawa' (eps, kappa), or 'lj' (eps, sigma)."""
        p = np.zeros(4)
        p[:len(params)] = params
        _check(self._lib.oracle_set_pair_style(self._h, a, b, self.STYLES[style], _dp(p),
                                               float(rc)))

    SHIFTS = {"energy": 0, "force": 1}

    def set_shift_mode(self, mode):
        """'energy': the energy is shifted to 0 at r_cut, the force is not (the default);
        'force': the force is shifted too (shifted-force form, both vanish at r_cut)."""
        _check(self._lib.oracle_set_shift_mode(self._h, self.SHIFTS[mode]))

    def set_nvt(self, kT, tau):
        """NVT (Nose-Hoover, symmetric splitting) at kT with time constant tau; tau may be
        float('inf') for zero coupling."""
        _check(self._lib.oracle_set_nvt(self._h, float(kT), float(tau)))

    def set_nve(self):
        _check(self._lib.oracle_set_nve(self._h))

    def thermostat(self):
        """(xi, eta, thermostat energy Q xi^2/2 + N_f kT eta)."""
        out = np.zeros(3)
        _check(self._lib.oracle_get_thermostat(self._h, _dp(out[0:1]), _dp(out[1:2]),
                                               _dp(out[2:3])))
        return float(out[0]), float(out[1]), float(out[2])

    def set_thermostat(self, xi, eta):
        _check(self._lib.oracle_set_thermostat(self._h, float(xi), float(eta)))

    def negate_velocities(self):
        _check(self._lib.oracle_negate_velocities(self._h))

    def counters(self):
        st = C.c_int64(0)
        b = C.c_int64(0)
        _check(self._lib.oracle_get_counters(self._h, C.byref(st), C.byref(b)))
        return int(st.value), int(b.value)
