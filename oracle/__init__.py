"""ctypes wrapper of the plain-C oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product package
(``paper_2302_08252_amd``) never imports this module, and this module never
imports the product package.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
HDR = os.path.join(HERE, "oracle.h")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]

SPARSE, DENSE = 0, 1
FP64, MIXED = 0, 1
AOS, SOA, AOSOA = 0, 1, 2
ELECTRON, POSITRON, GAMMA = 0, 1, 2
T_DEP_CONT, T_DEP_CUT, T_LAYER, T_ESCAPED, T_ROUND, T_INFLIGHT, T_CELLS, T_EIN = range(8)
OK, E_INVALID, E_CAPACITY, E_STATE, E_NOMEM = 0, -1, -2, -4, -5

TRACK_DTYPE = np.dtype(
    [
        ("pos", "<f8", (3,)),
        ("dir", "<f8", (3,)),
        ("E", "<f8"),
        ("numIALeft", "<f8"),
        ("trackId", "<u8"),
        ("parentId", "<u8"),
        ("rngSeed", "<u4"),
        ("rngCtr", "<u4"),
        ("volume", "<i4"),
        ("event", "<u4"),
    ],
    align=True,
)
assert TRACK_DTYPE.itemsize == 96


class Stats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_uint64),
        ("track_steps", ctypes.c_uint64 * 3),
        ("peak", ctypes.c_uint64 * 3),
        ("slots_touched", ctypes.c_uint64 * 3),
        ("error_iter", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


class Ledger(ctypes.Structure):
    _fields_ = [
        ("primaries", ctypes.c_uint64 * 3),
        ("created", ctypes.c_uint64 * 3),
        ("escaped", ctypes.c_uint64 * 3),
        ("cut", ctypes.c_uint64 * 3),
        ("annihilated", ctypes.c_uint64),
        ("absorbed", ctypes.c_uint64),
        ("n_brem", ctypes.c_uint64),
        ("n_pair", ctypes.c_uint64),
        ("n_compton", ctypes.c_uint64),
        ("n_annihilation", ctypes.c_uint64),
        ("survivors", ctypes.c_uint64 * 3),
        ("outputs", ctypes.c_uint64 * 3),
        ("off_mode", ctypes.c_uint64),
    ]


def build(force=False, src=SRC, out=LIB, extra_flags=()):
    """Compile liboracle.so with gcc (no FMA contraction, no fast-math).  src/out
    build another copy of the source (the mutation tests compile altered copies;
    extra_flags adds e.g. sanitizer options)."""
    if not force and os.path.exists(out):
        if os.path.getmtime(out) >= max(os.path.getmtime(src), os.path.getmtime(HDR)):
            return out
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, *extra_flags, "-I", HERE, "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = load(LIB)
    return _lib


def load(path):
    """A ctypes handle of an oracle library built from (a copy of) oracle.c."""
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    u64, u32, i32, dbl, flt = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_double, ctypes.c_float
    sig = {
        "or_create": (P, [i32, i32, u64, u32, P]),
        "or_destroy": (None, [P]),
        "or_set_scoring": (i32, [P, u32, u32, dbl]),
        "or_set_instrumented": (i32, [P, i32, u64]),
        "or_set_admission": (i32, [P, i32, dbl, P, u64]),
        "or_inject": (i32, [P, P, u64]),
        "or_stage": (i32, [P, P, u64]),
        "or_step": (i32, [P, P]),
        "or_run": (i32, [P, u64, P]),
        "or_counts": (i32, [P, P]),
        "or_tally": (i32, [P, i32, P, ctypes.c_size_t]),
        "or_stats_get": (i32, [P, P]),
        "or_ledger_get": (i32, [P, P]),
        "or_dump": (i32, [P, i32, P, P, u64, P]),
        "or_load": (i32, [P, i32, P, P, u64]),
        "or_ring_get": (i32, [P, i32, P, P, P]),
        "or_ring_set": (i32, [P, i32, P, u64, u64]),
        "or_set_iteration": (i32, [P, u64, i32]),
        "or_access_totals": (i32, [P, i32, i32, P, P]),
        "or_access_slotleaf": (i32, [P, i32, i32, P, u64]),
        "or_heat_words": (i32, [P, i32, i32, i32, u32, P, u64]),
        "or_philox4x32_10": (None, [P, P, P]),
        "or_u01": (dbl, [u32]),
        "or_u01f": (flt, [u32]),
        "or_log": (dbl, [dbl]),
        "or_exp": (dbl, [dbl]),
        "or_sincos": (None, [dbl, P, P]),
        "or_logf": (flt, [flt]),
        "or_expf": (flt, [flt]),
        "or_sincosf": (None, [flt, P, P]),
        "or_constants": (None, [P, P]),
        "or_leaf_addr": (u64, [i32, u32, i32, u64, u64, i32]),
        "or_buffer_bytes": (u64, [i32, u32, i32, u64]),
        "or_leaf_size": (u32, [i32, i32]),
        "or_child_id": (u64, [u32, u64, u32, u32]),
        "or_locate": (i32, [P, P]),
        "or_distance": (dbl, [P, P, i32, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


class Oracle:
    """One simulation context of the oracle."""

    def __init__(self, scheme=DENSE, precision=FP64, capacity=1 << 20, seeds=(1,), L=None):
        self.L = L if L is not None else lib()
        seeds = np.ascontiguousarray(seeds, dtype=np.uint32)
        self.h = self.L.or_create(scheme, precision, int(capacity), len(seeds), _ptr(seeds))
        if not self.h:
            raise OracleError(E_INVALID, "or_create")
        self.scheme, self.precision, self.capacity, self.n_events = scheme, precision, int(capacity), len(seeds)
        self.nx = self.ny = 0

    def close(self):
        if self.h:
            self.L.or_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != OK:
            raise OracleError(rc, what)

    def set_scoring(self, nx, ny, pitch):
        self._check(self.L.or_set_scoring(self.h, nx, ny, pitch), "set_scoring")
        self.nx, self.ny = nx, ny

    def set_instrumented(self, on, last_iter):
        self._check(self.L.or_set_instrumented(self.h, int(on), int(last_iter)), "set_instrumented")

    def set_admission(self, on, alpha, kappa, hold_iters=128):
        k = np.ascontiguousarray(kappa, dtype=np.float64)
        self._check(self.L.or_set_admission(self.h, int(on), float(alpha), _ptr(k), int(hold_iters)), "set_admission")

    def inject(self, prims):
        p = np.ascontiguousarray(prims)
        return self.L.or_inject(self.h, _ptr(p), len(p))

    def stage(self, prims):
        p = np.ascontiguousarray(prims)
        self._check(self.L.or_stage(self.h, _ptr(p), len(p)), "stage")

    def step(self):
        n = np.zeros(3, dtype=np.uint64)
        rc = self.L.or_step(self.h, _ptr(n))
        return rc, n

    def run(self, max_iter=1 << 62):
        it = ctypes.c_uint64(0)
        rc = self.L.or_run(self.h, int(max_iter), ctypes.byref(it))
        return rc, it.value

    def counts(self):
        n = np.zeros(3, dtype=np.uint64)
        self.L.or_counts(self.h, _ptr(n))
        return n

    def tally(self, kind):
        E = self.n_events
        size = {T_DEP_CONT: E * 100, T_DEP_CUT: E * 100, T_LAYER: E * 50, T_ESCAPED: E, T_ROUND: E,
                T_INFLIGHT: E, T_EIN: E, T_CELLS: 50 * self.nx * self.ny}[kind]
        out = np.zeros(size)
        self._check(self.L.or_tally(self.h, kind, _ptr(out), size), "tally")
        return out

    def stats(self):
        s = Stats()
        self.L.or_stats_get(self.h, ctypes.byref(s))
        return {"iterations": s.iterations, "track_steps": list(s.track_steps), "peak": list(s.peak),
                "slots_touched": list(s.slots_touched), "error_iter": s.error_iter, "status": s.status}

    def ledger(self):
        """The particle ledger (see oracle.h) plus the active counts ("inflight")."""
        g = Ledger()
        self._check(self.L.or_ledger_get(self.h, ctypes.byref(g)), "ledger")
        out = {name: (list(getattr(g, name)) if isinstance(getattr(g, name), ctypes.Array) else getattr(g, name))
               for name, _ in Ledger._fields_}
        out["inflight"] = [int(x) for x in self.counts()]
        return out

    def dump(self, ptype):
        n = int(self.counts()[ptype])
        out = np.zeros(max(n, 1), dtype=TRACK_DTYPE)
        slots = np.zeros(max(n, 1), dtype=np.uint32)
        m = ctypes.c_uint64(0)
        self._check(self.L.or_dump(self.h, ptype, _ptr(out), _ptr(slots), len(out), ctypes.byref(m)), "dump")
        return out[:n], slots[:n]

    def load(self, ptype, tracks, slots=None):
        t = np.ascontiguousarray(tracks, dtype=TRACK_DTYPE)
        s = np.ascontiguousarray(slots if slots is not None else np.arange(len(t)), dtype=np.uint32)
        self._check(self.L.or_load(self.h, ptype, _ptr(t), _ptr(s), len(t)), "load")

    def ring(self, ptype):
        r = np.zeros(self.capacity, dtype=np.uint32)
        h, c = ctypes.c_uint64(0), ctypes.c_uint64(0)
        self._check(self.L.or_ring_get(self.h, ptype, _ptr(r), ctypes.byref(h), ctypes.byref(c)), "ring_get")
        return r, h.value, c.value

    def set_ring(self, ptype, ring, head, count):
        r = np.ascontiguousarray(ring, dtype=np.uint32)
        self._check(self.L.or_ring_set(self.h, ptype, _ptr(r), int(head), int(count)), "ring_set")

    def set_iteration(self, it, dense_current_b=False):
        self._check(self.L.or_set_iteration(self.h, int(it), int(dense_current_b)), "set_iteration")

    def access_totals(self, ptype, buffer=0):
        r = np.zeros(14, dtype=np.uint64)
        w = np.zeros(14, dtype=np.uint64)
        self._check(self.L.or_access_totals(self.h, ptype, buffer, _ptr(r), _ptr(w)), "access_totals")
        return r, w

    def access_slotleaf(self, ptype, buffer=0):
        out = np.zeros(self.capacity * 14, dtype=np.uint32)
        self._check(self.L.or_access_slotleaf(self.h, ptype, buffer, _ptr(out), len(out)), "slotleaf")
        return out.reshape(self.capacity, 14)

    def heat_words(self, ptype, buffer, mapping, lanes=64):
        nbytes = buffer_bytes(mapping, lanes, self.precision, self.capacity)
        out = np.zeros(nbytes // 4, dtype=np.uint32)
        self._check(self.L.or_heat_words(self.h, ptype, buffer, mapping, lanes, _ptr(out), len(out)), "heat_words")
        return out


# ---- building blocks -------------------------------------------------------
def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return o


def u01(r):
    return lib().or_u01(int(r))


def u01f(r):
    return np.float32(lib().or_u01f(int(r)))


def log(x):
    return lib().or_log(float(x))


def exp(x):
    return lib().or_exp(float(x))


def sincos(x):
    s, c = ctypes.c_double(), ctypes.c_double()
    lib().or_sincos(float(x), ctypes.byref(s), ctypes.byref(c))
    return s.value, c.value


def logf(x):
    return np.float32(lib().or_logf(float(np.float32(x))))


def expf(x):
    return np.float32(lib().or_expf(float(np.float32(x))))


def sincosf(x):
    s, c = ctypes.c_float(), ctypes.c_float()
    lib().or_sincosf(float(np.float32(x)), ctypes.byref(s), ctypes.byref(c))
    return np.float32(s.value), np.float32(c.value)


def constants():
    d = np.zeros(8)
    f = np.zeros(8, dtype=np.float32)
    lib().or_constants(_ptr(d), _ptr(f))
    return d, f


def leaf_addr(mapping, lanes, precision, capacity, slot, leaf):
    return lib().or_leaf_addr(mapping, lanes, precision, capacity, slot, leaf)


def buffer_bytes(mapping, lanes, precision, capacity):
    return lib().or_buffer_bytes(mapping, lanes, precision, capacity)


def leaf_size(precision, leaf):
    return lib().or_leaf_size(precision, leaf)


def child_id(seed, parent_id, ctr, k):
    return lib().or_child_id(seed, parent_id, ctr, k)


def locate(pos):
    p = np.ascontiguousarray(pos, dtype=np.float64)
    v = ctypes.c_int32(0)
    rc = lib().or_locate(_ptr(p), ctypes.byref(v))
    return rc, v.value


def distance(pos, direction, volume):
    p = np.ascontiguousarray(pos, dtype=np.float64)
    d = np.ascontiguousarray(direction, dtype=np.float64)
    a = ctypes.c_int32(0)
    s = lib().or_distance(_ptr(p), _ptr(d), int(volume), ctypes.byref(a))
    return s, a.value


def run_workload(wl, scheme=DENSE, precision=FP64, capacity=1 << 20, max_iter=1 << 62, instrumented=None):
    """Inject all primaries of a workload at once and run to completion."""
    o = Oracle(scheme, precision, capacity, wl.seeds)
    if instrumented is not None:
        o.set_instrumented(True, instrumented)
    rc = o.inject(wl.primaries)
    if rc != OK:
        raise OracleError(rc, "inject")
    rc, it = o.run(max_iter)
    return o, rc, it
