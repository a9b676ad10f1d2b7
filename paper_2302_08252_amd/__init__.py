"""Python binding of libadept.so (include/adept.h): argument marshalling only.

Every entry point of the C ABI is exposed under the same name.  Device memory
and the stream come from PyTorch: ``Sim`` allocates the arena as a uint8 CUDA
tensor and binds it, together with torch's current stream, to the context.
All transport work runs in the HIP kernels of the library; if the library is
not built this module raises on import of the library (no fallback).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ADEPT_LIBRARY names another build of the same library (e.g. one made with
# build.py --define ... --out ...); the default is the in-tree build.
LIB_PATH = os.environ.get("ADEPT_LIBRARY") or os.path.join(HERE, "libadept.so")

OK, E_INVALID, E_CAPACITY, E_DEVICE, E_STATE, E_NOMEM, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
SPARSE_SINGLE, DENSE_DOUBLE = 0, 1
MAP_AOS, MAP_SOA, MAP_AOSOA = 0, 1, 2
FP64, MIXED = 0, 1
ELECTRON, POSITRON, GAMMA = 0, 1, 2
T_DEP_CONT, T_DEP_CUT, T_LAYER, T_ESCAPED, T_ROUND, T_INFLIGHT, T_CELLS, T_EIN = range(8)

PRIMARY_DTYPE = np.dtype(
    [("event", "<u4"), ("type", "<i4"), ("E", "<f8"), ("pos", "<f8", (3,)), ("dir", "<f8", (3,)),
     ("numIALeft", "<f8"), ("trackId", "<u8")], align=True)
TRACK_DTYPE = np.dtype(
    [("pos", "<f8", (3,)), ("dir", "<f8", (3,)), ("E", "<f8"), ("numIALeft", "<f8"), ("trackId", "<u8"),
     ("parentId", "<u8"), ("rngSeed", "<u4"), ("rngCtr", "<u4"), ("volume", "<i4"), ("event", "<u4")], align=True)
assert PRIMARY_DTYPE.itemsize == 80 and TRACK_DTYPE.itemsize == 96


class Layout(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("mapping", ctypes.c_int32), ("aosoa_lanes", ctypes.c_uint32)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_uint64), ("track_steps", ctypes.c_uint64 * 3), ("peak", ctypes.c_uint64 * 3),
                ("counts", ctypes.c_uint64 * 3), ("error_iter", ctypes.c_uint64),
                ("survivors", ctypes.c_uint64 * 3), ("outputs", ctypes.c_uint64 * 3),
                ("step_kernel_ms", ctypes.c_double), ("step_launches", ctypes.c_uint64), ("waves", ctypes.c_uint64),
                ("waves_divergent", ctypes.c_uint64), ("off_mode", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class Launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_uint32), ("grid", ctypes.c_uint32), ("graph_iters", ctypes.c_uint32),
                ("wave_tiles", ctypes.c_uint32)]


EXPORTS = [
    "adept_create", "adept_arena_bytes", "adept_bind", "adept_set_events", "adept_set_scoring",
    "adept_set_admission", "adept_set_instrumented", "adept_set_launch", "adept_get_launch", "adept_inject",
    "adept_inject_device", "adept_step", "adept_run", "adept_tally", "adept_access_counts", "adept_buffer_bytes",
    "adept_line_heat", "adept_layout_map", "adept_create_typed", "adept_type_buffer_bytes",
    "adept_autotune_type_layouts",
    "adept_stats_get", "adept_dump_tracks", "adept_dump_ring", "adept_reset", "adept_autotune",
    "adept_set_timing", "adept_autotune_layout", "adept_last_error", "adept_destroy", "adept_phase_clocks",
    "adept_dump_tracks_noalloc", "adept_set_divergence_count",
]

_lib = None


def lib():
    """Load libadept.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python paper_2302_08252_amd/build.py`")
    L = ctypes.CDLL(LIB_PATH)
    P, u64, u32, i32, dbl, sz = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    sig = {
        "adept_create": (i32, [Layout, i32, u64, P]),
        "adept_arena_bytes": (i32, [P, P]),
        "adept_bind": (i32, [P, P, sz, P]),
        "adept_set_events": (i32, [P, u32, P]),
        "adept_set_scoring": (i32, [P, u32, u32, dbl]),
        "adept_set_admission": (i32, [P, i32, dbl, P, u64]),
        "adept_set_instrumented": (i32, [P, i32, u64]),
        "adept_set_launch": (i32, [P, P]),
        "adept_get_launch": (i32, [P, P]),
        "adept_inject": (i32, [P, P, u64]),
        "adept_inject_device": (i32, [P, P, u64]),
        "adept_step": (i32, [P, P]),
        "adept_run": (i32, [P, u64, P]),
        "adept_tally": (i32, [P, i32, P, sz]),
        "adept_access_counts": (i32, [P, i32, u32, P, P, P, sz]),
        "adept_buffer_bytes": (i32, [P, P]),
        "adept_line_heat": (i32, [P, i32, u32, u32, P, sz]),
        "adept_layout_map": (i32, [Layout, i32, u64, u64, u64, P, P]),
        "adept_create_typed": (i32, [P, i32, u64, P]),
        "adept_type_buffer_bytes": (i32, [P, i32, P]),
        "adept_autotune_type_layouts": (i32, [i32, u64, P, u32, u32, P, P, u64, P, P, P]),
        "adept_stats_get": (i32, [P, P]),
        "adept_dump_tracks": (i32, [P, i32, P, P, u64, P]),
        "adept_dump_tracks_noalloc": (i32, [P, i32, P, P, u64, P]),
        "adept_dump_ring": (i32, [P, i32, P, u64, P, P]),
        "adept_reset": (i32, [P]),
        "adept_autotune": (i32, [P, P, u64, P]),
        "adept_set_timing": (i32, [P, i32]),
        "adept_set_divergence_count": (i32, [P, i32]),
        "adept_phase_clocks": (i32, [P, P]),
        "adept_autotune_layout": (i32, [i32, u64, P, u32, u32, P, P, u64, P, P, P]),
        "adept_last_error": (ctypes.c_char_p, [P]),
        "adept_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    _lib = L
    return L


class AdeptError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"adept status {code}: {msg}")
        self.code = code


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(ctx, rc, what):
    if rc != OK:
        msg = lib().adept_last_error(ctx).decode() if ctx else what
        raise AdeptError(rc, f"{what}: {msg}")


# ---- entry points, same names as the C ABI ---------------------------------
def adept_create(scheme, mapping, precision, capacity, aosoa_lanes=64):
    h = ctypes.c_void_p()
    rc = lib().adept_create(Layout(scheme, mapping, aosoa_lanes), precision, int(capacity), ctypes.byref(h))
    _check(None, rc, "adept_create")
    return h


def adept_create_typed(scheme, layouts, precision, capacity):
    """layouts: one (mapping, aosoa_lanes) per particle type (electron, positron, photon)."""
    arr = (Layout * 3)(*[Layout(scheme, m, n) for m, n in layouts])
    h = ctypes.c_void_p()
    rc = lib().adept_create_typed(ctypes.cast(arr, ctypes.c_void_p), precision, int(capacity), ctypes.byref(h))
    _check(None, rc, "adept_create_typed")
    return h


def adept_arena_bytes(ctx):
    n = ctypes.c_size_t()
    _check(ctx, lib().adept_arena_bytes(ctx, ctypes.byref(n)), "adept_arena_bytes")
    return n.value


def adept_bind(ctx, dev_ptr, nbytes, stream_handle):
    _check(ctx, lib().adept_bind(ctx, ctypes.c_void_p(dev_ptr), nbytes, ctypes.c_void_p(stream_handle)), "adept_bind")


def adept_set_events(ctx, seeds):
    s = np.ascontiguousarray(seeds, dtype=np.uint32)
    _check(ctx, lib().adept_set_events(ctx, len(s), _ptr(s)), "adept_set_events")


def adept_set_scoring(ctx, nx, ny, pitch):
    _check(ctx, lib().adept_set_scoring(ctx, nx, ny, pitch), "adept_set_scoring")


def adept_set_admission(ctx, on, alpha, kappa, hold_iters=128):
    k = np.ascontiguousarray(kappa, dtype=np.float64)
    _check(ctx, lib().adept_set_admission(ctx, int(on), float(alpha), _ptr(k), int(hold_iters)),
           "adept_set_admission")


def adept_set_instrumented(ctx, on, last_iter):
    _check(ctx, lib().adept_set_instrumented(ctx, int(on), int(last_iter)), "adept_set_instrumented")


def adept_set_launch(ctx, block=1024, grid=0, graph_iters=32, wave_tiles=0):
    l = Launch(block, grid, graph_iters, int(wave_tiles))
    _check(ctx, lib().adept_set_launch(ctx, ctypes.byref(l)), "adept_set_launch")


def adept_get_launch(ctx):
    l = Launch()
    _check(ctx, lib().adept_get_launch(ctx, ctypes.byref(l)), "adept_get_launch")
    return {"block": l.block, "grid": l.grid, "graph_iters": l.graph_iters, "wave_tiles": l.wave_tiles}


def adept_inject(ctx, primaries):
    p = np.ascontiguousarray(primaries).view(PRIMARY_DTYPE) if len(primaries) else np.zeros(0, PRIMARY_DTYPE)
    _check(ctx, lib().adept_inject(ctx, _ptr(p), len(p)), "adept_inject")


def adept_inject_device(ctx, dev_ptr, n):
    _check(ctx, lib().adept_inject_device(ctx, ctypes.c_void_p(dev_ptr), int(n)), "adept_inject_device")


def adept_step(ctx):
    n = np.zeros(3, dtype=np.uint64)
    _check(ctx, lib().adept_step(ctx, _ptr(n)), "adept_step")
    return n


def adept_run(ctx, max_iter=(1 << 63)):
    it = ctypes.c_uint64()
    _check(ctx, lib().adept_run(ctx, int(max_iter), ctypes.byref(it)), "adept_run")
    return it.value


def adept_tally(ctx, kind, size):
    out = np.zeros(size)
    _check(ctx, lib().adept_tally(ctx, kind, _ptr(out), size), "adept_tally")
    return out


def adept_buffer_bytes(ctx):
    n = ctypes.c_size_t()
    _check(ctx, lib().adept_buffer_bytes(ctx, ctypes.byref(n)), "adept_buffer_bytes")
    return n.value


def adept_type_buffer_bytes(ctx, ptype):
    n = ctypes.c_size_t()
    _check(ctx, lib().adept_type_buffer_bytes(ctx, ptype, ctypes.byref(n)), "adept_type_buffer_bytes")
    return n.value


def adept_access_counts(ctx, ptype, buffer=0, heat=False):
    r = np.zeros(14, dtype=np.uint64)
    w = np.zeros(14, dtype=np.uint64)
    hw = np.zeros(adept_type_buffer_bytes(ctx, ptype) // 4 if heat else 0, dtype=np.uint32)
    rc = lib().adept_access_counts(ctx, ptype, buffer, _ptr(r), _ptr(w), _ptr(hw) if heat else None, len(hw))
    _check(ctx, rc, "adept_access_counts")
    return (r, w, hw) if heat else (r, w)


def adept_line_heat(ctx, ptype, buffer=0, line_bytes=128):
    out = np.zeros(-(-adept_type_buffer_bytes(ctx, ptype) // line_bytes), dtype=np.uint64)
    _check(ctx, lib().adept_line_heat(ctx, ptype, buffer, line_bytes, _ptr(out), len(out)), "adept_line_heat")
    return out


def adept_layout_map(mapping, precision, capacity, first_byte=0, n=None, aosoa_lanes=64):
    """Field id (0-13, -1 padding) of each byte of a track buffer; n defaults to the rest of the buffer."""
    lay = Layout(0, mapping, aosoa_lanes if mapping == MAP_AOSOA else 1)
    total = ctypes.c_uint64()
    _check(None, lib().adept_layout_map(lay, precision, capacity, 0, 0, None, ctypes.byref(total)), "adept_layout_map")
    if n is None:
        n = max(total.value - first_byte, 0)
    out = np.zeros(n, dtype=np.int8)
    _check(None, lib().adept_layout_map(lay, precision, capacity, first_byte, n, _ptr(out), None), "adept_layout_map")
    return out


def layout_picture(leaf_map, bytes_per_row=128, rows=8):
    """Text picture of a byte map: one character per 4-byte word (field id in base 36, '.' padding)."""
    glyph = "0123456789abcd"
    words = leaf_map[: len(leaf_map) // 4 * 4].reshape(-1, 4)[:, 0]
    per_row = bytes_per_row // 4
    lines = []
    for r in range(min(rows, -(-len(words) // per_row))):
        w = words[r * per_row:(r + 1) * per_row]
        lines.append("".join("." if x < 0 else glyph[x] for x in w))
    return "\n".join(lines)


def adept_stats_get(ctx):
    s = Stats()
    _check(ctx, lib().adept_stats_get(ctx, ctypes.byref(s)), "adept_stats_get")
    return {"iterations": s.iterations, "track_steps": list(s.track_steps), "peak": list(s.peak),
            "counts": list(s.counts), "error_iter": s.error_iter, "survivors": list(s.survivors),
            "outputs": list(s.outputs), "step_kernel_ms": s.step_kernel_ms, "step_launches": s.step_launches,
            "waves": s.waves,
            "waves_divergent": s.waves_divergent, "off_mode": s.off_mode, "status": s.status}


def adept_dump_tracks(ctx, ptype):
    n = adept_stats_get(ctx)["counts"][ptype]
    out = np.zeros(max(n, 1), dtype=TRACK_DTYPE)
    slots = np.zeros(max(n, 1), dtype=np.uint32)
    m = ctypes.c_uint64()
    _check(ctx, lib().adept_dump_tracks(ctx, ptype, _ptr(out), _ptr(slots), len(out), ctypes.byref(m)),
           "adept_dump_tracks")
    return out[:m.value], slots[:m.value]


def adept_dump_tracks_noalloc(ctx, ptype, with_slots=True):
    """adept_dump_tracks through the library's fixed device staging array."""
    n = adept_stats_get(ctx)["counts"][ptype]
    out = np.zeros(max(n, 1), dtype=TRACK_DTYPE)
    slots = np.zeros(max(n, 1), dtype=np.uint32) if with_slots else None
    m = ctypes.c_uint64()
    _check(ctx, lib().adept_dump_tracks_noalloc(ctx, ptype, _ptr(out), _ptr(slots) if with_slots else None,
                                                len(out), ctypes.byref(m)), "adept_dump_tracks_noalloc")
    return out[:m.value], (slots[:m.value] if with_slots else None)


def adept_dump_ring(ctx, ptype, capacity):
    ring = np.zeros(capacity, dtype=np.uint32)
    h, c = ctypes.c_uint64(), ctypes.c_uint64()
    _check(ctx, lib().adept_dump_ring(ctx, ptype, _ptr(ring), capacity, ctypes.byref(h), ctypes.byref(c)),
           "adept_dump_ring")
    return ring, h.value, c.value


def adept_reset(ctx):
    _check(ctx, lib().adept_reset(ctx), "adept_reset")


def adept_autotune(ctx, primaries):
    p = np.ascontiguousarray(primaries).view(PRIMARY_DTYPE)
    l = Launch()
    _check(ctx, lib().adept_autotune(ctx, _ptr(p), len(p), ctypes.byref(l)), "adept_autotune")
    return {"block": l.block, "grid": l.grid, "graph_iters": l.graph_iters, "wave_tiles": l.wave_tiles}


def adept_phase_clocks(ctx):
    """Wave-cycles per step-kernel phase (zeros unless built with ADEPT_PHASE_CLOCKS)."""
    out = np.zeros(8, dtype=np.uint64)
    _check(ctx, lib().adept_phase_clocks(ctx, out.ctypes.data_as(ctypes.c_void_p)), "adept_phase_clocks")
    return out


def adept_set_divergence_count(ctx, on):
    _check(ctx, lib().adept_set_divergence_count(ctx, int(on)), "adept_set_divergence_count")


def adept_set_timing(ctx, on):
    _check(ctx, lib().adept_set_timing(ctx, int(on)), "adept_set_timing")


def adept_autotune_layout(precision, capacity, candidates, seeds, primaries):
    """candidates: (scheme, mapping, aosoa_lanes) tuples; returns (layout, launch, ms)."""
    arr = (Layout * len(candidates))(*[Layout(s, m, n) for s, m, n in candidates])
    sd = np.ascontiguousarray(seeds, dtype=np.uint32)
    p = np.ascontiguousarray(primaries).view(PRIMARY_DTYPE)
    best, l, ms = Layout(), Launch(), ctypes.c_double()
    rc = lib().adept_autotune_layout(precision, int(capacity), ctypes.cast(arr, ctypes.c_void_p), len(candidates),
                                     len(sd), _ptr(sd), _ptr(p), len(p), ctypes.byref(best), ctypes.byref(l),
                                     ctypes.byref(ms))
    _check(None, rc, "adept_autotune_layout")
    return ((best.scheme, best.mapping, best.aosoa_lanes),
            {"block": l.block, "grid": l.grid, "graph_iters": l.graph_iters, "wave_tiles": l.wave_tiles}, ms.value)


def adept_autotune_type_layouts(precision, capacity, candidates, seeds, primaries):
    """candidates: (scheme, mapping, aosoa_lanes) tuples of one scheme; returns
    ([(mapping, aosoa_lanes)] * 3 per type, launch, ms)."""
    arr = (Layout * len(candidates))(*[Layout(s, m, n) for s, m, n in candidates])
    sd = np.ascontiguousarray(seeds, dtype=np.uint32)
    p = np.ascontiguousarray(primaries).view(PRIMARY_DTYPE)
    best, l, ms = (Layout * 3)(), Launch(), ctypes.c_double()
    rc = lib().adept_autotune_type_layouts(precision, int(capacity), ctypes.cast(arr, ctypes.c_void_p),
                                           len(candidates), len(sd), _ptr(sd), _ptr(p), len(p),
                                           ctypes.cast(best, ctypes.c_void_p), ctypes.byref(l), ctypes.byref(ms))
    _check(None, rc, "adept_autotune_type_layouts")
    return ([(b.mapping, b.aosoa_lanes) for b in best],
            {"block": l.block, "grid": l.grid, "graph_iters": l.graph_iters, "wave_tiles": l.wave_tiles}, ms.value)


def adept_last_error(ctx):
    return lib().adept_last_error(ctx).decode()


def adept_destroy(ctx):
    lib().adept_destroy(ctx)


# ---- convenience: a context whose arena and stream are PyTorch's -------------
class Sim:
    """One context bound to a torch-owned device arena and torch's current stream."""

    def __init__(self, scheme=DENSE_DOUBLE, mapping=MAP_SOA, precision=MIXED, capacity=1 << 20, aosoa_lanes=64,
                 seeds=(1,), scoring=None, admission=None, instrumented=None, launch=None, device="cuda",
                 type_layouts=None):
        """type_layouts: one (mapping, aosoa_lanes) per particle type (adept_create_typed);
        mapping and aosoa_lanes are then ignored."""
        import torch

        self.scheme, self.mapping, self.precision, self.capacity = scheme, mapping, precision, int(capacity)
        self.n_events = len(seeds)
        self.nx = self.ny = 0
        if type_layouts is not None:
            self.ctx = adept_create_typed(scheme, type_layouts, precision, capacity)
        else:
            self.ctx = adept_create(scheme, mapping, precision, capacity, aosoa_lanes)
        try:
            adept_set_events(self.ctx, seeds)
            if scoring:
                adept_set_scoring(self.ctx, *scoring)
                self.nx, self.ny = scoring[0], scoring[1]
            if admission:
                adept_set_admission(self.ctx, True, *admission)
            if instrumented is not None:
                adept_set_instrumented(self.ctx, True, instrumented)
            if launch:
                adept_set_launch(self.ctx, **launch)
            nbytes = adept_arena_bytes(self.ctx)
            self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            base = self.arena.data_ptr()
            aligned = (base + 255) & ~255
            self.stream = torch.cuda.current_stream(device)
            adept_bind(self.ctx, aligned, nbytes, self.stream.cuda_stream)
        except Exception:
            adept_destroy(self.ctx)
            self.ctx = None
            raise

    def close(self):
        if getattr(self, "ctx", None):
            adept_destroy(self.ctx)
            self.ctx = None
        self.arena = None  # the device arena goes back to torch's allocator

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def inject(self, primaries):
        adept_inject(self.ctx, primaries)

    def step(self):
        return adept_step(self.ctx)

    def run(self, max_iter=(1 << 63)):
        return adept_run(self.ctx, max_iter)

    def tally(self, kind):
        E = self.n_events
        size = {T_DEP_CONT: E * 100, T_DEP_CUT: E * 100, T_LAYER: E * 50, T_ESCAPED: E, T_ROUND: E,
                T_INFLIGHT: E, T_EIN: E, T_CELLS: 50 * self.nx * self.ny}[kind]
        return adept_tally(self.ctx, kind, size)

    def stats(self):
        return adept_stats_get(self.ctx)

    def dump(self, ptype):
        return adept_dump_tracks(self.ctx, ptype)

    def ring(self, ptype):
        return adept_dump_ring(self.ctx, ptype, self.capacity)

    def access_counts(self, ptype, buffer=0, heat=False):
        return adept_access_counts(self.ctx, ptype, buffer, heat)

    def line_heat(self, ptype, buffer=0, line_bytes=128):
        return adept_line_heat(self.ctx, ptype, buffer, line_bytes)

    def reset(self):
        adept_reset(self.ctx)

    def counts(self):
        return np.array(self.stats()["counts"], dtype=np.uint64)
