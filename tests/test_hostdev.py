"""The HIP path's device model, compiled for the host, against the oracle.

``tests/hostdev/hostdev.cpp`` builds the library's own ``model.hpp`` and
``layout.hpp`` (the exact sources the gfx950 kernels use) for x86 with
-ffp-contract=off.  This is two independent implementations compared bit for
bit on the CPU: elementary functions, Philox, child ids, record layouts and one
transport step of random single tracks of every type, in both precision
policies.  It catches model mismatches before any GPU run; the GPU parity tests
then check the gfx950 arithmetic itself.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hostdev", "hostdev.cpp")


def _build_hostdev(tmp_path_factory, defines=()):
    out = str(tmp_path_factory.mktemp("hostdev") / "libhostdev.so")
    try:
        subprocess.check_call(["hipcc", "-x", "hip", "--offload-host-only", "-O2", "-std=c++17", "-ffp-contract=off",
                               *[f"-D{d}" for d in defines], "-fPIC", "-shared", "-o", out, SRC],
                              cwd=str(tmp_path_factory.getbasetemp()),
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    except (OSError, subprocess.CalledProcessError):
        pytest.skip("hipcc not available")
    return _bind(ctypes.CDLL(out))


@pytest.fixture(scope="module")
def hd(tmp_path_factory):
    return _build_hostdev(tmp_path_factory)


@pytest.fixture(scope="module")
def hd_per_path(tmp_path_factory):
    """The model built with ADEPT_RNG_PER_PATH=1: shared random-number blocks drawn on each path."""
    return _build_hostdev(tmp_path_factory, ["ADEPT_RNG_PER_PATH=1"])


def _bind(L):
    P = ctypes.c_void_p
    L.hd_log.restype = L.hd_exp.restype = ctypes.c_double
    L.hd_log.argtypes = L.hd_exp.argtypes = [ctypes.c_double]
    L.hd_logf.restype = L.hd_expf.restype = ctypes.c_float
    L.hd_logf.argtypes = L.hd_expf.argtypes = [ctypes.c_float]
    L.hd_sincos.argtypes = [ctypes.c_double, P, P]
    L.hd_sincosf.argtypes = [ctypes.c_float, P, P]
    L.hd_philox.argtypes = [P, P, P]
    L.hd_child_id.restype = ctypes.c_uint64
    L.hd_child_id.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
    L.hd_step.restype = ctypes.c_int
    L.hd_step.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P]
    L.hd_leaf_addr.restype = ctypes.c_uint64
    L.hd_leaf_addr.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                               ctypes.c_int]
    L.hd_distance.restype = ctypes.c_double
    L.hd_distance.argtypes = [P, P, ctypes.c_int, P]
    L.hd_buffer_bytes.restype = ctypes.c_uint64
    L.hd_buffer_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64]
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def test_math_bitwise(hd, oracle_mod):
    rng = np.random.default_rng(7)
    xs = np.concatenate([2.0 ** rng.uniform(-34, 17, 3000), [1.0, 0.5, 2.0, math.sqrt(0.5)]])
    for x in xs:
        assert hd.hd_log(x) == oracle_mod.log(x)
    for x in rng.uniform(-30, 12, 3000):
        assert hd.hd_exp(x) == oracle_mod.exp(x)
    s, c = ctypes.c_double(), ctypes.c_double()
    for x in np.concatenate([rng.uniform(0, 2 * math.pi, 3000), [0.0, math.pi]]):
        hd.hd_sincos(x, ctypes.byref(s), ctypes.byref(c))
        assert (s.value, c.value) == oracle_mod.sincos(x)
    sf, cf = ctypes.c_float(), ctypes.c_float()
    for x in rng.uniform(0, 2 * math.pi, 2000).astype(np.float32):
        hd.hd_sincosf(float(x), ctypes.byref(sf), ctypes.byref(cf))
        os_, oc = oracle_mod.sincosf(x)
        assert np.float32(sf.value) == os_ and np.float32(cf.value) == oc
    for x in (2.0 ** rng.uniform(-24, 17, 2000)).astype(np.float32):
        assert np.float32(hd.hd_logf(float(x))) == oracle_mod.logf(x)
    for x in rng.uniform(0, 11.6, 2000).astype(np.float32):
        assert np.float32(hd.hd_expf(float(x))) == oracle_mod.expf(x)


def test_philox_and_ids_bitwise(hd, oracle_mod):
    rng = np.random.default_rng(8)
    for _ in range(500):
        c = rng.integers(0, 2**32, 4, dtype=np.uint64).astype(np.uint32)
        k = rng.integers(0, 2**32, 2, dtype=np.uint64).astype(np.uint32)
        o = np.zeros(4, dtype=np.uint32)
        hd.hd_philox(_p(c), _p(k), _p(o))
        assert list(o) == list(oracle_mod.philox(c, k))
        seed, pid, n, kk = int(k[0]), int(rng.integers(0, 2**63)), int(c[0] % 5000), int(c[1] % 4)
        assert hd.hd_child_id(seed, pid, n, kk) == oracle_mod.child_id(seed, pid, n, kk)


@pytest.mark.parametrize("capacity", [4096, 1000, 4097])
@pytest.mark.parametrize("mixed", [0, 1])
@pytest.mark.parametrize("mapping,lanes", [(0, 1), (1, 1), (2, 2), (2, 16), (2, 64), (2, 256)])
def test_layouts_match_oracle_byte_map(hd, oracle_mod, mixed, mapping, lanes, capacity):
    """Capacities that are not multiples of 64 pad the SoA field arrays (256-byte starts)."""
    C = max(lanes, capacity // lanes * lanes)
    assert hd.hd_buffer_bytes(mapping, mixed, lanes, C) == oracle_mod.buffer_bytes(mapping, lanes, mixed, C)
    rng = np.random.default_rng(9)
    for slot in list(rng.integers(0, C, 300)) + [0, C - 1]:
        for leaf in range(14):
            assert hd.hd_leaf_addr(mapping, mixed, lanes, C, int(slot), leaf) == \
                oracle_mod.leaf_addr(mapping, lanes, mixed, C, int(slot), leaf)


def random_tracks(rng, n, ptype, mixed):
    t = np.zeros(n, dtype=oracle_TRACK())
    E = np.exp(rng.uniform(math.log(0.3), math.log(2e4), n))
    if ptype == 2:
        E[: n // 4] = rng.uniform(0.05, 3.0, n // 4)  # around the pair threshold and the photon cut
    z = rng.uniform(0, 399.999, n)
    x = rng.uniform(-199.9, 199.9, n)
    y = rng.uniform(-199.9, 199.9, n)
    x[: n // 10] = rng.choice([-200.0, 200.0, 199.999], n // 10)
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    d[n // 10: n // 5] = [0.0, 0.0, 1.0]
    d[n // 5: n // 5 + n // 20] = [0.0, 0.0, -1.0]
    nl = np.where(rng.random(n) < 0.5, -1.0, rng.uniform(0, 4, n))
    vol = np.array([2 * int(zz // 8.0) + (1 if zz >= 8.0 * int(zz // 8.0) + 2.3 else 0) for zz in z])
    # some tracks sit exactly on a plane of their volume
    on = rng.random(n) < 0.1
    for i in np.nonzero(on)[0]:
        v = vol[i]
        l = v >> 1
        z[i] = (8.0 * l + 2.3) if (v & 1) else 8.0 * l
    t["pos"][:, 0], t["pos"][:, 1], t["pos"][:, 2] = x, y, z
    t["dir"] = d
    t["E"] = E
    t["numIALeft"] = nl
    t["trackId"] = rng.integers(0, 2**63, n, dtype=np.uint64)
    t["parentId"] = rng.integers(0, 2**63, n, dtype=np.uint64)
    t["rngSeed"] = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    t["rngCtr"] = rng.integers(0, 3000, n)
    t["volume"] = vol
    t["event"] = 0
    if mixed:
        for f in ("dir", "E", "numIALeft"):
            t[f] = t[f].astype(np.float32).astype(np.float64)
    return t


def oracle_TRACK():
    import oracle

    return oracle.TRACK_DTYPE


@pytest.mark.parametrize("mixed", [0, 1])
@pytest.mark.parametrize("ptype", [0, 1, 2])
def test_single_step_bitwise(hd, oracle_mod, ptype, mixed):
    rng = np.random.default_rng(100 + 10 * ptype + mixed)
    tracks = random_tracks(rng, 1500, ptype, mixed)
    out = np.zeros(4, dtype=oracle_mod.TRACK_DTYPE)
    out_type = np.zeros(4, dtype=np.int32)
    dep = np.zeros(5)
    surv = ctypes.c_int()
    n_surv = n_sec = 0
    for t in tracks:
        tin = np.array([t], dtype=oracle_mod.TRACK_DTYPE)
        k = hd.hd_step(mixed, ptype, _p(tin), ctypes.byref(surv), _p(out), _p(out_type), _p(dep))
        o = oracle_mod.Oracle(oracle_mod.DENSE, mixed, 64, [1])
        o.load(ptype, tin)
        rc, n = o.step()
        assert rc == 0
        for d in range(3):
            got = out[:k][out_type[:k] == d]
            want, _ = o.dump(d)
            assert got.tobytes() == want.tobytes(), (t, d, got, want)
        v = int(t["volume"])
        cont = o.tally(oracle_mod.T_DEP_CONT)
        cut = o.tally(oracle_mod.T_DEP_CUT)
        assert cont[v] == dep[0] and np.count_nonzero(np.delete(cont, v)) == 0
        assert cut[v] == dep[1] and np.count_nonzero(np.delete(cut, v)) == 0
        assert o.tally(oracle_mod.T_ESCAPED)[0] == dep[2]
        assert o.tally(oracle_mod.T_ROUND)[0] == dep[3]
        n_surv += surv.value
        n_sec += k - surv.value
    # the sample exercised both outcomes and created secondaries
    assert 0 < n_surv < len(tracks) and n_sec > 50


@pytest.mark.parametrize("mixed", [0, 1])
@pytest.mark.parametrize("ptype", [0, 1, 2])
def test_random_blocks_per_path_give_the_same_step(hd, hd_per_path, oracle_mod, ptype, mixed):
    """Drawing the shared Philox blocks once per step (normal build) or on each path that uses
    them (the comparison build) yields the same step, bit for bit: the hoisting is a code
    transformation, not a change of the random numbers."""
    rng = np.random.default_rng(300 + 10 * ptype + mixed)
    tracks = random_tracks(rng, 1500, ptype, mixed)
    res = []
    for L in (hd, hd_per_path):
        outs = []
        for t in tracks:
            tin = np.array([t], dtype=oracle_mod.TRACK_DTYPE)
            out = np.zeros(4, dtype=oracle_mod.TRACK_DTYPE)
            out_type = np.zeros(4, dtype=np.int32)
            dep = np.zeros(5)
            surv = ctypes.c_int()
            k = L.hd_step(mixed, ptype, _p(tin), ctypes.byref(surv), _p(out), _p(out_type), _p(dep))
            outs.append((k, surv.value, out[:k].tobytes(), out_type[:k].tobytes(), dep.tobytes()))
        res.append(outs)
    assert res[0] == res[1]
    assert sum(o[0] - o[1] for o in res[0]) > 50  # creations were exercised


def test_distance_with_skipped_divisions_is_exact(hd, oracle_mod):
    """The device distance only divides out the transverse planes when they might
    win; on random and adversarial inputs (near-ties between the planes, points on
    the walls, axis-parallel and grazing directions) it must equal the oracle's
    plain evaluation of all three, distance and axis."""
    rng = np.random.default_rng(21)
    ax = ctypes.c_int()
    cases = []
    for _ in range(20000):
        v = int(rng.integers(0, 100))
        l = v >> 1
        zlo = 8.0 * l + 2.3 if v & 1 else 8.0 * l
        zhi = 8.0 * (l + 1) if v & 1 else 8.0 * l + 2.3
        z = rng.uniform(zlo, zhi)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        # choose x so that the x plane is hit at nearly the same distance as the z plane
        tz = ((zhi - z) / d[2]) if d[2] > 0 else ((zlo - z) / d[2])
        if d[0] != 0 and abs(tz * d[0]) < 399:
            x = (200.0 if d[0] > 0 else -200.0) - tz * d[0] * (1 + rng.choice([0, 1e-16, -1e-16, 1e-12, -1e-12]))
            x = float(np.clip(x, -200.0, 200.0))
        else:
            x = rng.uniform(-200, 200)
        y = rng.choice([rng.uniform(-200, 200), 200.0, -200.0, x])
        if rng.random() < 0.1:
            d = np.array([rng.choice([0.0, 1.0, -1.0]), 0.0, rng.choice([0.0, 1.0])])
            if not d.any():
                d[2] = 1.0
        cases.append((np.array([x, y, z]), d, v))
    for p, d, v in cases:
        p = np.ascontiguousarray(p)
        d = np.ascontiguousarray(d, dtype=np.float64)
        got = hd.hd_distance(_p(p), _p(d), v, ctypes.byref(ax))
        want, wax = oracle_mod.distance(p, d, v)
        assert (got, ax.value) == (want, wax) or (np.isnan(got) and np.isnan(want)), (p, d, v, got, want)
