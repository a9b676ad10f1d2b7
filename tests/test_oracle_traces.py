"""Hand-derived single-track traces and hand-counted field accesses pin the oracle.

The expected values live in ``tests/golden/hand_traces.txt`` with their
derivation from the toy shower model (slab calorimeter, Compton/pair/brem
processes, cuts) and from the access contract of the track buffers (paper
Sec. 5, per-field access counts).
"""
import math
import os

import numpy as np
import pytest

import workloads

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_traces.txt")


def golden():
    out = {}
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, *v = line.split()
        out[k] = [float(x) for x in v] if len(v) > 1 else float(v[0])
    return out


G = golden()


def one(ptype, E, nl=100.0, pos=(0.0, 0.0, 0.0), direction=(0.0, 0.0, 1.0)):
    return workloads.primaries(1, ptype, E, pos=pos, direction=direction, num_ia_left=nl)


@pytest.mark.parametrize("scheme", [0, 1])
def test_gamma_straight_through(oracle_mod, scheme):
    o = oracle_mod.Oracle(scheme, oracle_mod.FP64, 64, [1])
    o.set_instrumented(True, 1000)
    assert o.inject(one(workloads.GAMMA, 0.5)) == 0
    for it in range(1, 101):
        rc, n = o.step()
        assert rc == 0
        if it == 99:
            t, _ = o.dump(workloads.GAMMA)
            assert len(t) == 1 and t[0]["volume"] == 99 and t[0]["rngCtr"] == 99
            assert abs(t[0]["numIALeft"] - G["gamma_straight.numIALeft_after_99"]) < 1e-12
            assert t[0]["pos"][2] == 8.0 * 49 + 2.3
        if it < 100:
            assert list(n) == [0, 0, 1]
    assert list(n) == [0, 0, 0]
    st = o.stats()
    assert st["iterations"] == G["gamma_straight.iterations"]
    assert sum(st["track_steps"]) == 100
    assert o.tally(oracle_mod.T_ESCAPED)[0] == G["gamma_straight.escaped"]
    assert np.all(o.tally(oracle_mod.T_DEP_CONT) == 0) and np.all(o.tally(oracle_mod.T_DEP_CUT) == 0)
    key = "dense" if scheme == 1 else "sparse"
    r = np.zeros(14, dtype=np.uint64)
    w = np.zeros(14, dtype=np.uint64)
    for b in (0, 1):
        rb, wb = o.access_totals(workloads.GAMMA, b)
        r += rb
        w += wb
    assert list(r) == G[f"gamma_straight.{key}.reads"]
    assert list(w) == G[f"gamma_straight.{key}.writes"]
    if scheme == 1:
        # A holds the injection and even iterations' survivors, B the odd ones
        ra, wa = o.access_totals(workloads.GAMMA, 0)
        rb, wb = o.access_totals(workloads.GAMMA, 1)
        assert ra[0] == 50 and rb[0] == 50 and ra[9] == 50 and rb[9] == 49
        assert wa[0] == 50 and wb[0] == 50
    for t in range(2):
        rr, ww = o.access_totals(t, 0)
        assert rr.sum() == 0 and ww.sum() == 0


def test_electron_first_step(oracle_mod):
    o = oracle_mod.Oracle(oracle_mod.DENSE, oracle_mod.FP64, 64, [1])
    assert o.inject(one(workloads.ELECTRON, 1000.0)) == 0
    rc, n = o.step()
    assert rc == 0 and list(n) == [1, 0, 0]
    t, _ = o.dump(workloads.ELECTRON)
    t = t[0]
    assert t["pos"][2] == G["electron_first_step.z"] and t["pos"][0] == 0.0 and t["pos"][1] == 0.0
    assert t["volume"] == G["electron_first_step.volume"] and t["rngCtr"] == 1
    assert t["numIALeft"] == G["electron_first_step.numIALeft"]
    assert t["E"] == 1000.0 - 1.27 * 2.3
    dep = o.tally(oracle_mod.T_DEP_CONT)
    assert dep[0] == 1000.0 - (1000.0 - 1.27 * 2.3) and abs(dep[0] - 2.921) < 1e-12
    assert np.count_nonzero(dep) == 1
    a = oracle_mod.philox([0, 0, 0, 0], [1, 0])
    u1, u2 = (int(a[1]) + 0.5) * 2.0**-32, (int(a[2]) + 0.5) * 2.0**-32
    th0 = (13.6 / 1000.0) * math.sqrt(2.3 / 5.6)
    assert abs(th0 - G["electron_first_step.theta0"]) < 1e-17
    th = min(th0 * math.sqrt(-2.0 * math.log(u1)), math.pi)
    ph = 2.0 * math.pi * u2
    want = [math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)]
    assert np.allclose(t["dir"], want, rtol=0, atol=4e-16)


def test_positron_range_out(oracle_mod):
    o = oracle_mod.Oracle(oracle_mod.DENSE, oracle_mod.FP64, 64, [1])
    assert o.inject(one(workloads.POSITRON, 2.0)) == 0
    assert abs(o.tally(oracle_mod.T_EIN)[0] - G["positron_range_out.input_energy"]) < 1e-15
    rc, n = o.step()
    assert rc == 0 and list(n) == [0, 0, 2]
    assert o.tally(oracle_mod.T_DEP_CONT)[0] == G["positron_range_out.deposit_v0"]
    assert o.tally(oracle_mod.T_DEP_CUT)[0] == 0.0
    g, _ = o.dump(workloads.GAMMA)
    b = oracle_mod.philox([0, 1, 0, 0], [1, 0])
    c = 2.0 * ((int(b[1]) + 0.5) * 2.0**-32) - 1.0
    ph = 2.0 * math.pi * ((int(b[2]) + 0.5) * 2.0**-32)
    st = math.sqrt(max(0.0, 1.0 - c * c))
    d = np.array([st * math.cos(ph), st * math.sin(ph), c])
    assert np.allclose(g[0]["dir"], d, rtol=0, atol=4e-16)
    assert np.all(g[1]["dir"] == -g[0]["dir"])  # a bitwise sign flip
    for k in range(2):
        assert g[k]["E"] == 0.511 and g[k]["pos"][2] == 2.0 / 1.27 and g[k]["volume"] == 0
        assert g[k]["parentId"] == 0 and g[k]["rngCtr"] == 0 and g[k]["numIALeft"] == -1.0
        assert g[k]["trackId"] == oracle_mod.child_id(1, 0, 0, k)
        assert g[k]["trackId"] >> 63 == 1
    # children ids are the first two words of blocks 2 and 3, top bit forced
    b2 = oracle_mod.philox([0, 2, 0, 0], [1, 0])
    assert g[0]["trackId"] == (1 << 63) | (((int(b2[0]) << 32) | int(b2[1])) & ((1 << 63) - 1))


@pytest.mark.parametrize("scheme", [0, 1])
def test_subcut_creations(oracle_mod, scheme):
    o = oracle_mod.Oracle(scheme, oracle_mod.FP64, 64, [1])
    o.set_instrumented(True, 10)
    assert o.inject(one(workloads.GAMMA, 0.05, nl=-1.0)) == 0
    assert list(o.counts()) == [0, 0, 0]
    assert o.tally(oracle_mod.T_DEP_CUT)[0] == G["subcut_gamma.deposit"]
    for t in range(3):
        r, w = o.access_totals(t, 0)
        assert r.sum() == 0 and w.sum() == 0
    rc, it = o.run()
    assert rc == 0 and it == 0
    o2 = oracle_mod.Oracle(scheme, oracle_mod.FP64, 64, [1])
    assert o2.inject(one(workloads.POSITRON, 0.5, nl=-1.0)) == 0
    assert o2.tally(oracle_mod.T_DEP_CUT)[0] == G["subcut_positron.deposit"]
    assert abs(o2.tally(oracle_mod.T_EIN)[0] - G["subcut_positron.input_energy"]) < 1e-15
    g, _ = o2.dump(workloads.GAMMA)
    assert len(g) == 2 and np.all(g[1]["dir"] == -g[0]["dir"]) and np.all(g["E"] == 0.511)


def test_forced_no_brem_layer_deposit(oracle_mod):
    """A 100 GeV electron that never interacts loses 1.27*2.3 + 0.21*5.7 = 4.118 MeV per
    layer; its multiple scattering angle stays below 1e-3 so the path-length
    excess (theta^2/2) is below 1e-6."""
    o = oracle_mod.Oracle(oracle_mod.DENSE, oracle_mod.FP64, 64, [1])
    assert o.inject(one(workloads.ELECTRON, 1e5, nl=1e9)) == 0
    rc, it = o.run()
    assert rc == 0 and it == 100
    lay = o.tally(oracle_mod.T_LAYER)
    assert np.allclose(lay, 1.27 * 2.3 + 0.21 * 5.7, rtol=1e-6, atol=0)
    assert abs(o.tally(oracle_mod.T_ESCAPED)[0] - (1e5 - lay.sum())) < 1e-9
