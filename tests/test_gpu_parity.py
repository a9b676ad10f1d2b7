"""GPU parity: the HIP library (through its C ABI) against the oracle.

Bit-exact: active counts, slot lists and free rings (sparse), every field of
every track (FP64 and mixed, -ffp-contract=off on both sides), access counts
and heatmaps.  Tallies: per-layer deposits within 1e-12 relative (the GPU sums
in a different order).  Sizes span several tiles and a ragged last tile.
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

SCHEMES = [0, 1]
LAYOUTS = [(0, 1), (1, 1), (2, 64)]  # AoS, SoA, AoSoA-64


@pytest.fixture(scope="module")
def ad():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_08252_amd as ad

    ad.lib()
    return ad


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare_state(sim, o, it, scheme, what=""):
    for t in range(3):
        g, gs = sim.dump(t)
        w, ws = o.dump(t)
        assert len(g) == len(w), (what, it, t, len(g), len(w))
        if g.tobytes() != w.tobytes():
            bad = np.nonzero(g.view(np.uint8).reshape(len(g), -1).any(axis=1) !=
                             w.view(np.uint8).reshape(len(w), -1).any(axis=1))[0]
            diff = [i for i in range(len(g)) if g[i].tobytes() != w[i].tobytes()][:3]
            raise AssertionError(f"{what} iter {it} type {t}: first differing tracks {diff}: "
                                 f"gpu {g[diff[0]]} oracle {w[diff[0]]} ({len(bad)})")
        if scheme == 0:
            assert np.array_equal(gs, ws), (what, it, t)


def compare_tallies(sim, o, oracle_mod, rtol=1e-12):
    E = o.n_events
    gl = sim.tally(oracle_mod.T_LAYER).reshape(E, 50)
    wl = o.tally(oracle_mod.T_LAYER).reshape(E, 50)
    assert np.all(np.abs(gl - wl) <= rtol * np.abs(wl) + 1e-300), np.max(np.abs(gl - wl) / np.maximum(np.abs(wl), 1e-300))
    for k in (oracle_mod.T_ESCAPED, oracle_mod.T_EIN):
        g, w = sim.tally(k), o.tally(k)
        assert np.all(np.abs(g - w) <= rtol * np.abs(w) + 1e-300)
    g, w = sim.tally(oracle_mod.T_ROUND), o.tally(oracle_mod.T_ROUND)
    assert np.all(np.abs(g - w) <= 1e-12 * o.tally(oracle_mod.T_EIN))


@pytest.mark.parametrize("wave", [0, 1], ids=["blocktile", "wavetile"])
@pytest.mark.parametrize("block", [64, 1024])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("mapping,lanes", LAYOUTS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_iterations_bitwise(ad, oracle_mod, scheme, mapping, lanes, precision, block, wave):
    """Primaries of 300 MeV to 3 GeV (several tiles, ragged tails): state after every
    iteration.  Block 64 runs one track per lane; block 1024 runs two per lane, with
    a tile of 2048 tracks (block tiles) or 128 (wave tiles), so the larger workload
    there."""
    say(f"case iterations_bitwise scheme={scheme} mapping={mapping} lanes={lanes} precision={precision} "
        f"block={block} wave={wave}")
    C = 1 << 16
    n_e, e_e = (10, 300.0) if block == 64 else (40, 3000.0)
    prims = np.concatenate([workloads.primaries(n_e, workloads.ELECTRON, e_e),
                            workloads.primaries(1, workloads.POSITRON, 40.0, first_id=n_e),
                            workloads.primaries(1, workloads.GAMMA, 25.0, first_id=n_e + 1)])
    sim = ad.Sim(scheme, mapping, precision, C, lanes, seeds=[3],
                 launch={"block": block, "graph_iters": 8, "wave_tiles": wave})
    o = oracle_mod.Oracle(scheme, precision, C, [3])
    sim.inject(prims)
    assert o.inject(prims) == 0
    compare_state(sim, o, 0, scheme, "inject")
    it = 0
    while True:
        g = sim.step()
        rc, w = o.step()
        it += 1
        assert rc == 0 and list(g) == list(w), (it, g, w)
        compare_state(sim, o, it, scheme)
        if scheme == 0:
            for t in range(3):
                gr, gh, gc = sim.ring(t)
                wr, wh, wc = o.ring(t)
                assert (gh, gc) == (wh, wc) and np.array_equal(gr, wr), (it, t)
        if w.sum() == 0:
            break
    compare_tallies(sim, o, oracle_mod)
    gs, ws = sim.stats(), o.stats()
    assert gs["track_steps"] == ws["track_steps"] and gs["iterations"] == ws["iterations"]
    led = o.ledger()  # the counters the roofline's byte count is built from
    assert gs["survivors"] == led["survivors"] and gs["outputs"] == led["outputs"], (gs, led)
    assert gs["off_mode"] == led["off_mode"], (gs["off_mode"], led["off_mode"])  # divergence diagnostic
    sim.close()


ANCHOR_LAUNCHES = [(64, 0), (128, 0), (256, 0), (512, 0), (1024, 0), (64, 1), (256, 1), (1024, 1)]


@pytest.mark.parametrize("block,wave", ANCHOR_LAUNCHES,
                         ids=[f"b{b}-{'wavetile' if w else 'blocktile'}" for b, w in ANCHOR_LAUNCHES])
def test_anchor_run_graph(ad, oracle_mod, block, wave):
    """showers_100e_1gev as specified (sparse AoS FP64, 2^20 slots, 100 e- of 1 GeV, seed 1) through
    adept_run's graph replay: counts and stats exact, per-layer deposits 1e-12."""
    say(f"case anchor_run_graph block={block} wave={wave}")
    wl = workloads.showers_100e_1gev()
    sim = ad.Sim(0, 0, 0, 1 << 20, 1, seeds=wl.seeds,
                 launch={"block": block, "graph_iters": 32, "wave_tiles": wave})
    sim.inject(wl.primaries)
    it = sim.run()
    o, rc, oit = oracle_mod.run_workload(wl, oracle_mod.SPARSE, oracle_mod.FP64, 1 << 20)
    assert rc == 0 and it == oit
    gs, ws = sim.stats(), o.stats()
    assert gs["track_steps"] == ws["track_steps"] and gs["peak"] == ws["peak"]
    led = o.ledger()
    assert gs["survivors"] == led["survivors"] and gs["outputs"] == led["outputs"]
    assert gs["off_mode"] == led["off_mode"]
    compare_tallies(sim, o, oracle_mod)
    for t in range(3):
        gr, gh, gc = sim.ring(t)
        wr, wh, wc = o.ring(t)
        assert (gh, gc) == (wh, wc) and np.array_equal(gr, wr)
    sim.close()


def test_single_track_traces(ad, oracle_mod):
    say("case single_track_traces")
    for scheme in SCHEMES:
        for precision in (0, 1):
            sim = ad.Sim(scheme, 1, precision, 256, 1, seeds=[1], instrumented=1000)
            o = oracle_mod.Oracle(scheme, precision, 256, [1])
            o.set_instrumented(True, 1000)
            p = workloads.primaries(1, workloads.GAMMA, 0.5, num_ia_left=100.0)
            sim.inject(p)
            o.inject(p)
            for it in range(1, 101):
                assert list(sim.step()) == list(o.step()[1])
                compare_state(sim, o, it, scheme, "gamma")
            assert sim.tally(oracle_mod.T_ESCAPED)[0] == 0.5
            for b in range(2 if scheme else 1):
                r, w = sim.access_counts(2, b)
                rr, ww = o.access_totals(2, b)
                assert np.array_equal(r, rr) and np.array_equal(w, ww)
            sim.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("mapping,lanes", [(0, 1), (1, 1), (2, 64), (2, 8)])
@pytest.mark.parametrize("scheme", SCHEMES)
def test_instrumented_counts_and_heatmaps(ad, oracle_mod, scheme, mapping, lanes, precision):
    """Instrumented mode over injection + the first 20 iterations: per-field read/write
    totals and per-word heatmaps bit-exact with the oracle's counts expanded through its
    own byte map of the same layout."""
    say(f"case instrumented scheme={scheme} mapping={mapping} lanes={lanes} precision={precision}")
    C = 1 << 12
    prims = workloads.primaries(4, workloads.ELECTRON, 200.0)
    sim = ad.Sim(scheme, mapping, precision, C, lanes, seeds=[1], instrumented=20, launch={"block": 128})
    o = oracle_mod.Oracle(scheme, precision, C, [1])
    o.set_instrumented(True, 20)
    sim.inject(prims)
    o.inject(prims)
    sim.run(30)
    o.run(30)
    for t in range(3):
        for b in range(2 if scheme else 1):
            r, w, h = sim.access_counts(t, b, heat=True)
            rr, ww = o.access_totals(t, b)
            assert np.array_equal(r, rr) and np.array_equal(w, ww), (t, b, r, rr, w, ww)
            want = o.heat_words(t, b, mapping, lanes)
            assert np.array_equal(h, want), (t, b)
            for lb in (64, 128):  # per-cache-line heat, ragged last line included
                pad = np.zeros(-len(want) % (lb // 4), dtype=np.uint64)
                lines = np.concatenate([want.astype(np.uint64), pad]).reshape(-1, lb // 4).sum(axis=1)
                assert np.array_equal(sim.line_heat(t, b, lb), lines), (t, b, lb)
    sim.close()


@pytest.mark.parametrize("scheme", SCHEMES)
def test_capacity_overflow_iteration(ad, oracle_mod, scheme):
    say(f"case overflow scheme={scheme}")
    prims = workloads.primaries(3, workloads.ELECTRON, 1000.0)
    C = 64
    o = oracle_mod.Oracle(scheme, 0, C, [1])
    o.inject(prims)
    rc, _ = o.run()
    assert rc == oracle_mod.E_CAPACITY
    sim = ad.Sim(scheme, 0, 0, C, 1, seeds=[1])
    sim.inject(prims)
    with pytest.raises(ad.AdeptError) as e:
        sim.run()
    assert e.value.code == ad.E_CAPACITY
    assert sim.stats()["error_iter"] == o.stats()["error_iter"]
    sim.close()


def test_invalid_primaries_rejected(ad):
    say("case invalid primaries")
    sim = ad.Sim(1, 1, 1, 1024, 1, seeds=[1])
    bad = workloads.primaries(2, workloads.ELECTRON, 10.0)
    bad["pos"][1, 2] = 401.0
    with pytest.raises(ad.AdeptError) as e:
        sim.inject(bad)
    assert e.value.code == ad.E_INVALID
    assert list(sim.counts()) == [0, 0, 0]
    bad = workloads.primaries(1, workloads.ELECTRON, float("nan"))
    with pytest.raises(ad.AdeptError):
        sim.inject(bad)
    bad = workloads.primaries(1, 5, 10.0)
    with pytest.raises(ad.AdeptError):
        sim.inject(bad)
    sim.inject(workloads.primaries(1, workloads.ELECTRON, 10.0))
    assert sum(sim.counts()) == 1
    sim.close()


@pytest.mark.parametrize("precision,hold,block", [(0, 128, 128), (1, 128, 1024), (1, 0, 128), (0, 40, 1024), (1, 40, 512)])
def test_batched_admission_and_cells(ad, oracle_mod, precision, hold, block):
    """Uneven events of mixed particle types with per-event tallies, admission
    (with several reservation windows) and per-cell scoring, against the oracle
    under the same admission rule.  Block 128 runs more blocks than there are
    tally rows (the rest add to the tallies directly); 512 and 1024 run tiles of
    two tracks per lane under the mixed policy."""
    say(f"case batched precision={precision} hold={hold} block={block}")
    wl = workloads.uneven_512_events(n_events=24, max_per_event=6)
    kappa = [3.0, 2.0, 25.0]
    C = 1 << 14  # tight enough that admission staggers the events for hold > 0
    sim = ad.Sim(1, 1, precision, C, 1, seeds=wl.seeds, scoring=(100, 100, 4.0), admission=(0.8, kappa, hold),
                 launch={"block": block, "graph_iters": 16})
    o = oracle_mod.Oracle(oracle_mod.DENSE, precision, C, wl.seeds)
    o.set_scoring(100, 100, 4.0)
    o.set_admission(True, 0.8, kappa, hold)
    o.stage(wl.primaries)
    sim.inject(wl.primaries)
    for it in range(1, 40):
        g = sim.step()
        rc, w = o.step()
        assert rc == 0 and list(g) == list(w), it
        compare_state(sim, o, it, 1, "batched")
    rc, oit = o.run()
    assert rc == 0
    it = sim.run()
    assert it == oit
    compare_tallies(sim, o, oracle_mod)
    gc, wc = sim.tally(oracle_mod.T_CELLS), o.tally(oracle_mod.T_CELLS)
    assert np.allclose(gc, wc, rtol=1e-12, atol=1e-9)
    gs, led = sim.stats(), o.ledger()
    assert gs["track_steps"] == o.stats()["track_steps"]
    assert gs["survivors"] == led["survivors"] and gs["outputs"] == led["outputs"]
    sim.close()


def test_determinism_and_launch_invariance(ad, oracle_mod):
    say("case determinism")
    wl = workloads.showers_100e_1gev().subset(20)
    res = []
    for block, k in ((64, 4), (256, 32), (128, 1)):
        sim = ad.Sim(1, 2, 1, 1 << 16, 32, seeds=wl.seeds, launch={"block": block, "graph_iters": k})
        sim.inject(wl.primaries)
        sim.run(25)
        res.append([sim.dump(t)[0].tobytes() for t in range(3)] + [sim.stats()["track_steps"]])
        sim.close()
    assert res[0] == res[1] == res[2]


def test_layout_study_counts_full_size(ad, oracle_mod):
    """The layout study at full size: 10^4 e- of 10 GeV (seed 1), instrumented over
    injection + the first 20 iterations, in sparse AoS and dense AoS / SoA / AoSoA-64
    (FP64).  Per-field read/write totals and per-word heatmaps bit-exact; the per-field
    totals are the same for every layout of one scheme."""
    say("case showers_10ke_10gev layout study, full size")
    wl = workloads.showers_10ke_10gev()
    C = 1 << 22
    for scheme, layouts in ((0, [(0, 1)]), (1, [(0, 1), (1, 1), (2, 64)])):
        o = oracle_mod.Oracle(scheme, 0, C, wl.seeds)
        o.set_instrumented(True, 20)
        assert o.inject(wl.primaries) == 0
        rc, _ = o.run(20)
        assert rc == 0
        for mapping, lanes in layouts:
            say(f"  scheme={scheme} mapping={mapping} lanes={lanes}")
            sim = ad.Sim(scheme, mapping, 0, C, lanes, seeds=wl.seeds, instrumented=20,
                         launch={"block": 256, "graph_iters": 32})
            sim.inject(wl.primaries)
            assert sim.run(20) == 20
            for t in range(3):
                for b in range(2 if scheme else 1):
                    r, w, h = sim.access_counts(t, b, heat=True)
                    rr, ww = o.access_totals(t, b)
                    assert np.array_equal(r, rr) and np.array_equal(w, ww), (scheme, mapping, t, b)
                    assert np.array_equal(h, o.heat_words(t, b, mapping, lanes)), (scheme, mapping, t, b)
            gs = sim.stats()
            assert gs["track_steps"] == o.stats()["track_steps"]
            sim.close()


def test_autotune_keeps_results(ad, oracle_mod):
    """The autotuner only changes the launch configuration: the run it leaves behind
    reproduces the oracle's counts and deposits."""
    say("case autotune")
    wl = workloads.uneven_512_events(n_events=16, max_per_event=20)
    C = 1 << 16
    sim = ad.Sim(1, 1, 1, C, 1, seeds=wl.seeds)
    choice = ad.adept_autotune(sim.ctx, wl.primaries)
    assert choice["block"] in (64, 128, 256, 512, 1024) and choice["graph_iters"] in (16, 64)
    sim.inject(wl.primaries)
    sim.run()
    o, rc, _ = oracle_mod.run_workload(wl, oracle_mod.DENSE, oracle_mod.MIXED, C)
    assert rc == 0
    assert sim.stats()["track_steps"] == o.stats()["track_steps"]
    compare_tallies(sim, o, oracle_mod)
    sim.close()


def test_layout_autotuner_keeps_results(ad, oracle_mod):
    """adept_autotune_layout picks one of the candidate layouts; a run in the chosen
    layout and launch configuration reproduces the oracle's state and deposits."""
    say("case layout autotuner")
    wl = workloads.uneven_512_events(n_events=8, max_per_event=12)
    cands = [(1, 0, 1), (1, 1, 1), (1, 2, 64), (0, 0, 1)]
    C = 1 << 16
    layout, launch, ms = ad.adept_autotune_layout(ad.MIXED, C, cands, wl.seeds, wl.primaries)
    assert layout in cands and ms > 0
    sim = ad.Sim(layout[0], layout[1], ad.MIXED, C, layout[2], seeds=wl.seeds, launch=launch)
    sim.inject(wl.primaries)
    o = oracle_mod.Oracle(layout[0], oracle_mod.MIXED, C, wl.seeds)
    assert o.inject(wl.primaries) == 0
    sim.run(30)
    o.run(30)
    compare_state(sim, o, 30, layout[0], "autotuned layout")
    sim.run()
    o.run()
    compare_tallies(sim, o, oracle_mod)
    sim.close()


def test_timed_mode_keeps_results(ad, oracle_mod):
    """Timed mode (iterations launched one by one with an event pair around every step
    kernel, in chunks of graph_iters) gives the untimed results; every step launch is
    timed and the summed kernel time fits inside the wall time of the run."""
    import time

    import torch

    say("case timed_mode")
    wl = workloads.showers_100e_1gev()
    sim = ad.Sim(1, 1, 1, 1 << 16, seeds=wl.seeds, launch={"block": 1024, "graph_iters": 16})
    sim.inject(wl.primaries)
    ref_it = sim.run()
    ref = sim.tally(oracle_mod.T_LAYER)
    sim.reset()
    ad.adept_set_timing(sim.ctx, True)
    sim.inject(wl.primaries)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = sim.run(5)  # a partial chunk
    it += sim.run()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    st = sim.stats()
    assert it == ref_it and np.array_equal(sim.tally(oracle_mod.T_LAYER), ref)
    assert st["step_launches"] == 5 + -(-(ref_it - 5) // 16) * 16
    assert 0 < st["step_kernel_ms"] < wall_ms
    sim.close()
