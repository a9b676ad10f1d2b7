"""GPU parity of the per-particle-type layouts (one record layout per type's
buffers, the future work of paper Sec. 6) against the oracle: the same bit-exact
bar as the shared layouts, since no result depends on where a field is stored."""
import ctypes

import numpy as np
import pytest

import workloads
from test_gpu_parity import ad, compare_state, compare_tallies, say  # noqa: F401  (ad is a fixture)

pytestmark = pytest.mark.gpu

# electron, positron, photon: three different mappings
TYPED = [(0, 1), (2, 8), (1, 1)]
TYPED_B = [(2, 64), (1, 1), (0, 1)]


@pytest.mark.parametrize("block", [64, 1024])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheme", [0, 1])
def test_typed_iterations_bitwise(ad, oracle_mod, scheme, precision, block):
    say(f"case typed_iterations_bitwise scheme={scheme} precision={precision} block={block}")
    C = 1 << 16
    n_e, e_e = (10, 300.0) if block == 64 else (40, 3000.0)
    prims = np.concatenate([workloads.primaries(n_e, workloads.ELECTRON, e_e),
                            workloads.primaries(1, workloads.POSITRON, 40.0, first_id=n_e),
                            workloads.primaries(1, workloads.GAMMA, 25.0, first_id=n_e + 1)])
    lay = TYPED if block == 64 else TYPED_B
    sim = ad.Sim(scheme, 0, precision, C, seeds=[3], launch={"block": block, "graph_iters": 8}, type_layouts=lay)
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
    sim.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheme", [0, 1])
def test_typed_heatmaps_and_sizes(ad, oracle_mod, scheme, precision):
    """Instrumented injection + 20 iterations: per-field totals and per-word heatmaps
    of every type's buffers equal the oracle's counts expanded through that type's
    own mapping; buffer sizes per type; the shared-size query refuses."""
    say(f"case typed_heatmaps scheme={scheme} precision={precision}")
    C = 1 << 12
    prims = workloads.primaries(4, workloads.ELECTRON, 200.0)
    sim = ad.Sim(scheme, 0, precision, C, seeds=[1], instrumented=20, launch={"block": 128}, type_layouts=TYPED)
    o = oracle_mod.Oracle(scheme, precision, C, [1])
    o.set_instrumented(True, 20)
    sim.inject(prims)
    o.inject(prims)
    sim.run(30)
    o.run(30)
    for t, (mapping, lanes) in enumerate(TYPED):
        assert ad.adept_type_buffer_bytes(sim.ctx, t) == oracle_mod.buffer_bytes(mapping, lanes, precision, C)
        for b in range(2 if scheme else 1):
            r, w, h = sim.access_counts(t, b, heat=True)
            rr, ww = o.access_totals(t, b)
            assert np.array_equal(r, rr) and np.array_equal(w, ww), (t, b)
            want = o.heat_words(t, b, mapping, lanes)
            assert np.array_equal(h, want), (t, b)
            pad = np.zeros(-len(want) % 32, dtype=np.uint64)
            assert np.array_equal(sim.line_heat(t, b, 128),
                                  np.concatenate([want.astype(np.uint64), pad]).reshape(-1, 32).sum(axis=1))
    n = ctypes.c_size_t()
    assert ad.lib().adept_buffer_bytes(sim.ctx, ctypes.byref(n)) == ad.E_INVALID
    sim.close()


def test_typed_autotuner_keeps_results(ad, oracle_mod):
    """The per-type autotuner on a small sample returns valid layouts; a run with its
    choice gives the oracle's counts and tallies."""
    say("case typed_autotuner")
    wl = workloads.showers_100e_1gev()
    cands = [(1, 0, 1), (1, 1, 1), (1, 2, 64)]
    lay, launch, ms = ad.adept_autotune_type_layouts(ad.MIXED, 1 << 16, cands, wl.seeds, wl.primaries)
    assert ms > 0 and all(l in [(m, n) for _, m, n in cands] for l in lay), lay
    sim = ad.Sim(1, 0, ad.MIXED, 1 << 16, seeds=wl.seeds, launch=launch, type_layouts=lay)
    sim.inject(wl.primaries)
    it = sim.run()
    o, rc, oit = oracle_mod.run_workload(wl, oracle_mod.DENSE, oracle_mod.MIXED, 1 << 16)
    assert rc == 0 and it == oit
    assert sim.stats()["track_steps"] == o.stats()["track_steps"]
    compare_tallies(sim, o, oracle_mod)
    sim.close()
