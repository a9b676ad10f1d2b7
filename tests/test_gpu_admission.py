"""Admission runs whose iterations inject many tiles of primaries at once.

During an admission run the injection kernel is launched before every iteration on
a small fixed grid (64 blocks), so an iteration that admits more tiles than that
has each block loop over several tiles, their order fixed by the look-back.  Here
(2^17 slots, 64-lane tiles) the first iteration admits an event of 5 000 primaries
(79 tiles), the ninth two events of 5 000 and 3 000 together (125 tiles) and the
seventeenth the last event of 6 000 (94 tiles), the schedule the oracle's admission
rule gives for these events; per-iteration
state (slot lists and free rings in the sparse scheme), per-event deposits and
the admission schedule must match the oracle under the same rule, in both buffer
schemes and both precision policies.
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


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


def large_events():
    """Four events of 5000, 5000, 3000 and 6000 primaries of 20-200 MeV (log-uniform),
    70/20/10 % electrons/photons/positrons, from one seeded generator."""
    g = np.random.Generator(np.random.PCG64(11))
    parts = []
    for e, n in enumerate((5000, 5000, 3000, 6000)):
        p = workloads.primaries(n, workloads.ELECTRON, 0.0, event=e)
        u = g.random(n)
        p["type"] = np.where(u < 0.7, workloads.ELECTRON, np.where(u < 0.9, workloads.GAMMA, workloads.POSITRON))
        p["E"] = 20.0 * np.power(10.0, g.random(n))
        parts.append(p)
    return np.concatenate(parts), np.array([11, 12, 13, 14], dtype=np.uint32)


def compare(sim, o, it, scheme):
    for t in range(3):
        g, gs = sim.dump(t)
        w, ws = o.dump(t)
        assert len(g) == len(w), (it, t, len(g), len(w))
        assert g.tobytes() == w.tobytes(), (it, t)
        if scheme == 0:
            assert np.array_equal(gs, ws), (it, t)
            gr, gh, gc = sim.ring(t)
            wr, wh, wc = o.ring(t)
            assert (gh, gc) == (wh, wc) and np.array_equal(gr, wr), (it, t)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheme", [0, 1])
def test_admission_injects_many_tiles_per_iteration(ad, oracle_mod, scheme, precision):
    say(f"case admission many tiles scheme={scheme} precision={precision}")
    prims, seeds = large_events()
    C = 1 << 17
    # peak tracks per GeV of these low-energy showers are about (12, 6, 64) when an
    # event's primaries start together; twice that keeps the events apart
    kappa = [26.0, 14.0, 140.0]
    sim = ad.Sim(scheme, 0, precision, C, 1, seeds=seeds, admission=(0.8, kappa, 8),
                 launch={"block": 64, "graph_iters": 8})
    o = oracle_mod.Oracle(scheme, precision, C, seeds)
    o.set_admission(True, 0.8, kappa, 8)
    o.stage(prims)
    sim.inject(prims)
    admitted = []
    it = 0
    while True:
        g = sim.step()
        rc, w = o.step()
        it += 1
        assert rc == 0 and list(g) == list(w), (it, g, w)
        compare(sim, o, it, scheme)
        ein = sim.tally(oracle_mod.T_EIN)
        assert np.array_equal(ein > 0, o.tally(oracle_mod.T_EIN) > 0), it
        admitted.append(int(np.count_nonzero(ein)))
        if w.sum() == 0 and admitted[-1] == len(seeds):
            break
        assert it < 5000
    say(f"  {it} iterations; events admitted by iteration 1: {admitted[0]}, "
        f"all four by iteration {admitted.index(len(seeds)) + 1}")
    assert admitted[0] == 1 and admitted.index(3) == 8 and admitted.index(len(seeds)) == 16, admitted[:20]
    E = len(seeds)
    gl = sim.tally(oracle_mod.T_LAYER).reshape(E, 50)
    wl = o.tally(oracle_mod.T_LAYER).reshape(E, 50)
    assert np.all(np.abs(gl - wl) <= 1e-12 * np.abs(wl) + 1e-300)
    for k in (oracle_mod.T_ESCAPED, oracle_mod.T_EIN, oracle_mod.T_ROUND):
        assert np.all(np.abs(sim.tally(k) - o.tally(k)) <= 1e-12 * o.tally(oracle_mod.T_EIN))
    st, led = sim.stats(), o.ledger()
    assert st["track_steps"] == o.stats()["track_steps"]
    assert st["survivors"] == led["survivors"] and st["outputs"] == led["outputs"]
    sim.close()
