"""adept_dump_tracks_noalloc (device staging in the library's fixed per-GPU
array) against adept_dump_tracks (staging allocated per call): the same records
and slot numbers byte for byte, on two calls in a row of which the second dumps
fewer tracks than the first (the array still holds the first call's records
beyond them), in both track data structures; a dump larger than the array is
refused with ADEPT_E_INVALID and leaves the context usable."""
import os
import re
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


def same_dump(ad, sim, what):
    sizes = []
    for t in range(3):
        g, gs = ad.adept_dump_tracks(sim.ctx, t)
        h, hs = ad.adept_dump_tracks_noalloc(sim.ctx, t)
        assert len(g) == len(h), (what, t)
        assert g.tobytes() == h.tobytes(), (what, t)
        assert np.array_equal(gs, hs), (what, t)
        h2, none = ad.adept_dump_tracks_noalloc(sim.ctx, t, with_slots=False)
        assert none is None and h2.tobytes() == g.tobytes(), (what, t)
        sizes.append(len(g))
    return sizes


@pytest.mark.parametrize("scheme,mapping", [(1, 1), (0, 0)])
def test_noalloc_dump_matches_dump_twice_smaller_second(ad, scheme, mapping):
    wl = workloads.showers_100e_1gev()
    say(f"no-alloc dump: scheme {scheme} mapping {mapping}, 100 e- x 1 GeV, then 20 of them")
    sim = ad.Sim(scheme, mapping, ad.MIXED, 1 << 18, seeds=wl.seeds)
    sim.inject(wl.primaries)
    for _ in range(40):
        sim.step()
    first = same_dump(ad, sim, "first")
    sim.close()
    small = wl.subset(20)
    sim = ad.Sim(scheme, mapping, ad.MIXED, 1 << 18, seeds=small.seeds)
    sim.inject(small.primaries)
    for _ in range(25):
        sim.step()
    second = same_dump(ad, sim, "second")
    sim.close()
    say(f"  tracks per type: first {first}, second {second}")
    assert sum(first) > 0 and all(s <= f for s, f in zip(second, first)) and sum(second) < sum(first)


def noalloc_bytes():
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "adept.h")).read()
    m = re.search(r"#define ADEPT_NOALLOC_BYTES \((\d+)u << (\d+)\)", hdr)
    return int(m.group(1)) << int(m.group(2))


def test_noalloc_dump_refuses_beyond_its_array(ad):
    limit = noalloc_bytes()
    n = 2 * (limit // 96)  # about a quarter interact in the first absorber: still more photons than fit
    say(f"no-alloc dump: {n} photons of 10 MeV, one iteration, beyond the {limit}-byte array")
    prims = workloads.primaries(n, ptype=workloads.GAMMA, energy=10.0)
    sim = ad.Sim(1, 1, ad.MIXED, 1 << 19, seeds=(1,))
    sim.inject(prims)
    sim.step()
    cnt = sim.stats()["counts"][workloads.GAMMA]
    assert cnt * 96 > limit
    with pytest.raises(ad.AdeptError) as e:
        ad.adept_dump_tracks_noalloc(sim.ctx, workloads.GAMMA)
    assert e.value.code == -1 and "no-alloc" in str(e.value)
    g, _ = ad.adept_dump_tracks(sim.ctx, workloads.GAMMA)  # the context is still usable
    assert len(g) == cnt
    sim.close()
