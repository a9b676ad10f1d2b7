"""Invariants of the oracle that hold at any size.

* exact energy closure: input energy = continuous + cut deposits + escaped +
  in flight + rounding residual, to the tally summation rounding (<= 1e-13);
* the two buffer schemes of paper Sec. 2 carry identical track histories in
  identical order (only slot numbers differ), hence identical tallies;
* batch invariance: an event's tracks do not depend on other events;
* sparse slot bookkeeping against a naive FIFO free-list model (brute force on
  tiny capacities), including the iteration at which an overflow latches;
* heatmaps (paper Sec. 5): the per-byte maps of every layout expand the same
  per-(slot, field) counts, padding stays 0, totals match the field totals;
* the mixed-precision policy changes few discrete decisions.
"""
import collections
import math

import numpy as np
import pytest

import workloads


def closure(o, oracle_mod):
    ein = o.tally(oracle_mod.T_EIN)
    cont = o.tally(oracle_mod.T_DEP_CONT).reshape(len(ein), 100).sum(axis=1)
    cut = o.tally(oracle_mod.T_DEP_CUT).reshape(len(ein), 100).sum(axis=1)
    tot = cont + cut + o.tally(oracle_mod.T_ESCAPED) + o.tally(oracle_mod.T_INFLIGHT) + o.tally(oracle_mod.T_ROUND)
    return np.abs(ein - tot) / ein


def small_mixed_batch():
    """Three events: electrons, photons and positrons of several energies."""
    parts = [
        workloads.primaries(4, workloads.ELECTRON, 300.0, event=0),
        workloads.primaries(3, workloads.GAMMA, 120.0, event=1),
        workloads.primaries(3, workloads.POSITRON, 80.0, event=2),
        workloads.primaries(2, workloads.POSITRON, 0.7, event=2, first_id=3),
        workloads.primaries(1, workloads.GAMMA, 0.05, event=1, first_id=3),
    ]
    return np.concatenate(parts)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheme", [0, 1])
def test_energy_closure(oracle_mod, scheme, precision):
    o = oracle_mod.Oracle(scheme, precision, 1 << 14, [5, 6, 7])
    assert o.inject(small_mixed_batch()) == 0
    rc, it = o.run(30)
    assert rc == 0 and it == 30
    assert np.all(closure(o, oracle_mod) <= 1e-13)
    assert o.tally(oracle_mod.T_INFLIGHT).sum() > 0
    rc, it = o.run()
    assert rc == 0 and list(o.counts()) == [0, 0, 0]
    assert np.all(closure(o, oracle_mod) <= 1e-13)
    assert o.tally(oracle_mod.T_INFLIGHT).sum() == 0
    if precision == 0:
        # binary64: the only residuals are the pair-threshold TwoSums
        assert np.all(np.abs(o.tally(oracle_mod.T_ROUND)) < 1e-12)


@pytest.mark.parametrize("precision", [0, 1])
def test_dense_and_sparse_agree(oracle_mod, precision):
    wl = workloads.showers_100e_1gev().subset(10)
    od = oracle_mod.Oracle(oracle_mod.DENSE, precision, 1 << 14, wl.seeds)
    os_ = oracle_mod.Oracle(oracle_mod.SPARSE, precision, 1 << 14, wl.seeds)
    assert od.inject(wl.primaries) == 0 and os_.inject(wl.primaries) == 0
    while True:
        rc1, n1 = od.step()
        rc2, n2 = os_.step()
        assert rc1 == rc2 == 0 and list(n1) == list(n2)
        for t in range(3):
            a, _ = od.dump(t)
            b, _ = os_.dump(t)
            assert a.tobytes() == b.tobytes()
        if n1.sum() == 0:
            break
    for k in (oracle_mod.T_DEP_CONT, oracle_mod.T_DEP_CUT, oracle_mod.T_ESCAPED, oracle_mod.T_ROUND):
        assert np.array_equal(od.tally(k), os_.tally(k))
    assert od.stats()["track_steps"] == os_.stats()["track_steps"]


def test_batch_invariance(oracle_mod):
    a = workloads.primaries(3, workloads.ELECTRON, 500.0, event=0)
    b = workloads.primaries(5, workloads.GAMMA, 200.0, event=1)
    solo = oracle_mod.Oracle(oracle_mod.DENSE, 0, 1 << 14, [11])
    both = oracle_mod.Oracle(oracle_mod.DENSE, 0, 1 << 14, [11, 12])
    assert solo.inject(a) == 0 and both.inject(np.concatenate([b, a])) == 0
    for _ in range(400):
        r1, n1 = solo.step()
        r2, _ = both.step()
        assert r1 == r2 == 0
        for t in range(3):
            x, _ = solo.dump(t)
            y, _ = both.dump(t)
            y = y[y["event"] == 0]
            assert np.array_equal(x[list(x.dtype.names[:-1])], y[list(y.dtype.names[:-1])])
        if n1.sum() == 0:
            break
    assert np.array_equal(solo.tally(oracle_mod.T_LAYER), both.tally(oracle_mod.T_LAYER)[:50])


def naive_sparse_slots(oracle_mod, prims, seeds, C, n_iter):
    """Slots of every current track per iteration, from a FIFO free list kept in a
    deque, replaying the canonical track order of a dense run."""
    d = oracle_mod.Oracle(oracle_mod.DENSE, 0, 1 << 20, seeds)
    assert d.inject(prims) == 0
    free = [collections.deque(range(C)) for _ in range(3)]
    slot_of = [dict() for _ in range(3)]
    cur = []
    overflow = None
    for t in range(3):
        tr, _ = d.dump(t)
        if len(tr) > len(free[t]):
            return None, 0
        for x in tr:
            slot_of[t][int(x["trackId"])] = free[t].popleft()
        cur.append([int(x["trackId"]) for x in tr])
    history = [[[slot_of[t][i] for i in cur[t]] for t in range(3)]]
    for it in range(1, n_iter + 1):
        rc, n = d.step()
        assert rc == 0
        new_cur = []
        for t in range(3):
            tr, _ = d.dump(t)
            ids = [int(x["trackId"]) for x in tr]
            old = set(cur[t])
            allocs = [i for i in ids if i not in old]
            if len(allocs) > len(free[t]) and overflow is None:
                overflow = it
                return history, overflow
            for i in allocs:
                slot_of[t][i] = free[t].popleft()
            kept = set(ids)
            for i in cur[t]:
                if i not in kept:
                    free[t].append(slot_of[t].pop(i))
            new_cur.append(ids)
        cur = new_cur
        history.append([[slot_of[t][i] for i in cur[t]] for t in range(3)])
        if n.sum() == 0:
            break
    return history, overflow


def test_sparse_slots_match_naive_fifo(oracle_mod):
    prims = workloads.primaries(2, workloads.ELECTRON, 200.0)
    C = 256
    hist, ovf = naive_sparse_slots(oracle_mod, prims, [1], C, 2000)
    assert ovf is None
    s = oracle_mod.Oracle(oracle_mod.SPARSE, 0, C, [1])
    assert s.inject(prims) == 0
    for it, want in enumerate(hist):
        if it > 0:
            rc, _ = s.step()
            assert rc == 0
        for t in range(3):
            _, slots = s.dump(t)
            assert list(slots) == want[t], (it, t)
    # the whole ring was walked: many distinct slots were used
    assert s.stats()["slots_touched"][2] > 64


@pytest.mark.parametrize("scheme", [0, 1])
def test_overflow_iteration_predicted(oracle_mod, scheme):
    prims = workloads.primaries(3, workloads.ELECTRON, 1000.0)
    C = 48
    if scheme == 1:
        d = oracle_mod.Oracle(oracle_mod.DENSE, 0, 1 << 20, [1])
        d.inject(prims)
        want = None
        for it in range(1, 1000):
            _, n = d.step()
            if n.max() > C:
                want = it
                break
    else:
        _, want = naive_sparse_slots(oracle_mod, prims, [1], C, 1000)
    assert want is not None
    o = oracle_mod.Oracle(scheme, 0, C, [1])
    assert o.inject(prims) == 0
    rc, it = o.run()
    assert rc == oracle_mod.E_CAPACITY
    assert o.stats()["error_iter"] == want and it == want - 1


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheme", [0, 1])
def test_heatmaps_expand_field_counts(oracle_mod, scheme, precision):
    C = 1024
    o = oracle_mod.Oracle(scheme, precision, C, [1])
    o.set_instrumented(True, 20)
    assert o.inject(workloads.primaries(2, workloads.ELECTRON, 100.0)) == 0
    o.run(40)
    sizes = np.array([oracle_mod.leaf_size(precision, l) for l in range(14)])
    for t in range(3):
        for b in range(2 if scheme == 1 else 1):
            sl = o.access_slotleaf(t, b)
            r, w = o.access_totals(t, b)
            assert np.array_equal(sl.sum(axis=0), (r + w).astype(np.uint32))
            want_total = int((sl.astype(np.int64) * (sizes // 4)).sum())
            for mapping, lanes in ((0, 1), (1, 1), (2, 64), (2, 4)):
                h = o.heat_words(t, b, mapping, lanes)
                assert int(h.sum(dtype=np.int64)) == want_total
                if mapping == 0 and precision == 1:
                    assert np.all(h.reshape(C, 20)[:, 11] == 0)  # the 4 padding bytes of each record
                # per-slot totals are the same whatever the layout
                if mapping == 0:
                    per_slot = h.reshape(C, -1).sum(axis=1)
                    assert np.array_equal(per_slot, (sl.astype(np.int64) * (sizes // 4)).sum(axis=1))


def test_counts_stop_after_window(oracle_mod):
    o = oracle_mod.Oracle(oracle_mod.DENSE, 0, 4096, [1])
    o.set_instrumented(True, 3)
    assert o.inject(workloads.primaries(1, workloads.GAMMA, 0.5, num_ia_left=100.0)) == 0
    o.run(10)
    r, w = o.access_totals(workloads.GAMMA, 0)
    r2, w2 = o.access_totals(workloads.GAMMA, 1)
    assert (r + r2)[0] == 3 and (w + w2)[0] == 4  # injection + 3 iterations


def test_mixed_policy_flips_are_rare(oracle_mod):
    wl = workloads.showers_100e_1gev().subset(50)
    a = oracle_mod.Oracle(oracle_mod.DENSE, 0, 1 << 16, wl.seeds)
    b = oracle_mod.Oracle(oracle_mod.DENSE, 1, 1 << 16, wl.seeds)
    a.inject(wl.primaries)
    b.inject(wl.primaries)
    for _ in range(40):
        a.step()
        b.step()
    same = total = 0
    for t in range(3):
        x, _ = a.dump(t)
        y, _ = b.dump(t)
        kx = {(int(r["trackId"]), int(r["rngCtr"]), int(r["volume"])) for r in x}
        ky = {(int(r["trackId"]), int(r["rngCtr"]), int(r["volume"])) for r in y}
        same += len(kx & ky)
        total += max(len(kx), len(ky))
    assert total > 1000 and same / total > 0.99


def test_cell_scoring_closed_form(oracle_mod):
    """A non-interacting 100 GeV electron along z at x = 10.5, y = -3 deposits its
    whole continuous loss of every layer in cell (floor(210.5/4), floor(197/4)) = (52, 49)."""
    o = oracle_mod.Oracle(oracle_mod.DENSE, 0, 64, [1])
    o.set_scoring(100, 100, 4.0)
    p = workloads.primaries(1, workloads.ELECTRON, 1e5, pos=(10.5, -3.0, 0.0), num_ia_left=1e9)
    assert o.inject(p) == 0
    o.run()
    cells = o.tally(oracle_mod.T_CELLS).reshape(50, 100, 100)
    lay = o.tally(oracle_mod.T_LAYER)
    assert np.allclose(cells[:, 52, 49], lay, rtol=1e-12, atol=0)
    assert np.count_nonzero(cells) == 50
    # an edge position clamps into the last cell
    o2 = oracle_mod.Oracle(oracle_mod.DENSE, 0, 64, [1])
    o2.set_scoring(100, 100, 4.0)
    p2 = workloads.primaries(1, workloads.GAMMA, 0.05, pos=(200.0, -200.0, 0.0))
    o2.inject(p2)
    c2 = o2.tally(oracle_mod.T_CELLS).reshape(50, 100, 100)
    assert c2[0, 99, 0] == 0.05


def test_admission_properties(oracle_mod):
    wl = workloads.uneven_512_events(n_events=6, max_per_event=3)
    kappa = [2.0, 2.0, 20.0]
    solo = oracle_mod.Oracle(oracle_mod.DENSE, 0, 1 << 16, wl.seeds)
    assert solo.inject(wl.primaries) == 0
    solo.run()
    # generous limit: everything is admitted before the first iteration
    a = oracle_mod.Oracle(oracle_mod.DENSE, 0, 1 << 16, wl.seeds)
    a.set_admission(True, 0.8, kappa)
    a.stage(wl.primaries)
    a.run()
    for k in (oracle_mod.T_DEP_CONT, oracle_mod.T_DEP_CUT, oracle_mod.T_ESCAPED):
        assert np.array_equal(a.tally(k), solo.tally(k))
    assert a.stats()["iterations"] == solo.stats()["iterations"]
    # tight limit: events enter one at a time, per-event tallies are unchanged
    # (histories do not depend on admission timing) but the run is longer
    b = oracle_mod.Oracle(oracle_mod.DENSE, 0, 4096, wl.seeds)
    b.set_admission(True, 1e-6, kappa)
    b.stage(wl.primaries)
    rc, it = b.run()
    assert rc == 0
    assert it > solo.stats()["iterations"]
    assert np.allclose(b.tally(oracle_mod.T_LAYER), solo.tally(oracle_mod.T_LAYER), rtol=1e-12, atol=1e-12)
    assert b.stats()["track_steps"] == solo.stats()["track_steps"]


def _admission_trace(oracle_mod, wl, kappa, alpha, C, hold):
    """Step the oracle one iteration at a time; return, per iteration, the counts
    before it and the events whose energy entered during it."""
    o = oracle_mod.Oracle(oracle_mod.DENSE, 0, C, wl.seeds)
    o.set_admission(True, alpha, kappa, hold)
    o.stage(wl.primaries)
    seen = np.zeros(len(wl.seeds), dtype=bool)
    trace = []
    for _ in range(5000):
        before = o.counts().copy()
        rc, n = o.step()
        assert rc == 0
        ein = o.tally(oracle_mod.T_EIN)
        new = np.nonzero((ein > 0) & ~seen)[0]
        seen |= ein > 0
        trace.append((before, list(new)))
        if n.sum() == 0 and seen.all():
            break
    return o, trace


def test_admission_reservation_limits(oracle_mod):
    """The reservation window at its two ends: with an unbounded hold nothing is
    ever released, so after the first batch events enter one at a time and only
    when no track is active; with hold 0 every admission satisfies
    n + sum of projected peaks <= alpha * C on the counts of that iteration.
    Per-event tallies never depend on the hold."""
    wl = workloads.uneven_512_events(n_events=12, max_per_event=2)
    kappa = [4.0, 4.0, 40.0]
    alpha, C = 0.5, 4096
    E = wl.event_energy()
    need = lambda e: [math.ceil(k * E[e] / 1000.0) for k in kappa]
    inf, trace_inf = _admission_trace(oracle_mod, wl, kappa, alpha, C, 1 << 62)
    zero, trace_zero = _admission_trace(oracle_mod, wl, kappa, alpha, C, 0)
    first = True
    for before, new in trace_inf:
        if not new:
            continue
        if first:
            first = False
            tot = [sum(need(e)[d] for e in new) for d in range(3)]
            assert all(t <= alpha * C for t in tot) or len(new) == 1
        else:
            assert before.sum() == 0 and len(new) == 1, (before, new)
    batches = 0
    for before, new in trace_zero:
        if not new:
            continue
        batches += 1
        tot = [before[d] + sum(need(e)[d] for e in new) for d in range(3)]
        assert all(t <= alpha * C for t in tot) or (before.sum() == 0 and len(new) == 1), (before, new)
    assert batches >= 2
    # events admitted in order, each exactly once
    order = [e for _, new in trace_inf for e in new]
    assert order == list(range(len(wl.seeds)))
    assert [e for _, new in trace_zero for e in new] == order
    assert np.allclose(inf.tally(oracle_mod.T_LAYER), zero.tally(oracle_mod.T_LAYER), rtol=1e-12, atol=1e-12)
    assert inf.stats()["track_steps"] == zero.stats()["track_steps"]
    assert len(trace_inf) > len(trace_zero)


@pytest.mark.parametrize("scheme", [0, 1])
def test_divergence_diagnostic_groups_of_64(oracle_mod, scheme):
    """Per group of 64 consecutive sources of a type, the sources whose outcome
    differs from the group's most common one (case and expected count in
    oracle_pins.divergence_groups)."""
    import oracle_pins

    oracle_pins.divergence_groups(oracle_mod.load(oracle_mod.LIB), scheme)


def test_divergence_diagnostic_zero_for_uniform_groups(oracle_mod):
    """Identical photons that never interact share every outcome: nothing differs."""
    p = workloads.primaries(130, workloads.GAMMA, 10.0, num_ia_left=1000.0)
    o = oracle_mod.Oracle(1, oracle_mod.FP64, 1 << 10, [1])
    assert o.inject(p) == 0
    for _ in range(5):
        assert o.step()[0] == 0
    assert o.ledger()["off_mode"] == 0
    o.close()
