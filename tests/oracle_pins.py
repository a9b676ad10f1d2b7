"""Pins of the oracle's Compton branch, interaction-length resamples and particle
ledger, written as functions of the oracle library handle so that the same checks
run against the oracle as built (test_oracle_compton.py) and against copies with one
planted mistake each (test_oracle_mutations.py), where they must fail.

What pins what (toy shower model: photons below the pair threshold 1.022 MeV
Compton-scatter with mean free path 2 X0 and hand a uniform share of their energy
to an electron; the photon is cut below 0.1 MeV, the electron below 1 MeV):

* kill fraction: a photon of energy E keeps E' = E - U E, so P(E' < 0.1) = 0.1 / E
  (binomial);
* spectrum: among surviving photons E'/E is uniform on (0.1 / E, 1) (KS);
* buffered electrons: only for 1.0 < E <= 1.022, with P(T >= 1) = 1 - 1 / E (binomial);
* hand trace: the transfer T = U(a3) E from word a3 of Philox block 0, the photon
  keeps E - T, the electron's T is the exact complement, the resampled interaction
  length is -log U(b0) from block 1 (computed here from the Philox words);
* resamples: after a Compton step and after a bremsstrahlung step the stored
  interaction length is Exp(1) (KS);
* ledger: primaries + creations = deaths + tracks in flight, per type; every
  Compton step makes one electron, every pair one electron and one positron, every
  bremsstrahlung one photon, every annihilation two photons; so the charge of all
  creations is minus the number of Compton steps.
"""
import math

import numpy as np
from scipy import stats

import oracle
import workloads

N = 20000


def _one_step(L, ptype, E, nl, precision, n=N, seed=3, scheme=oracle.DENSE):
    o = oracle.Oracle(scheme, precision, 1 << 16, [seed], L=L)
    p = workloads.primaries(n, ptype, E, num_ia_left=nl)
    assert o.inject(p) == 0
    rc, _ = o.step()
    assert rc == 0
    return o


def _binomial_ok(k, n, p, z=5.0):
    return abs(k - n * p) < z * math.sqrt(n * p * (1.0 - p))


def compton_kill_and_spectrum(L, E, precision):
    """Photons forced to interact at their first step (numIALeft 1e-9, s = 1.1e-8 mm)."""
    assert E < 1.022
    o = _one_step(L, workloads.GAMMA, E, 1e-9, precision)
    g, _ = o.dump(workloads.GAMMA)
    e, _ = o.dump(workloads.ELECTRON)
    assert np.all(g["volume"] == 0) and np.all(g["rngCtr"] == 1)
    killed = N - len(g)
    assert _binomial_ok(killed, N, 0.1 / E), (E, killed, N * 0.1 / E)
    lo = 0.1 / E
    u = (g["E"] / E - lo) / (1.0 - lo)
    assert np.all((u >= -1e-6) & (u <= 1.0)), (u.min(), u.max())
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    if E <= 1.0:
        assert len(e) == 0  # the electron's share never reaches the 1 MeV cut
    else:
        assert _binomial_ok(len(e), N, 1.0 - 1.0 / E), (len(e), N * (1.0 - 1.0 / E))
        assert np.all((e["E"] >= 1.0) & (e["E"] < E))
        assert np.all(e["numIALeft"] == -1.0) and np.all(e["rngCtr"] == 0)
    # every photon interacted: the electrons' sub-cut shares, the killed photons,
    # the buffered tracks and the rounding ledger (binary32 energies) add up to the
    # injected energy
    total = o.tally(oracle.T_DEP_CUT).sum() + g["E"].sum() + e["E"].sum() + o.tally(oracle.T_ROUND).sum()
    assert abs(total - N * E) <= 1e-12 * N * E
    return o


def _u64(r):
    return (int(r) + 0.5) * 2.0**-32


def _u32(r):
    return np.float32(np.float32(int(r) >> 9) + np.float32(0.5)) * np.float32(2.0**-23)


def compton_hand_trace(L, precision, n_tracks=32, E=0.5, seed=1):
    """One Compton step per track, recomputed here from the Philox words."""
    survivors = kills = 0
    for tid in range(n_tracks):
        o = oracle.Oracle(oracle.DENSE, precision, 64, [seed], L=L)
        p = workloads.primaries(1, workloads.GAMMA, E, num_ia_left=1e-3, first_id=tid)
        assert o.inject(p) == 0
        rc, n = o.step()
        assert rc == 0
        a = oracle.philox([0, 0, 0, 0], [seed, tid])
        b = oracle.philox([0, 1, 0, 0], [seed, tid])
        if precision == oracle.FP64:
            T0 = _u64(a[3]) * E
            Ep = E - T0
            T = E - Ep
            survive = not (Ep < 0.1)
            nl_want = -math.log(_u64(b[0]))
            nl_tol = 1e-15 * nl_want
        else:
            Ef = np.float32(E)
            T0 = _u32(a[3]) * Ef
            Ep = np.float32(Ef - T0)
            T = np.float32(Ef - Ep)
            survive = not (Ep < np.float32(0.1))
            nl_want = float(-np.log(np.float64(_u32(b[0]))))
            nl_tol = 4 * 2.0**-23 * max(nl_want, 1.0)
        assert float(T) + float(Ep) == E  # the complement is exact
        cut = o.tally(oracle.T_DEP_CUT)
        g, _ = o.dump(workloads.GAMMA)
        assert len(o.dump(workloads.ELECTRON)[0]) == 0  # T < 1 MeV: deposited at once
        if survive:
            survivors += 1
            assert list(n) == [0, 0, 1]
            assert g[0]["E"] == float(Ep), (tid, g[0]["E"], Ep)
            assert cut[0] == float(T) and np.count_nonzero(cut) == 1
            assert abs(g[0]["numIALeft"] - nl_want) <= nl_tol, (tid, g[0]["numIALeft"], nl_want)
            assert g[0]["rngCtr"] == 1 and g[0]["volume"] == 0
            assert list(g[0]["dir"]) == [0.0, 0.0, 1.0]
            s = np.float32(1e-3) * np.float32(11.2) if precision else 1e-3 * 11.2
            assert g[0]["pos"][2] == float(s)
        else:
            kills += 1
            assert list(n) == [0, 0, 0]
            assert cut[0] == E  # T + E' booked as local deposits: all of E
    assert survivors > 0 and kills > 0  # both branches traced
    return survivors, kills


def resample_after_compton(L, precision):
    o = _one_step(L, workloads.GAMMA, 0.5, 1e-9, precision)
    g, _ = o.dump(workloads.GAMMA)
    assert len(g) > 0.7 * N
    assert np.all(g["numIALeft"] > 0.0)
    assert stats.kstest(g["numIALeft"], "expon").pvalue > 1e-3


def resample_after_brem(L, precision):
    o = _one_step(L, workloads.ELECTRON, 100.0, 1e-9, precision)
    e, _ = o.dump(workloads.ELECTRON)
    g, _ = o.dump(workloads.GAMMA)
    assert len(g) == N  # every electron radiated at its first step
    assert len(e) > 0.9 * N
    assert np.all(e["numIALeft"] > 0.0)
    assert stats.kstest(e["numIALeft"], "expon").pvalue > 1e-3


def ledger_relations(o):
    """The integer identities of the particle ledger of one oracle context."""
    g = o.ledger()
    E, P, G = workloads.ELECTRON, workloads.POSITRON, workloads.GAMMA
    deaths = [g["escaped"][E] + g["cut"][E],
              g["escaped"][P] + g["cut"][P] + g["annihilated"],
              g["escaped"][G] + g["cut"][G] + g["absorbed"]]
    for t in range(3):
        assert g["primaries"][t] + g["created"][t] == deaths[t] + g["inflight"][t], (t, g)
    assert g["cut"][P] == 0  # a stopped positron annihilates
    assert g["created"][E] == g["n_pair"] + g["n_compton"], g
    assert g["created"][P] == g["n_pair"], g
    assert g["created"][G] == g["n_brem"] + 2 * g["n_annihilation"], g
    assert g["annihilated"] == g["n_annihilation"], g
    assert g["absorbed"] == g["n_pair"], g
    # charge: pair production is neutral, a Compton step ejects one electron
    assert g["created"][P] - g["created"][E] == -g["n_compton"], g
    return g


def ledger_mixed_shower(L, precision, scheme=oracle.DENSE, every_iteration=True):
    """Electrons, positrons and photons of several energies (sub-cut ones too):
    the ledger holds after injection and after every iteration."""
    p = np.concatenate([
        workloads.primaries(6, workloads.ELECTRON, 2000.0),
        workloads.primaries(4, workloads.POSITRON, 500.0, first_id=6),
        workloads.primaries(4, workloads.GAMMA, 300.0, first_id=10),
        workloads.primaries(3, workloads.GAMMA, 0.05, first_id=14),     # below the photon cut
        workloads.primaries(3, workloads.POSITRON, 0.5, first_id=17),   # below the e+- cut: annihilates
        workloads.primaries(3, workloads.ELECTRON, 0.7, first_id=20),   # below the e+- cut
    ])
    o = oracle.Oracle(scheme, precision, 1 << 16, [5], L=L)
    assert o.inject(p) == 0
    g = ledger_relations(o)
    assert g["primaries"] == [9, 7, 7]
    while True:
        rc, n = o.step()
        assert rc == 0
        if every_iteration or n.sum() == 0:
            g = ledger_relations(o)
        if n.sum() == 0:
            break
    assert g["n_compton"] > 0 and g["n_pair"] > 0 and g["n_brem"] > 0 and g["n_annihilation"] > 0
    st = o.stats()
    for t in range(3):  # a source step either survives (and is written again) or ends the track
        assert g["survivors"][t] <= st["track_steps"][t] and g["survivors"][t] <= g["outputs"][t]
    return o, g, st


def divergence_groups(L, scheme=oracle.DENSE):
    """The lane-weighted divergence count after one iteration of 100 positrons at
    the front face along +z: the first 40 and the ten at 64..73 have 1.01 MeV
    (range 0.80 mm, inside the first absorber: killed, two annihilation photons
    buffered), the rest 10 MeV with a forced interaction length of 100 X0 (a 2.3
    mm geometry step: survive, nothing created).  Group 0 holds 40 of the first
    kind and 24 of the second (24 differ from the group's most common outcome),
    group 1 ten and 26 (10 differ): 34.  Groups of 128 would give 50, of 32 give
    18; counting the most common outcome itself would give 66."""
    p = workloads.primaries(100, workloads.POSITRON, 10.0, num_ia_left=100.0)
    short = list(range(40)) + list(range(64, 74))
    p["E"][short] = 1.01
    p["numIALeft"][short] = -1.0
    o = oracle.Oracle(scheme, oracle.FP64, 1 << 10, [1], L=L)
    assert o.inject(p) == 0
    rc, nxt = o.step()
    assert rc == 0
    led = o.ledger()
    o.close()
    assert led["survivors"][1] == 50 and list(nxt) == [0, 50, 100], (led["survivors"], nxt)
    assert led["off_mode"] == 34, led["off_mode"]
