"""Seeded synthetic inputs shared by the oracle and the HIP library.

This module holds the workload definitions only: which primaries enter the
calorimeter (type, energy, position, direction, forced interaction length,
track id, event) and the per-event seeds.  It contains none of the transport
arithmetic.  Both the oracle (``oracle/``) and the GPU library consume the
arrays produced here through the same binary record layout (``PRIMARY_DTYPE``,
80 bytes, identical to ``adept_primary`` in ``include/adept.h``).

Workloads (energies in MeV, lengths in mm):

* ``showers_100e_1gev``: one event, 100 electrons of 1000 MeV at the origin along +z, seed 1.
* ``showers_10ke_10gev``: one event, 10^4 electrons of 10^4 MeV, seed 1.
* ``showers_100ke_10gev``: one event, 10^5 electrons of 10^4 MeV, seed 7.
* ``uneven_512_events``: 512 events of uneven size.  A ``numpy.random.Generator(PCG64(3))``
  draws the per-event primary counts ``integers(1, 2001, 512)``; then, event by
  event, ``random(N_e)`` picks the type (u < 0.7 electron, u < 0.9 photon, else
  positron) and a second ``random(N_e)`` the energy ``E = 100 * 1000**u``.
  Event ``e`` has seed ``e + 1``.
* ``segmented_1000_events``: 1000 events x 1000 electrons of 10^4 MeV, event ``e`` seed ``e + 1``.

Every primary starts at (0, 0, 0) moving along +z with its interaction length
unset (``numIALeft = -1``: sampled at its first step), and its track id is its
index within its event.
"""
import numpy as np

ELECTRON, POSITRON, GAMMA = 0, 1, 2

PRIMARY_DTYPE = np.dtype(
    [
        ("event", "<u4"),
        ("type", "<i4"),
        ("E", "<f8"),
        ("pos", "<f8", (3,)),
        ("dir", "<f8", (3,)),
        ("numIALeft", "<f8"),
        ("trackId", "<u8"),
    ],
    align=True,
)
assert PRIMARY_DTYPE.itemsize == 80


def primaries(n, ptype=ELECTRON, energy=1000.0, event=0, pos=(0.0, 0.0, 0.0),
              direction=(0.0, 0.0, 1.0), num_ia_left=-1.0, first_id=0):
    """``n`` identical primaries of one event with consecutive track ids."""
    p = np.zeros(n, dtype=PRIMARY_DTYPE)
    p["event"] = event
    p["type"] = ptype
    p["E"] = energy
    p["pos"] = pos
    p["dir"] = direction
    p["numIALeft"] = num_ia_left
    p["trackId"] = np.arange(first_id, first_id + n, dtype=np.uint64)
    return p


class Workload:
    """Primaries, per-event seeds and the nominal scheme of one configuration."""

    def __init__(self, name, prims, seeds, description):
        self.name = name
        self.primaries = prims
        self.seeds = np.asarray(seeds, dtype=np.uint32)
        self.description = description

    @property
    def n_events(self):
        return len(self.seeds)

    def event_energy(self):
        """Per-event total primary kinetic energy (MeV), host doubles."""
        out = np.zeros(self.n_events)
        np.add.at(out, self.primaries["event"], self.primaries["E"])
        return out

    def subset(self, n_primaries):
        """The first ``n_primaries`` primaries (for bounded samples)."""
        return Workload(self.name + f"[:{n_primaries}]", self.primaries[:n_primaries].copy(),
                        self.seeds, self.description + f" (first {n_primaries} primaries)")


def showers_100e_1gev():
    return Workload("showers_100e_1gev", primaries(100, ELECTRON, 1000.0), [1],
                    "1 event x 100 e- at 1 GeV, seed 1")


def showers_10ke_10gev(n=10_000):
    return Workload("showers_10ke_10gev", primaries(n, ELECTRON, 10_000.0), [1],
                    f"1 event x {n} e- at 10 GeV, seed 1")


def showers_100ke_10gev(n=100_000):
    return Workload("showers_100ke_10gev", primaries(n, ELECTRON, 10_000.0), [7],
                    f"1 event x {n} e- at 10 GeV, seed 7")


def uneven_512_events(n_events=512, max_per_event=2000):
    g = np.random.Generator(np.random.PCG64(3))
    counts = g.integers(1, max_per_event + 1, n_events)
    parts = []
    for e in range(n_events):
        n = int(counts[e])
        ut = g.random(n)
        ue = g.random(n)
        p = primaries(n, ELECTRON, 0.0, event=e)
        p["type"] = np.where(ut < 0.7, ELECTRON, np.where(ut < 0.9, GAMMA, POSITRON))
        p["E"] = 100.0 * np.power(1000.0, ue)
        parts.append(p)
    prims = np.concatenate(parts)
    return Workload("uneven_512_events", prims, np.arange(1, n_events + 1),
                    f"{n_events} events x U{{1..{max_per_event}}} primaries, 70/20/10 e-/gamma/e+, "
                    "E log-uniform in [100 MeV, 100 GeV], seeds e+1")


def segmented_1000_events(n_events=1000, per_event=1000):
    parts = [primaries(per_event, ELECTRON, 10_000.0, event=e) for e in range(n_events)]
    return Workload("segmented_1000_events", np.concatenate(parts), np.arange(1, n_events + 1),
                    f"{n_events} events x {per_event} e- at 10 GeV, seeds e+1")


def by_name(name, **kw):
    return {"showers_100e_1gev": showers_100e_1gev, "showers_10ke_10gev": showers_10ke_10gev, "showers_100ke_10gev": showers_100ke_10gev, "uneven_512_events": uneven_512_events, "segmented_1000_events": segmented_1000_events}[name](**kw)
