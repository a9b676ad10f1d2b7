#!/usr/bin/env python3
"""Track-steps/s of the transport iteration on one MI355X.

One benchmark step = one whole run of the workload: inject every primary (already
resident in device memory) and iterate until no track is left.  The headline
workload is 10^5 electrons of 10 GeV in one event (seed 7) on the dense double
buffer with the SoA layout in mixed precision; the same workload is timed
alongside in FP64 (dense SoA, and the sparse single buffer with the AoS layout,
the paper's baseline structure), and the per-layer deposit difference between the
mixed and the FP64 runs is stated.

Prints one JSON line (rank 0).  Only one GPU is used: --gpus above 1 exits.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, AMD's published figure
KERNEL_SOURCES = ["kernels.hpp", "layout.hpp", "model.hpp", "inst_dense_mixed.hip"]
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_step_100ke_10gev_dense_soa_mixed_pmc.md")
BATCHED_TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_step_512_uneven_events_dense_aosoa64_mixed_pmc.md")


def progress(msg):
    """One line on stderr when a section of the benchmark ends."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the step kernel's sources and of the build script (its compiler flags)."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2302_08252_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    with open(os.path.join(ROOT, "paper_2302_08252_amd", "build.py"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def profile_fields(path=TRAFFIC_SUMMARY):
    """The '- key: value' lines of a committed rocprofv3 --pmc summary (by default the
    headline kernel's), or {} if the kernel sources changed since it was taken."""
    try:
        text = open(path).read()
    except OSError:
        return {}
    fields = dict(line.split(":", 1) for line in text.splitlines() if line.startswith("- ") and ":" in line)
    fields = {k[2:].strip(): v.strip() for k, v in fields.items()}
    return fields if fields.get("kernel source hash") == kernel_source_hash() else {}


def measured_traffic(path=TRAFFIC_SUMMARY):
    """HBM bytes per step-kernel launch (FETCH_SIZE + WRITE_SIZE, scaled by the same
    counters on a plain copy of known size), or None."""
    try:
        return float(profile_fields(path)["scaled HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def measured_lane_use():
    """Active lanes per VALU instruction of the headline kernel (of 64), or None."""
    try:
        return float(profile_fields()["active lanes per VALU instruction"].split()[0])
    except (KeyError, ValueError, IndexError):
        return None


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--primaries", type=int, default=100_000)
    ap.add_argument("--capacity-log2", type=int, default=25)
    ap.add_argument("--block", type=int, default=1024)
    ap.add_argument("--graph-iters", type=int, default=32)
    ap.add_argument("--grid", type=int, default=0, help="resident blocks of the step kernel (0: library default)")
    ap.add_argument("--wave-tiles", type=int, default=0, choices=[0, 1],
                    help="compaction tile of the step kernel: 0 = the block, 1 = the wavefront")
    ap.add_argument("--fp64-steps", type=int, default=2, help="timed runs of each FP64 comparison path (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=9600, help="primaries of the workload run by the oracle")
    ap.add_argument("--headline-only", action="store_true", help="only the headline path (for profilers)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched uneven-events section")
    ap.add_argument("--batched-profile", action="store_true",
                    help="only the 512 uneven events, twice, with the tuned layout fixed (AoSoA-64, block 1024, "
                         "graphs of 16): the command behind the batched kernel-trace summary")
    ap.add_argument("--per-event-sample", type=int, default=32, help="events timed one launch sequence each")
    ap.add_argument("--batched-capacity-log2", type=int, default=28,
                    help="slots per particle type of the 512-event runs (admission keeps the tracks below 0.8 of it)")
    ap.add_argument("--no-segmented", action="store_true", help="skip 10^6 e- in 1000 events with 500k cells")
    ap.add_argument("--no-layout-study", action="store_true",
                    help="skip showers_10ke_10gev in the paper's four layouts (timings and access counts)")
    ap.add_argument("--flip-sample", type=int, default=512,
                    help="primaries whose showers the oracle runs in both precision policies (flip count)")
    ap.add_argument("--line-check", choices=["sparse-aos", "dense-aos", "dense-soa"], default=None,
                    help="showers_10ke_10gev, FP64: injection + 20 iterations uninstrumented (the dispatches a "
                         "counter run measures), then the same instrumented, printing the cache-line model of "
                         "the bytes moved")
    ap.add_argument("--segmented-profile", action="store_true",
                    help="only the 1000-event cell workload, mixed, twice (for profilers)")
    ap.add_argument("--layout-pair", action="store_true",
                    help="the headline workload once in SoA and once in AoSoA-64 (graph replay), for counter runs")
    ap.add_argument("--pmc-summary", nargs="+", default=None, metavar="CSV",
                    help="sum rocprofv3 counter CSVs per kernel and counter (no GPU use)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device to device (a plain copy of known size for scaling counters)")
    return ap.parse_args()


def algorithmic_bytes(st, scheme, precision):
    """Bytes the method must move for the steps recorded in st (access contract of
    the track buffers; dense: 13 fields read per source, parentId per survivor,
    every output written whole; sparse adds the u32 slot-list and ring traffic)."""
    R = 68 if precision == 1 else 88
    W = 76 if precision == 1 else 96
    src = sum(st["track_steps"])
    surv = sum(st["survivors"])
    outs = sum(st["outputs"])
    if scheme == 1:
        return src * R + surv * 8 + outs * W
    charged_w = 52 if precision == 1 else 72
    gamma_w = 40 if precision == 1 else 48
    surv_w = (st["survivors"][0] + st["survivors"][1]) * charged_w + st["survivors"][2] * gamma_w
    created = outs - surv
    killed = src - surv
    return src * (R + 4) + surv_w + outs * 4 + created * (W + 4) + killed * 4


def kernel_roofline(st, scheme, precision):
    """Step-kernel roofline of one timed run: its algorithmic bytes over the summed
    HIP-event durations of its step-kernel launches."""
    alg = algorithmic_bytes(st, scheme, precision)
    ks = st["step_kernel_ms"] / 1e3
    gbps = alg / ks / 1e9 if ks > 0 else None
    return {"bound": "hbm", "kernel": "k_step", "achieved": gbps, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": gbps / PEAK_HBM_GBS if gbps else None, "algorithmic_bytes": alg,
            "step_launches": st["step_launches"], "avg_step_kernel_ms": st["step_kernel_ms"] / max(st["step_launches"], 1)}


def time_path(ad, torch, wl, dev_prims, scheme, mapping, precision, C, args, steps, warmup, timing):
    sim = ad.Sim(scheme, mapping, precision, C, 64, seeds=wl.seeds,
                 launch={"block": args.block, "grid": args.grid, "graph_iters": args.graph_iters,
                         "wave_tiles": args.wave_tiles})
    n = len(wl.primaries)
    for _ in range(max(warmup, 1)):  # the warm-up run also counts the lane-weighted divergence
        sim.reset()
        ad.adept_inject_device(sim.ctx, dev_prims.data_ptr(), n)
        sim.run()
    w = sim.stats()
    off_mode = w["off_mode"] / max(sum(w["track_steps"]), 1)
    ad.adept_set_divergence_count(sim.ctx, False)  # timed runs leave the diagnostic out (about 1%)
    total = 0.0
    runs = []
    per_run = None
    for k in range(steps):
        sim.reset()
        ad.adept_set_timing(sim.ctx, timing)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ad.adept_inject_device(sim.ctx, dev_prims.data_ptr(), n)
        iters = sim.run()
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t0)
        total += runs[-1]
        st = sim.stats()
        if per_run is None:
            per_run = dict(st, iterations=iters)
            per_run["step_kernel_ms"] = 0.0
            per_run["step_launches"] = 0
        else:
            assert st["track_steps"] == per_run["track_steps"], "runs must be identical"
        per_run["step_kernel_ms"] += st["step_kernel_ms"]
        per_run["step_launches"] += st["step_launches"]
    phase = ad.adept_phase_clocks(sim.ctx)
    layer = sim.tally(ad.T_LAYER)
    ein = sim.tally(ad.T_EIN)
    tot = (sim.tally(ad.T_DEP_CONT).sum() + sim.tally(ad.T_DEP_CUT).sum() + sim.tally(ad.T_ESCAPED).sum()
           + sim.tally(ad.T_ROUND).sum())
    closure = abs(ein.sum() - tot) / ein.sum()
    closure_no_round = abs(ein.sum() - (tot - sim.tally(ad.T_ROUND).sum())) / ein.sum()
    sim.close()
    ts = sum(per_run["track_steps"])
    mean = total / steps
    cv = (sum((r - mean) ** 2 for r in runs) / steps) ** 0.5 / mean if steps > 1 else 0.0
    return {
        "seconds": total, "ms_per_step": 1e3 * mean, "ms_min": 1e3 * min(runs), "cv": cv, "track_steps_per_run": ts,
        "track_steps_per_s": ts * steps / total, "primaries_per_s": n * steps / total,
        "iterations": per_run["iterations"], "stats": per_run, "layer": layer, "closure": closure, "phase": phase,
        "lanes_off_mode_fraction": off_mode,
        "closure_without_rounding_ledger": closure_no_round,
    }


# Worker processes of the CPU baseline: the host cores this process may use, capped at
# 16, the CPU share that goes with one GPU on the benchmark boxes (their affinity
# mask may show more cores than that share).
CPU_SHARE = 16


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, sample, precision, repeats=3, flip_sample=64):
    """The oracle, unchanged, on a bounded sample of the workload: disjoint chunks of
    primaries in worker processes (track histories do not depend on batching), best of
    `repeats` timed runs, plus a one-core rate.  Runs before the process touches the
    GPU, so the forked workers inherit no HIP runtime state.  Also (untimed) the
    mixed-precision flip count on `flip_sample` primaries: each primary's shower run by
    the oracle under both precision policies, a shower counted as flipped when its
    discrete history (per-type steps, creations, deaths and interactions) differs."""
    import multiprocessing as mp

    import oracle

    oracle.build()
    avail = len(os.sched_getaffinity(0))
    cores = max(1, min(CPU_SHARE, avail))
    prims = wl.primaries[:sample]
    chunks = [prims[i::cores] for i in range(cores)]
    args = [(c, wl.seeds, precision) for c in chunks if len(c)]
    times = []
    with mp.get_context("fork").Pool(len(args)) as pool:
        for _ in range(repeats):
            t0 = time.perf_counter()
            steps = pool.map(_oracle_chunk, args)
            times.append(time.perf_counter() - t0)
        flips = pool.map(_oracle_flip, [(p, wl.seeds) for p in wl.primaries[:flip_sample]])
    dt = min(times)
    # one core on a twentieth of the sample, for the per-core rate
    t1 = time.perf_counter()
    steps1 = _oracle_chunk((prims[:max(1, sample // 20)], wl.seeds, precision))
    dt1 = time.perf_counter() - t1
    return {"value": sum(steps) / dt, "unit": "track-steps/s", "cores": len(args), "kind": "oracle",
            "cpu_model": cpu_model(), "cores_available": avail,
            "cores_note": f"worker processes = min(affinity {avail}, {CPU_SHARE}): {CPU_SHARE} host cores is the "
                          "CPU share of one GPU on the benchmark boxes",
            "sample": f"first {sample} primaries of the workload, dense double buffer, "
                      f"{'mixed' if precision else 'FP64'} policy, {sum(steps)} track-steps, best of {repeats} "
                      f"runs: {dt:.2f} s wall (runs {', '.join(f'{t:.2f}' for t in times)} s)",
            "single_core": {"value": steps1 / dt1, "sample": f"first {max(1, sample // 20)} primaries, "
                                                              f"{steps1} track-steps in {dt1:.2f} s"},
            "mixed_precision_flips": {"primaries_compared": len(flips), "showers_with_a_flip": int(sum(flips)),
                                      "method": "each primary's shower run alone by the oracle in FP64 and mixed; "
                                                "flipped if any discrete count differs"}}


def _oracle_chunk(a):
    import oracle
    import workloads

    prims, seeds, precision = a
    wl = workloads.Workload("chunk", prims, seeds, "")
    o, rc, _ = oracle.run_workload(wl, oracle.DENSE, precision, 1 << 24)
    assert rc == 0
    return sum(o.stats()["track_steps"])


def _oracle_flip(a):
    """1 if one primary's shower differs in any discrete count between the policies."""
    import numpy as np

    import oracle
    import workloads

    prim, seeds = a
    hist = []
    for precision in (oracle.FP64, oracle.MIXED):
        wl = workloads.Workload("one", np.array([prim]), seeds, "")
        o, rc, it = oracle.run_workload(wl, oracle.DENSE, precision, 1 << 22)
        assert rc == 0
        g = o.ledger()
        hist.append((it, tuple(o.stats()["track_steps"]), tuple(g["created"]), tuple(g["escaped"]),
                     tuple(g["cut"]), g["n_brem"], g["n_pair"], g["n_compton"], g["n_annihilation"]))
    return int(hist[0] != hist[1])


def kappa_per_gev():
    path = os.path.join(ROOT, "tests", "golden", "kappa_per_gev.txt")
    line = [l for l in open(path) if not l.startswith("#")][0]
    return [float(x) for x in line.split()]


def run_once(ad, torch, sim, prims=None, dev=None):
    """Time one run (primaries staged beforehand: admission uploads them at the
    first call, which max_iter=0 triggers outside the timed region)."""
    sim.reset()
    if dev is not None:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ad.adept_inject_device(sim.ctx, dev.data_ptr(), len(prims))
    else:
        sim.inject(prims)
        sim.run(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
    it = sim.run()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, it, sim.stats()


def batched_section(ad, torch, np, workloads, args):
    """512 uneven events (uneven_512_events): layout and launch picked by the autotuner on a
    64-event sample, events admitted by the capacity rule, per-event tallies.  The track
    buffers get most of the HBM (2^28 slots per type by default, 122 GB in the mixed
    record): admission then takes every event at once and the run needs 251 iterations
    instead of 1937 at 2^24, with fewer, larger launches."""
    wl = workloads.uneven_512_events()
    kappa = kappa_per_gev()
    # the largest capacity up to the requested one whose mixed AoSoA-64 buffers (six
    # of 76 bytes per slot) fit in 90 % of the free device memory
    free, _ = torch.cuda.mem_get_info()
    lg = args.batched_capacity_log2
    while lg > 20 and 6 * 76 * (1 << lg) > 0.9 * free:
        lg -= 1
    C = 1 << lg
    if lg != args.batched_capacity_log2:
        progress(f"batched: 2^{args.batched_capacity_log2} slots per type do not fit, using 2^{lg}")
    cands = [(1, 0, 1), (1, 1, 1), (1, 2, 16), (1, 2, 64), (1, 2, 256)]
    sample = wl.primaries[wl.primaries["event"] < 64]  # ~64k primaries: peak below 1e7 photons < 2^24
    layout, launch, _ = ad.adept_autotune_layout(ad.MIXED, 1 << 24, cands, wl.seeds[:64], sample)
    progress(f"batched: autotuned layout {layout}, launch {launch}")
    out = {"workload": wl.description, "capacity_per_type": C, "admission": {"alpha": 0.8, "kappa_per_GeV": kappa},
           "autotuned": {"layout": {"scheme": "dense" if layout[0] else "sparse",
                                    "mapping": ["AoS", "SoA", "AoSoA"][layout[1]], "lanes": layout[2]},
                         "launch": launch, "tuning_sample": "events 0-63, capacity 2^24"}}
    sim = ad.Sim(layout[0], layout[1], ad.MIXED, C, layout[2], seeds=wl.seeds, admission=(0.8, kappa), launch=launch)
    _, _, st_w = run_once(ad, torch, sim, wl.primaries)  # warm-up, with the lane-weighted divergence count
    progress("batched: warm-up run done")
    ad.adept_set_divergence_count(sim.ctx, False)
    dt, it, st = run_once(ad, torch, sim, wl.primaries)
    ts = sum(st["track_steps"])
    lay_m = sim.tally(ad.T_LAYER).reshape(len(wl.seeds), 50).sum(axis=0)
    # the same run in timed mode (iterations launched one by one, HIP events around
    # every step kernel): the step kernel's own bandwidth
    ad.adept_set_timing(sim.ctx, True)
    _, _, st_t = run_once(ad, torch, sim, wl.primaries)
    ad.adept_set_timing(sim.ctx, False)
    sim.close()
    assert st_t["track_steps"] == st["track_steps"]
    out["mixed"] = {"seconds": dt, "track_steps": ts, "track_steps_per_s": ts / dt, "iterations": it,
                    "algorithmic_GBps_run": algorithmic_bytes(st, layout[0], 1) / dt / 1e9,
                    "primaries_per_s": len(wl.primaries) / dt,
                    "divergent_wave_fraction": st["waves_divergent"] / max(st["waves"], 1),
                    "lanes_off_mode_fraction": st_w["off_mode"] / max(sum(st_w["track_steps"]), 1),
                    "roofline": kernel_roofline(st_t, layout[0], 1)}
    # the layout, tile shape and capacity the counter summary was taken with
    if (layout == (1, 2, 64) and launch.get("block") == 1024 and not launch.get("wave_tiles")
            and profile_fields(BATCHED_TRAFFIC_SUMMARY).get("capacity per type") == str(C)):
        out["mixed"]["roofline"]["traffic"] = measured_traffic(BATCHED_TRAFFIC_SUMMARY)
    # the FP64 sparse single buffer (the paper's baseline structure), same admission
    sp = ad.Sim(0, 0, ad.FP64, C, 1, seeds=wl.seeds, admission=(0.8, kappa), launch=launch)
    dt2, it2, st2 = run_once(ad, torch, sp, wl.primaries)
    progress("batched: FP64 sparse AoS run done")
    lay_f = sp.tally(ad.T_LAYER).reshape(len(wl.seeds), 50).sum(axis=0)
    sp.close()
    ts2 = sum(st2["track_steps"])
    out["fp64_sparse_aos"] = {"seconds": dt2, "track_steps_per_s": ts2 / dt2,
                              "algorithmic_GBps_run": algorithmic_bytes(st2, 0, 0) / dt2 / 1e9,
                              "divergent_wave_fraction": st2["waves_divergent"] / max(st2["waves"], 1),
                              "lanes_off_mode_fraction": st2["off_mode"] / max(sum(st2["track_steps"]), 1)}
    out["speedup_vs_fp64_sparse_aos"] = dt2 / dt
    rel = np.abs(lay_m - lay_f) / lay_f
    out["edep_per_layer_rel_error_mixed_vs_fp64"] = {"max": float(rel.max()),
                                                     "total": float(abs(lay_m.sum() - lay_f.sum()) / lay_f.sum())}
    # one launch sequence per event, on a sample of events
    k = args.per_event_sample
    pe = ad.Sim(layout[0], layout[1], ad.MIXED, C, layout[2], seeds=wl.seeds, launch=launch)
    tot_t = tot_s = 0.0
    for e in range(k):
        d, _, s = run_once(ad, torch, pe, wl.primaries[wl.primaries["event"] == e])
        tot_t += d
        tot_s += sum(s["track_steps"])
    pe.close()
    out["one_launch_sequence_per_event"] = {"events_sampled": k, "track_steps_per_s": tot_s / tot_t}
    out["batched_speedup_vs_per_event"] = (ts / dt) / (tot_s / tot_t)
    return out


def batched_profile(ad, torch, np, workloads, args):
    wl = workloads.uneven_512_events()
    sim = ad.Sim(ad.DENSE_DOUBLE, ad.MAP_AOSOA, ad.MIXED, 1 << args.batched_capacity_log2, 64, seeds=wl.seeds,
                 admission=(0.8, kappa_per_gev()), launch={"block": 1024, "graph_iters": 16})
    runs = []
    for _ in range(2):
        dt, it, st = run_once(ad, torch, sim, wl.primaries)
        runs.append({"seconds": dt, "iterations": it, "track_steps_per_s": sum(st["track_steps"]) / dt})
    sim.close()
    return {"workload": wl.description, "layout": "dense AoSoA-64, mixed", "runs": runs}


def segmented_profile(ad, torch, np, workloads):
    """The mixed run of the segmented section, twice (graph replay), for counter runs."""
    wl = workloads.segmented_1000_events()
    sim = ad.Sim(ad.DENSE_DOUBLE, ad.MAP_SOA, ad.MIXED, 1 << 28, 64, seeds=wl.seeds, scoring=(100, 100, 4.0),
                 admission=(0.8, kappa_per_gev()), launch={"block": 1024, "graph_iters": 32})
    ad.adept_set_divergence_count(sim.ctx, False)
    runs = []
    for _ in range(2):
        dt, it, st = run_once(ad, torch, sim, wl.primaries)
        runs.append({"seconds": dt, "iterations": it, "track_steps_per_s": sum(st["track_steps"]) / dt,
                     "algorithmic_bytes": algorithmic_bytes(st, 1, 1)})
    sim.close()
    return {"workload": wl.description + ", 100x100 cells of 4 mm per layer", "layout": "dense SoA, mixed",
            "runs": runs}


LINE_LAYOUTS = {"sparse-aos": (0, 0, 1), "dense-aos": (1, 0, 1), "dense-soa": (1, 1, 1)}


def line_model(ad, np, sim, scheme):
    """Bytes the cache-line model says move: every 128-byte line of every track
    buffer moves once per access of its most accessed 4-byte word (heatmap of an
    instrumented run); bytes used = 4 x the word counts."""
    used = moved = 0
    for t in range(3):
        for b in range(2 if scheme else 1):
            words = sim.access_counts(t, b, heat=True)[2].astype(np.uint64)
            words = np.concatenate([words, np.zeros(-len(words) % 32, dtype=np.uint64)]).reshape(-1, 32)
            used += 4 * int(words.sum())
            moved += 128 * int(words.max(axis=1).sum())
    return used, moved


def line_check(ad, torch, np, workloads, which):
    """showers_10ke_10gev in FP64: injection and 20 iterations without instrumentation
    (k_step / k_inject launches with INSTR = false: what a counter run sums), then the
    same window instrumented for the cache-line model of the track-buffer bytes."""
    wl = workloads.showers_10ke_10gev()
    s, m, n = LINE_LAYOUTS[which]
    C = 1 << 22
    sim = ad.Sim(s, m, ad.FP64, C, n, seeds=wl.seeds, launch={"block": 1024, "graph_iters": 20})
    sim.inject(wl.primaries)
    assert sim.run(20) == 20
    st = sim.stats()
    sim.close()
    sim = ad.Sim(s, m, ad.FP64, C, n, seeds=wl.seeds, instrumented=20, launch={"block": 1024, "graph_iters": 20})
    sim.inject(wl.primaries)
    assert sim.run(20) == 20
    used, moved = line_model(ad, np, sim, s)
    sim.close()
    return {"workload": wl.description, "layout": which, "precision": "FP64", "iterations": 20,
            "track_steps": sum(st["track_steps"]), "line_model_bytes_moved": moved, "bytes_used": used,
            "algorithmic_step_bytes": algorithmic_bytes(st, s, 0)}


def layout_pair(ad, torch, wl, args):
    """The headline workload (mixed, dense) once in SoA and once in AoSoA-64, graph
    replay, for counter runs that compare the two layouts (k_step<1, 1, ...> is the
    SoA kernel, k_step<1, 2, ...> the AoSoA one)."""
    out = []
    for mapping, lanes, name in ((ad.MAP_SOA, 1, "SoA"), (ad.MAP_AOSOA, 64, "AoSoA-64")):
        sim = ad.Sim(ad.DENSE_DOUBLE, mapping, ad.MIXED, 1 << args.capacity_log2, lanes, seeds=wl.seeds,
                     launch={"block": args.block, "graph_iters": args.graph_iters})
        ad.adept_set_divergence_count(sim.ctx, False)
        dt, it, st = run_once(ad, torch, sim, wl.primaries)
        out.append({"layout": name, "seconds": dt, "iterations": it, "track_steps_per_s": sum(st["track_steps"]) / dt})
        sim.close()
        del sim
    return out


def kernel_base_name(name):
    """A kernel's name without its trailing argument list."""
    if name.endswith(")"):
        depth = 0
        for i in range(len(name) - 1, -1, -1):
            depth += {")": 1, "(": -1}.get(name[i], 0)
            if depth == 0:
                return name[:i]
    return name


def pmc_summary(paths):
    """Per (kernel, counter) sums over the dispatches of rocprofv3 counter CSVs."""
    import csv
    out = {}
    for path in paths:
        for r in csv.DictReader(open(path)):
            key = f"{kernel_base_name(r['Kernel_Name'])} | {r['Counter_Name']}"
            e = out.setdefault(key, {"sum": 0.0, "dispatches": 0})
            e["sum"] += float(r["Counter_Value"])
            e["dispatches"] += 1
    return out


def segmented_section(ad, torch, np, workloads):
    """10^6 e- of 10 GeV in 1000 events with 100x100 cells per layer, mixed, dense SoA,
    admission: wall-clock rate, step-kernel roofline (timed run), and the per-layer
    and per-cell deposit error against the same workload in FP64 (the FP64 GPU path
    is bit-exact with the FP64 oracle per track)."""
    wl = workloads.segmented_1000_events()
    C = 1 << 28
    kappa = kappa_per_gev()
    res = {"workload": wl.description + ", 100x100 cells of 4 mm per layer", "capacity_per_type": C}
    tallies = {}
    for prec in (ad.MIXED, ad.FP64):
        sim = ad.Sim(ad.DENSE_DOUBLE, ad.MAP_SOA, prec, C, 64, seeds=wl.seeds, scoring=(100, 100, 4.0),
                     admission=(0.8, kappa), launch={"block": 1024, "graph_iters": 32})
        dt, it, st = run_once(ad, torch, sim, wl.primaries)
        progress(f"segmented: {'mixed' if prec == ad.MIXED else 'FP64'} run done")
        tallies[prec] = (sim.tally(ad.T_LAYER).reshape(len(wl.seeds), 50).sum(axis=0), sim.tally(ad.T_CELLS))
        rec = {"seconds": dt, "track_steps_per_s": sum(st["track_steps"]) / dt, "iterations": it,
               "divergent_wave_fraction": st["waves_divergent"] / max(st["waves"], 1),
               "lanes_off_mode_fraction": st["off_mode"] / max(sum(st["track_steps"]), 1)}
        if prec == ad.MIXED:
            ad.adept_set_timing(sim.ctx, True)
            _, _, st_t = run_once(ad, torch, sim, wl.primaries)
            assert st_t["track_steps"] == st["track_steps"]
            rec["roofline"] = kernel_roofline(st_t, 1, 1)
        sim.close()
        res["mixed" if prec == ad.MIXED else "fp64"] = rec
    (lm, cm), (lf, cf) = tallies[ad.MIXED], tallies[ad.FP64]
    rel = np.abs(lm - lf) / lf
    big = cf > 1e-6 * cf.sum()
    res["edep_rel_error_mixed_vs_fp64"] = {
        "per_layer_max": float(rel.max()), "per_layer_max_over_layers_above_1e-3_of_total":
            float(rel[lf > 1e-3 * lf.sum()].max()), "total": float(abs(lm.sum() - lf.sum()) / lf.sum()),
        "per_cell_max_over_cells_above_1e-6_of_total": float((np.abs(cm - cf)[big] / cf[big]).max()),
        "cells_sum_over_layer_sum_mixed": float(cm.sum() / lm.sum())}
    res["speedup_mixed_vs_fp64"] = res["fp64"]["seconds"] / res["mixed"]["seconds"]
    return res


def layout_study(ad, torch, np, workloads):
    """Paper Sec. 4-5 on the toy model: 10^4 e- of 10 GeV (FP64) timed in the sparse
    single buffer (AoS) and the dense double buffer (AoS, SoA, AoSoA-64); then, in
    instrumented mode over injection + 20 iterations, the per-field access counts of
    the electron buffer, slot utilisation and the per-type maximum access counts."""
    wl = workloads.showers_10ke_10gev()
    C = 1 << 22
    dev = torch.from_numpy(wl.primaries.view(np.uint8).copy()).cuda()
    res = {"workload": wl.description, "precision": "FP64", "timings": {},
           "note": "the active set peaks near 10^6 tracks (about 0.1 GB per buffer), largely inside the 256 MB "
                   "Infinity Cache: the rooflines here are not HBM measurements"}
    for name, (s, m, n) in {"sparse AoS": (0, 0, 1), "dense AoS": (1, 0, 1), "dense SoA": (1, 1, 1),
                            "dense AoSoA-64": (1, 2, 64)}.items():
        sim = ad.Sim(s, m, ad.FP64, C, n, seeds=wl.seeds, launch={"block": 1024, "graph_iters": 32})
        best = 1e9
        for r in range(3):
            dt, it, st = run_once(ad, torch, sim, wl.primaries, dev)
            if r:
                best = min(best, dt)
        ad.adept_set_timing(sim.ctx, True)
        _, _, st_t = run_once(ad, torch, sim, wl.primaries, dev)
        sim.close()
        res["timings"][name] = {"ms": best * 1e3, "track_steps_per_s": sum(st["track_steps"]) / best,
                                "roofline": kernel_roofline(st_t, s, 0)}
    counts = {}
    for name, (s, m, n) in {"sparse AoS": (0, 0, 1), "dense AoS": (1, 0, 1)}.items():
        sim = ad.Sim(s, m, ad.FP64, C, n, seeds=wl.seeds, instrumented=20)
        sim.inject(wl.primaries)
        sim.run(20)
        rec = {}
        for t, tn in enumerate(("electrons", "positrons", "photons")):
            hs = [sim.access_counts(t, b, heat=True) for b in range(2 if s else 1)]
            heat = np.concatenate([h[2] for h in hs])
            per_slot = heat.reshape(-1, 24).sum(axis=1)  # 96-byte records = 24 words
            rec[tn] = {"reads_per_field": [int(x) for x in sum(h[0] for h in hs)],
                       "writes_per_field": [int(x) for x in sum(h[1] for h in hs)],
                       "max_word_count": int(heat.max()), "slots_touched": int(np.count_nonzero(per_slot))}
        sim.close()
        counts[name] = rec
    res["instrumented_first_20_iterations"] = counts
    # Cache-line view (Sec. 5 heatmaps at the granularity HBM moves): each 128-byte
    # line is taken to move once per access of its most accessed word, so the bytes
    # moved are 128 x the per-line maxima and the bytes used are 4 x the word counts.
    lines = {}
    for name, (s, m, n) in {"sparse AoS": (0, 0, 1), "sparse SoA": (0, 1, 1), "dense AoS": (1, 0, 1),
                            "dense SoA": (1, 1, 1), "dense AoSoA-64": (1, 2, 64)}.items():
        sim = ad.Sim(s, m, ad.FP64, C, n, seeds=wl.seeds, instrumented=20)
        sim.inject(wl.primaries)
        sim.run(20)
        used = moved = touched = 0
        for t in range(3):
            for b in range(2 if s else 1):
                words = sim.access_counts(t, b, heat=True)[2].astype(np.uint64)
                lh = sim.line_heat(t, b, 128)
                words = np.concatenate([words, np.zeros(-len(words) % 32, dtype=np.uint64)]).reshape(-1, 32)
                assert np.array_equal(words.sum(axis=1), lh)
                used += 4 * int(words.sum())
                moved += 128 * int(words.max(axis=1).sum())
                touched += int(np.count_nonzero(lh))
        sim.close()
        lines[name] = {"bytes_used": used, "bytes_moved_line_model": moved, "useful_fraction": used / max(moved, 1),
                       "lines_touched": touched}
    res["cache_lines_first_20_iterations"] = lines
    # Per-particle-type layouts (Sec. 6 future work): the per-type autotuner over
    # the sparse single buffer's AoS / SoA / AoSoA-64, on the whole workload.
    steps = sum(st["track_steps"])
    cands = [(0, 0, 1), (0, 1, 1), (0, 2, 64)]
    lay, launch, ms = ad.adept_autotune_type_layouts(ad.FP64, C, cands, wl.seeds, wl.primaries)
    names = {(0, 1): "AoS", (1, 1): "SoA", (2, 64): "AoSoA-64"}
    res["per_type_layouts_sparse"] = {
        "autotuned": {t: names.get(tuple(l), str(l)) for t, l in zip(("electrons", "positrons", "photons"), lay)},
        "launch": launch, "ms": ms, "track_steps_per_s": steps / (ms * 1e-3),
        "note": "per-type contexts address every field through one general mapping form"}
    sp, dn = counts["sparse AoS"], counts["dense AoS"]
    res["paper_claims"] = {
        "slots_touched_sparse_vs_dense_electrons": [sp["electrons"]["slots_touched"], dn["electrons"]["slots_touched"]],
        "max_access_ratio_e-/e+_sparse": sp["electrons"]["max_word_count"] / max(sp["positrons"]["max_word_count"], 1),
        "max_access_ratio_e-/gamma_sparse": sp["electrons"]["max_word_count"] / max(sp["photons"]["max_word_count"], 1),
    }
    return res


def main():
    args = parse()
    if args.pmc_summary:
        print(json.dumps(pmc_summary(args.pmc_summary), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the transport path shards by events "
              "with no exchange until a final tally reduction, which this build does not run.", file=sys.stderr)
        sys.exit(2)
    import numpy as np

    import workloads

    wl = workloads.showers_100ke_10gev(args.primaries)
    # the CPU baseline first: the oracle's worker processes are forked before this
    # process initialises the GPU
    cpu = None
    if not args.headline_only and not args.batched_profile and not args.line_check and not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, args.cpu_sample, 1, flip_sample=args.flip_sample)
        progress(f"cpu baseline: {cpu['value']:.3e} track-steps/s on {cpu['cores']} cores")
    import torch

    import paper_2302_08252_amd as ad

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ad.lib()
    if args.copy_calibration:
        src = torch.ones(args.copy_calibration << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.batched_profile:
        print(json.dumps({"batched_profile": batched_profile(ad, torch, np, workloads, args)}), flush=True)
        return
    if args.line_check:
        print(json.dumps({"line_check": line_check(ad, torch, np, workloads, args.line_check)}), flush=True)
        return
    if args.segmented_profile:
        print(json.dumps({"segmented_profile": segmented_profile(ad, torch, np, workloads)}), flush=True)
        return
    if args.layout_pair:
        print(json.dumps({"layout_pair": layout_pair(ad, torch, wl, args)}), flush=True)
        return
    C = 1 << args.capacity_log2
    dev_prims = torch.from_numpy(wl.primaries.view(np.uint8).copy()).cuda()
    head = time_path(ad, torch, wl, dev_prims, ad.DENSE_DOUBLE, ad.MAP_SOA, ad.MIXED, C, args, args.steps,
                     args.warmup, timing=True)
    progress(f"headline: {head['track_steps_per_s']:.3e} track-steps/s")
    st = head["stats"]
    alg = algorithmic_bytes(st, 1, 1)  # bytes of one run
    kernel_s = st["step_kernel_ms"] / 1e3
    achieved = alg * args.steps / kernel_s / 1e9 if kernel_s > 0 else None
    out = {
        "metric": "track-steps/sec on 1 MI355X: mixed vs FP64 layout, per-layer Edep error stated",
        "value": head["track_steps_per_s"],
        "unit": "track-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64 (mixed)",
        "data": "synthetic",
        "config": {
            "workload": f"1 event x {args.primaries} e- at 10 GeV from (0,0,0) along +z, seed 7; "
                        "50-layer absorber/gap calorimeter; all primaries injected at once",
            "scheme": "dense double buffer", "layout": "SoA", "precision": "mixed",
            "capacity_per_type": C, "block": args.block, "graph_iters": args.graph_iters,
            "wave_tiles": args.wave_tiles,
        },
        "primaries_per_s": head["primaries_per_s"],
        "timed_runs": {"ms_mean": head["ms_per_step"], "ms_min": head["ms_min"], "cv": head["cv"]},
        "track_steps_per_run": head["track_steps_per_run"],
        "iterations_per_run": head["iterations"],
        "divergent_wave_fraction": st["waves_divergent"] / max(st["waves"], 1),
        "lanes_off_mode_fraction": head["lanes_off_mode_fraction"],
        "divergence_rate_rocprof": (1.0 - measured_lane_use() / 64.0) if measured_lane_use() else None,
        "closure_error": head["closure"],
        "roofline": {
            "bound": "hbm", "kernel": "k_step (fused transport step)",
            "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": (achieved / PEAK_HBM_GBS) if achieved else None,
            "traffic": measured_traffic(),
            "kernel_source_hash": kernel_source_hash(),
            "algorithmic_bytes_per_run": alg,
            "step_launches_timed": st["step_launches"],
            "avg_step_kernel_ms": st["step_kernel_ms"] / max(st["step_launches"], 1),
        },
    }
    if head["phase"].any():  # a library built with ADEPT_PHASE_CLOCKS=1 (ADEPT_LIBRARY)
        names = ["load_and_step", "block_scan_and_slowest_wave", "look_back", "writes", "end_of_tile",
                 "before_first_tile", "after_last_tile"]
        tot = float(head["phase"].sum())
        out["phase_clocks"] = {"fractions_of_wave_cycles": {n: float(v) / tot for n, v in zip(names, head["phase"])},
                               "wave_cycles": int(tot), "library": ad.LIB_PATH}
    if not args.headline_only and args.fp64_steps > 0:
        f64 = time_path(ad, torch, wl, dev_prims, ad.DENSE_DOUBLE, ad.MAP_SOA, ad.FP64, C, args, args.fp64_steps,
                        1, timing=False)
        sp = time_path(ad, torch, wl, dev_prims, ad.SPARSE_SINGLE, ad.MAP_AOS, ad.FP64, C, args, args.fp64_steps,
                       1, timing=False)
        lm, lf = head["layer"], f64["layer"]
        rel = np.abs(lm - lf) / np.maximum(np.abs(lf), 1e-300)
        assert np.array_equal(lf, sp["layer"]) or np.allclose(lf, sp["layer"], rtol=1e-12)
        def run_gbps(r, scheme, precision):  # algorithmic bytes of a run over its wall time
            return algorithmic_bytes(r["stats"], scheme, precision) / (r["ms_per_step"] * 1e-3) / 1e9

        def div(r):
            return {"waves_with_disagreeing_lanes": r["stats"]["waves_divergent"] / max(r["stats"]["waves"], 1),
                    "lanes_off_mode": r["lanes_off_mode_fraction"]}

        out["fp64_dense_soa"] = {"track_steps_per_s": f64["track_steps_per_s"], "ms_per_step": f64["ms_per_step"],
                                 "closure_error": f64["closure"], "algorithmic_GBps_run": run_gbps(f64, 1, 0),
                                 "divergence": div(f64)}
        out["fp64_sparse_aos"] = {"track_steps_per_s": sp["track_steps_per_s"], "ms_per_step": sp["ms_per_step"],
                                  "closure_error": sp["closure"], "algorithmic_GBps_run": run_gbps(sp, 0, 0),
                                  "divergence": div(sp)}
        progress("FP64 comparison paths done")
        out["algorithmic_GBps_run"] = run_gbps(head, 1, 1)
        out["speedup_vs_fp64_sparse_aos"] = sp["ms_per_step"] / head["ms_per_step"]
        out["edep_per_layer_rel_error_mixed_vs_fp64"] = {
            "max": float(rel.max()), "max_over_layers_above_1e-3_of_total": float(rel[lf > 1e-3 * lf.sum()].max()),
            "total": float(abs(lm.sum() - lf.sum()) / lf.sum()),
            "reference": "the same workload in FP64 on the GPU (bit-exact with the FP64 oracle per track)",
        }
    if not args.headline_only and not args.no_batched:
        out["batched_512_events"] = batched_section(ad, torch, np, workloads, args)
        progress("batched section done")
    if not args.headline_only and not args.no_segmented:
        out["segmented_1000_events"] = segmented_section(ad, torch, np, workloads)
        progress("segmented section done")
    if not args.headline_only and not args.no_layout_study:
        out["layout_study_10ke"] = layout_study(ad, torch, np, workloads)
        progress("layout study done")
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
