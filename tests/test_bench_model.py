"""The roofline numerator of bench.py (algorithmic bytes of the dense double
buffer) equals the record traffic the oracle counts field by field in its
instrumented mode, over a whole run (CPU only)."""
import numpy as np

import workloads


def test_dense_algorithmic_bytes_match_counted_accesses(oracle_mod):
    import bench

    for precision in (0, 1):
        wl = workloads.showers_100e_1gev().subset(12)
        o = oracle_mod.Oracle(oracle_mod.DENSE, precision, 1 << 16, wl.seeds)
        o.set_instrumented(True, 1 << 40)
        o.inject(wl.primaries)
        outputs = 0
        while True:
            rc, cnt = o.step()
            assert rc == 0
            outputs += int(cnt.sum())
            if cnt.sum() == 0:
                break
        size = np.array([oracle_mod.leaf_size(precision, l) for l in range(14)], dtype=np.uint64)
        read = written = 0
        survivors = 0
        for t in range(3):
            for b in range(2):
                r, w = o.access_totals(t, b)
                read += int((r * size).sum())
                written += int((w * size).sum())
                survivors += int(r[9])  # a dense survivor reads its parent id once
        rec = int(size.sum())
        injected = len(wl.primaries)  # every 1 GeV primary is buffered: one whole record each
        steps = sum(o.stats()["track_steps"])
        assert steps > 1000 and survivors > 0 and outputs > survivors
        st = {"track_steps": [steps, 0, 0], "survivors": [survivors, 0, 0], "outputs": [outputs, 0, 0]}
        assert written == (outputs + injected) * rec
        assert read + written - injected * rec == bench.algorithmic_bytes(st, 1, precision)


def test_sparse_record_bytes_match_counted_accesses(oracle_mod):
    """The record part of the sparse byte model (reads of every source, in-place
    writes of survivors, whole records for creations) against the counted accesses;
    the u32 slot-list and ring words it adds are not track fields."""
    import bench

    for precision in (0, 1):
        wl = workloads.showers_100e_1gev().subset(12)
        o = oracle_mod.Oracle(oracle_mod.SPARSE, precision, 1 << 16, wl.seeds)
        o.set_instrumented(True, 1 << 40)
        o.inject(wl.primaries)
        outputs = 0
        while True:
            rc, cnt = o.step()
            assert rc == 0
            outputs += int(cnt.sum())
            if cnt.sum() == 0:
                break
        size = np.array([oracle_mod.leaf_size(precision, l) for l in range(14)], dtype=np.uint64)
        rec = int(size.sum())
        injected = len(wl.primaries)
        read = written = 0
        surv = [0, 0, 0]
        for t in range(3):
            r, w = o.access_totals(t, 0)
            read += int((r * size).sum())
            written += int((w * size).sum())
            # rngCtr is written by every survivor and every whole record, parentId only by whole records
            surv[t] = int(w[11]) - int(w[9])
        steps = sum(o.stats()["track_steps"])
        created = outputs - sum(surv)
        killed = steps - sum(surv)
        st = {"track_steps": [steps, 0, 0], "survivors": surv, "outputs": [outputs, 0, 0]}
        lists = steps * 4 + outputs * 4 + created * 4 + killed * 4  # u32 list and ring words of the model
        assert steps > 1000 and created > 0 and killed > 0
        assert read + written - injected * rec == bench.algorithmic_bytes(st, 0, precision) - lists
