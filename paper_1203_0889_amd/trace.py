"""Summaries of the device task trace (FMM_FLAG_TRACE, fmm_get_trace).

The paper judges its runtime by a per-core task timeline (Sec. 5): how
evenly the tasks fill the cores and how long the tail is.  Here a "core" is
a compute unit; an M2L task occupies one wave on each of the four SIMDs of a
compute unit, a P2P task one wave.
"""
import numpy as np

TICK_US = 0.01   # the device real-time clock runs at 100 MHz


def units(rec):
    """(xcc, shader engine, shader array, CU) of every record, as one int."""
    hw = rec["hw_id"].astype(np.int64)
    cu = (hw >> 8) & 15
    sa = (hw >> 12) & 1
    se = (hw >> 13) & 7
    return ((rec["xcc"].astype(np.int64) * 8 + se) * 2 + sa) * 16 + cu


def summarize(rec):
    """Counts, span, task durations and per-CU balance of one traced queue run."""
    if len(rec) == 0:
        return {"tasks": 0}
    t0 = int(rec["start"].min())
    start = (rec["start"].astype(np.int64) - t0) * TICK_US
    end = (rec["end"].astype(np.int64) - t0) * TICK_US
    dur = end - start
    waves = np.where(rec["kind"] == 0, 4.0, 1.0)   # an M2L task holds a whole workgroup
    u = units(rec)
    ids, inv = np.unique(u, return_inverse=True)
    busy = np.bincount(inv, weights=dur * waves)
    last = np.zeros(len(ids))
    np.maximum.at(last, inv, end)
    out = {"tasks": int(len(rec)), "span_us": float(end.max()), "compute_units": int(len(ids))}
    for kind, name in ((0, "m2l"), (1, "p2p")):
        m = rec["kind"] == kind
        if m.any():
            out[name] = {"tasks": int(m.sum()), "mean_us": float(dur[m].mean()),
                         "median_us": float(np.median(dur[m])), "max_us": float(dur[m].max()),
                         "by_side_kernel": int((rec["kernel"][m] == 1).sum())}
    out["cu_busy_wave_us"] = {"mean": float(busy.mean()), "min": float(busy.min()), "max": float(busy.max())}
    out["cu_busy_imbalance"] = float(busy.max() / busy.mean())
    out["cu_last_end_us"] = {"min": float(last.min()), "median": float(np.median(last)), "max": float(last.max())}
    return out
