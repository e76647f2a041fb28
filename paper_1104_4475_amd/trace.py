"""Summary of an executor trace (Factors.trace()): per-kernel durations,
dependency waits and workgroup utilization."""

import numpy as np

KIND_NAMES = ["GEQRT", "UNMQR", "TSQRT", "TSMQR", "TTQRT", "TTMQR", "APPLY_GE", "APPLY_TS", "APPLY_TT"]


def summarize(tr, rate):
    """tr: int64 (n, 10) from Factors.trace(); rate: ticks per second.
    Returns a dict of per-kind statistics (microseconds) and totals."""
    tr = np.asarray(tr)
    us = 1e6 / rate
    ticket, ready, end, wg = tr[:, 6], tr[:, 7], tr[:, 8], tr[:, 9]
    t0 = ticket.min()
    makespan = (end.max() - t0) * us
    run = (end - ready) * us
    wait = (ready - ticket) * us
    nwg = len(np.unique(wg))
    out = {"subtasks": int(len(tr)), "workgroups": nwg, "makespan_us": float(makespan),
           "busy_us": float(run.sum()), "wait_us": float(wait.sum()),
           "utilization": float(run.sum() / (nwg * makespan)) if makespan > 0 else 0.0, "kinds": {}}
    for k in np.unique(tr[:, 0]):
        sel = tr[:, 0] == k
        out["kinds"][KIND_NAMES[int(k)]] = {
            "count": int(sel.sum()), "mean_us": float(run[sel].mean()), "max_us": float(run[sel].max()),
            "total_us": float(run[sel].sum()), "mean_wait_us": float(wait[sel].mean())}
    return out


def format_summary(s):
    lines = ["subtasks %d on %d workgroups: makespan %.1f us, utilization %.1f%%, waiting %.1f%% of workgroup time"
             % (s["subtasks"], s["workgroups"], s["makespan_us"], 100 * s["utilization"],
                100 * s["wait_us"] / max(1e-9, s["workgroups"] * s["makespan_us"]))]
    for k, v in sorted(s["kinds"].items(), key=lambda kv: -kv[1]["total_us"]):
        lines.append("  %-8s n=%6d mean %8.1f us max %8.1f us total %10.0f us mean wait %8.1f us"
                     % (k, v["count"], v["mean_us"], v["max_us"], v["total_us"], v["mean_wait_us"]))
    return "\n".join(lines)
