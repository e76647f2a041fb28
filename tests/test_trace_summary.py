"""Host summary of an executor trace (paper_1104_4475_amd.trace) on a
hand-made trace whose totals are known."""

import numpy as np

from paper_1104_4475_amd import trace


def test_summary_of_a_known_trace():
    # (kind, i, piv, k, j, slab, ticket, ready, end, workgroup), ticks of 1 us
    rows = [
        (0, 0, 0, 0, 0, 0, 0, 0, 10, 0),    # GEQRT: runs 10, waits 0
        (3, 1, 0, 0, 1, 0, 0, 10, 30, 1),   # TSMQR: waits 10, runs 20
        (3, 1, 0, 0, 1, 1, 10, 10, 40, 0),  # TSMQR: runs 30
    ]
    s = trace.summarize(np.array(rows, dtype=np.int64), 1e6)
    assert s["subtasks"] == 3 and s["workgroups"] == 2
    assert s["makespan_us"] == 40.0
    assert s["busy_us"] == 60.0 and s["wait_us"] == 10.0
    assert s["utilization"] == 60.0 / (2 * 40.0)
    k = s["kinds"]
    assert set(k) == {"GEQRT", "TSMQR"}
    assert k["GEQRT"]["count"] == 1 and k["GEQRT"]["mean_us"] == 10.0
    assert k["TSMQR"]["count"] == 2 and k["TSMQR"]["mean_us"] == 25.0 and k["TSMQR"]["max_us"] == 30.0
    assert k["TSMQR"]["mean_wait_us"] == 5.0
    text = trace.format_summary(s)
    assert "utilization 75.0%" in text and "TSMQR" in text
