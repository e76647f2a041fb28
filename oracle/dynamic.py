"""Run-time pairing schemes ASAP and GRASAP(k) (oracle; test infrastructure
only).

Sec. 3.2 (the tiled model, discussion of Table 4): in the tiled model with
TT kernels and the Table 1 weights, ASAP decides the pairs of every column
while the factorization runs.  Whenever at least two rows of a column are
ready, it starts eliminations at once: with s = floor(r / 2) for r ready
rows, it pairs them as the coarse-grain schemes do, the first of the 2s rows
with row s + 1, the second with row s + 2, and so on.  GRASAP(k) pairs the
first q - k columns by the Greedy list and the last k columns by ASAP;
GRASAP(0) is Greedy and GRASAP(q) is ASAP.

Reading of the parts the text leaves open (recorded with the design notes):
  * A row is ready in column k when its tile (i, k) has been triangularized
    (its GEQRT has finished, which waits for every update of column k - 1),
    and idle when it is not taking part in a running TTQRT.  Rows are
    examined at integer times; the ready idle rows of a column, sorted top
    to bottom, give the 2s rows to pair: the bottom s are killed by the s
    rows right above them (the top row is left over when r is odd, so the
    diagonal row is never killed).
  * Every other task starts as soon as its inputs are ready (Sec. 2.3), with
    the data flow of Algorithm 3: GEQRT(i, k) after the last update of tile
    (i, k); UNMQR(i, k, j) after GEQRT(i, k) and the last update of (i, j);
    TTMQR(i, piv, k, j) after its TTQRT and the last updates of (piv, j) and
    (i, j).  A TTQRT only needs the triangles of its two rows.
This reading reproduces the ASAP column and the Greedy column of Table 4(a)
exactly, the critical path 62 of GRASAP(1) on 15 x 3, and 9 of the 10 ASAP
entries of Table 4(b) (the exceptions are listed with the tests).

The schemes' pairs form an ordinary elimination list: the static part in its
own order, then the run-time eliminations in the order they start (ties by
column, then killed row).  Fed to the task DAG of Algorithm 3 with list-order
data flow, that list is scheduled exactly as the simulation ran it.
"""

import heapq

from . import trees

W_GEQRT, W_UNMQR, W_TTQRT, W_TTMQR = 4, 6, 2, 6


def simulate(p, q, static, dynamic_from):
    """Tiled TT simulation.  static: eliminations (i, piv, k) of the columns
    k < dynamic_from, in list order; columns k >= dynamic_from are paired at
    run time.  Returns (list, zero_times, critical_path)."""
    kmax = min(p, q)
    avail = {}     # tile (r, j) -> finish of its last update
    ready = {}     # (r, k) -> finish of GEQRT(r, k)
    rbusy = {}     # row -> finish of the running TTQRT that uses it
    zero = {}      # (i, k) -> finish of the TTQRT that zeroed it
    cp = [0]

    def upd(tile, fin):
        avail[tile] = fin
        cp[0] = max(cp[0], fin)

    def enter(r, k):
        """Row r starts column k: GEQRT(r, k) and its UNMQRs."""
        s = avail.get((r, k), 0)
        f = s + W_GEQRT
        ready[(r, k)] = f
        upd((r, k), f)
        for j in range(k + 1, q + 1):
            upd((r, j), max(f, avail.get((r, j), 0)) + W_UNMQR)
        return f

    def eliminate(i, piv, k, t):
        """TTQRT(i, piv, k) at t and its TTMQRs; row i then enters k + 1."""
        f = t + W_TTQRT
        rbusy[i] = rbusy[piv] = f
        zero[(i, k)] = f
        cp[0] = max(cp[0], f)
        for j in range(k + 1, q + 1):
            u = max(f, avail.get((piv, j), 0), avail.get((i, j), 0)) + W_TTMQR
            upd((piv, j), u)
            upd((i, j), u)
        if k + 1 <= kmax:  # (for p = q the last column is GEQRT(q, q) alone)
            return enter(i, k + 1)
        return None

    out = []
    # Column 1 (all rows), then the static columns in list order: a TTQRT
    # starts when both triangles are free (their last writer finished).
    rfree = {}  # (r, k) -> time the triangle of (r, k) is free
    for r in range(1, p + 1):
        rfree[(r, 1)] = enter(r, 1)
    for (i, piv, k) in static:
        t = max(rfree[(piv, k)], rfree[(i, k)])
        f = eliminate(i, piv, k, t)
        rfree[(piv, k)] = t + W_TTQRT
        if f is not None:
            rfree[(i, k + 1)] = f
        out.append((i, piv, k))
    # Run-time columns: event-driven over the times at which a row of a
    # column becomes ready or idle.
    alive = {k: set() for k in range(dynamic_from, kmax + 1)}
    events = []
    for k in range(dynamic_from, kmax + 1):
        for r in range(k, p + 1):
            if (r, k) in ready:
                alive[k].add(r)
                heapq.heappush(events, (ready[(r, k)], k))
    dyn = []
    while events:
        t = events[0][0]
        cols = set()
        while events and events[0][0] == t:
            cols.add(heapq.heappop(events)[1])
        for k in sorted(cols):
            rows = sorted(r for r in alive[k] if ready[(r, k)] <= t and rbusy.get(r, 0) <= t)
            s = len(rows) // 2
            if s == 0:
                continue
            piv_rows, kill_rows = rows[len(rows) - 2 * s:len(rows) - s], rows[len(rows) - s:]
            for piv, i in zip(piv_rows, kill_rows):
                f = eliminate(i, piv, k, t)
                alive[k].discard(i)
                dyn.append((t, k, i, piv))
                if f is not None:
                    alive[k + 1].add(i)
                    heapq.heappush(events, (f, k + 1))
            heapq.heappush(events, (t + W_TTQRT, k))
    dyn.sort()
    out += [(i, piv, k) for (_t, k, i, piv) in dyn]
    return out, zero, cp[0]


def asap(p, q):
    """ASAP elimination list (Sec. 3.2)."""
    trees._check(p, q)
    return simulate(p, q, [], 1)[0]


def grasap(p, q, k):
    """GRASAP(k): Greedy pairs for columns 1..q-k, ASAP for the last k."""
    trees._check(p, q)
    if k < 0:
        raise ValueError("k must be >= 0")
    cut = max(1, min(p, q) - k + 1) if k > 0 else min(p, q) + 1
    static = [e for e in trees.greedy_tree(p, q) if e[2] < cut]
    return simulate(p, q, static, cut)[0]


def asap_times(p, q, k=None):
    """(zero_times, critical_path) of ASAP (k None) or GRASAP(k)."""
    trees._check(p, q)
    if k is None:
        _, z, cp = simulate(p, q, [], 1)
        return z, cp
    cut = max(1, min(p, q) - k + 1) if k > 0 else min(p, q) + 1
    static = [e for e in trees.greedy_tree(p, q) if e[2] < cut]
    _, z, cp = simulate(p, q, static, cut)
    return z, cp
