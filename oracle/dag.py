"""Kernel-task DAG and as-soon-as-possible schedule (oracle; test
infrastructure only).

Each elimination (i, piv, k) of a list expands into tile kernels:
  * TT kernels (Algorithm 3): GEQRT + UNMQR on both rows if their tile in
    column k is not yet a triangle, then TTQRT and the TTMQR updates.
  * TS kernels (Algorithm 2): GEQRT + UNMQR on the pivot row if needed, then
    TSQRT and the TSMQR updates.  On trees other than FlatTree a killed row
    that is itself a pivot in column k has already been triangularized, so it
    is eliminated with TT kernels; a TS kernel is used only when the killed
    row is a leaf of the column's tree.  This is the TS-to-TT conversion of
    Sec. 2.1 applied only where TS cannot be used.
  * A tile already in triangle form is not factored again (Sec. 2.1).
  * For a square tile matrix the last diagonal tile only needs its GEQRT
    (proof of Theorem 1(1)).

Dependencies are the data flow between tiles in list order.  The upper
(R / TT reflector) part and the strictly lower (GEQRT reflector) part of a
triangularized tile are tracked separately: update kernels only read the
reflectors, and the TT factor kernels only write the upper part, so an UNMQR
may run alongside the TTQRT that uses its row as pivot (Sec. 2.1 and the
NODEP flag of Sec. 4).  Weights are those of Table 1 in units of nb^3/3 flops.

Parity: the schedule reproduces Tables 3, 4(a) (Greedy) and 5 of the paper,
Theorem 1(1) and Propositions 1 and 2 (tests in tests/test_oracle_trees.py).
"""

from . import trees

GEQRT, UNMQR, TSQRT, TSMQR, TTQRT, TTMQR = 0, 1, 2, 3, 4, 5
KIND_NAMES = ["GEQRT", "UNMQR", "TSQRT", "TSMQR", "TTQRT", "TTMQR"]
WEIGHT = [4, 6, 6, 12, 2, 6]

KERN_DEFAULT, KERN_TT, KERN_TS = 0, 1, 2


def resolve_kernels(tree, kernels):
    """Default family: TS for FlatTree (PLASMA's algorithm, Proposition 2),
    TT for every other tree (the paper's algorithms, Sec. 2.1)."""
    if kernels == KERN_DEFAULT:
        return KERN_TS if tree == trees.FLAT else KERN_TT
    if kernels not in (KERN_TT, KERN_TS):
        raise ValueError("unknown kernel family")
    return kernels


def build_tasks(p, q, elims, kernels):
    """Expand an elimination list into tasks.

    Returns (tasks, preds): tasks is a list of (kind, i, piv, k, j) with 0 for
    unused fields (GEQRT: (0, r, 0, k, 0); UNMQR: (1, r, 0, k, j)); preds[t]
    is the sorted list of distinct predecessor task indices of task t.
    """
    if kernels not in (KERN_TT, KERN_TS):
        raise ValueError("kernels must be KERN_TT or KERN_TS here")
    tasks, preds = [], []
    last_r = {}   # tile -> last task writing its upper / whole part
    last_v = {}   # tile -> last task writing its strictly lower part
    tri = set()   # tiles already in triangle form

    pivots = {}
    for (i, piv, k) in elims:
        pivots.setdefault(k, set()).add(piv)

    def add(task, deps):
        idx = len(tasks)
        tasks.append(task)
        preds.append(sorted({d for d in deps if d is not None}))
        return idx

    def whole(tile):
        return [last_r.get(tile), last_v.get(tile)]

    def triangularize(r, k):
        t = add((GEQRT, r, 0, k, 0), whole((r, k)))
        last_r[(r, k)] = last_v[(r, k)] = t
        tri.add((r, k))
        for j in range(k + 1, q + 1):
            u = add((UNMQR, r, 0, k, j), [t] + whole((r, j)))
            last_r[(r, j)] = last_v[(r, j)] = u

    for (i, piv, k) in elims:
        if (piv, k) not in tri:
            triangularize(piv, k)
        leaf = i not in pivots.get(k, ())
        if kernels == KERN_TS and leaf and (i, k) not in tri:
            f = add((TSQRT, i, piv, k, 0), [last_r.get((piv, k))] + whole((i, k)))
            last_r[(piv, k)] = f
            last_r[(i, k)] = last_v[(i, k)] = f
            upd = TSMQR
        else:
            if (i, k) not in tri:
                triangularize(i, k)
            f = add((TTQRT, i, piv, k, 0), [last_r.get((piv, k)), last_r.get((i, k))])
            last_r[(piv, k)] = f
            last_r[(i, k)] = f
            upd = TTMQR
        for j in range(k + 1, q + 1):
            u = add((upd, i, piv, k, j), [f] + whole((piv, j)) + whole((i, j)))
            last_r[(piv, j)] = last_v[(piv, j)] = u
            last_r[(i, j)] = last_v[(i, j)] = u
    if p == q and (q, q) not in tri:
        triangularize(q, q)
    return tasks, preds


def asap(tasks, preds, weights=WEIGHT):
    """Unbounded-processor ASAP schedule (Sec. 2.3): a task starts when its
    last predecessor finishes.  Returns (start, finish, critical_path)."""
    start, finish = [], []
    for t, task in enumerate(tasks):
        s = max((finish[d] for d in preds[t]), default=0)
        start.append(s)
        finish.append(s + weights[task[0]])
    return start, finish, max(finish, default=0)


def schedule(p, q, tree, bs=1, kernels=KERN_DEFAULT):
    """List -> tasks -> schedule.  Returns (rows, cp) where rows are
    (kind, i, piv, k, j, start, finish) in task emission order."""
    kern = resolve_kernels(tree, kernels)
    elims = trees.elim_list(p, q, tree, bs)
    tasks, preds = build_tasks(p, q, elims, kern)
    start, finish, cp = asap(tasks, preds)
    rows = [tuple(t) + (s, f) for t, s, f in zip(tasks, start, finish)]
    return rows, cp


def critical_path(p, q, tree, bs=1, kernels=KERN_DEFAULT):
    return schedule(p, q, tree, bs, kernels)[1]


def zero_times(p, q, tree, bs=1, kernels=KERN_DEFAULT):
    """Time at which each tile (i, k), i > k, is zeroed: the finish time of
    its TTQRT or TSQRT task (the quantity printed in Tables 3 and 4)."""
    rows, _ = schedule(p, q, tree, bs, kernels)
    return {(r[1], r[3]): r[6] for r in rows if r[0] in (TTQRT, TSQRT)}


def best_plasma_bs(p, q, kernels=KERN_TT):
    """Exhaustive search over BS in [1, p] (Sec. 4), smallest BS among ties.
    Returns (cp, bs)."""
    best = None
    for bs in range(1, p + 1):
        cp = critical_path(p, q, trees.PLASMA, bs, kernels)
        if best is None or cp < best[0]:
            best = (cp, bs)
    return best


def total_work_units(tasks):
    return sum(WEIGHT[t[0]] for t in tasks)
