"""Elimination lists (oracle; test infrastructure only).

An elimination list is an ordered list of triples (i, piv, k), 1-based, meaning
"zero tile (i, k) by combining row i with row piv" (Sec. 2.2).  Each generator
below emits its list in a fixed order; that order is the one the GPU library's
host planner must reproduce byte for byte.

Trees (Sec. 3.1 and Sec. 3.2):
  FlatTree == Sameh-Kuck   column k: row k kills rows k+1..p in order.
  BinaryTree               per column, a binary reduction rooted at row k.
  Fibonacci                Modi-Clarke order-1 scheme with closed-form steps.
  Greedy                   Algorithm 4 (rounds of nT/nZ counters).
  PlasmaTree(BS)           flat trees inside domains of BS rows anchored at
                           row k, then a binary merge of the domain heads.
  ASAP, GRASAP(k)          run-time pairings of the tiled model
                           (oracle/dynamic.py).
  Hadri(BS)                PlasmaTree with fixed domains (rows 1..BS, ...):
                           the top domain shrinks (Sec. 4).

Readings where the text leaves room (each pinned by Table 3 of the paper):
  * BinaryTree is re-rooted at row k in every column (offsets from k).
  * Fibonacci column k uses the column-1 step table shifted down by k-1 rows
    plus 2(k-1), truncated at row p; the z rows zeroed at one step pair with
    the z rows immediately above them, z counted after truncation.
  * PlasmaTree domains start at row k, so only the bottom domain shrinks;
    all flat trees of a column are emitted before the merges.

Parity: pinned by Tables 2, 3, 4 and 5 of the paper (golden fixtures in
tests/golden/), by the list identities PT(1) == BinaryTree, PT(p) == FlatTree,
and by the validity conditions of Sec. 2.2 and Lemma 1.
"""

FLAT, SAMEH_KUCK, BINARY, FIBONACCI, GREEDY, PLASMA, ASAP, GRASAP, HADRI = 0, 1, 2, 3, 4, 5, 6, 7, 8
TREE_NAMES = {FLAT: "FlatTree", SAMEH_KUCK: "Sameh-Kuck", BINARY: "BinaryTree",
              FIBONACCI: "Fibonacci", GREEDY: "Greedy", PLASMA: "PlasmaTree",
              ASAP: "ASAP", GRASAP: "GRASAP", HADRI: "Hadri (Semi/Fully-Parallel)"}


def _check(p, q):
    if p < 1 or q < 1 or p < q:
        raise ValueError("need p >= q >= 1 (p=%r, q=%r)" % (p, q))


def flat_tree(p, q):
    """Sameh-Kuck / FlatTree list, Sec. 3.1 (formal list) and Sec. 3.2."""
    _check(p, q)
    out = []
    for k in range(1, min(p, q) + 1):
        for i in range(k + 1, p + 1):
            out.append((i, k, k))
    return out


def binary_tree(p, q):
    """BinaryTree, Sec. 3.2 (before Proposition 1).

    In column k the rows k..p are reduced pairwise: at level l the row at
    offset o (from k) with o mod 2^l == 2^(l-1) is killed by the row at
    offset o - 2^(l-1).
    """
    _check(p, q)
    out = []
    for k in range(1, min(p, q) + 1):
        n = p - k + 1
        half = 1
        while half < n:
            for o in range(half, n, 2 * half):
                out.append((k + o, k + o - half, k))
            half *= 2
    return out


def _least_tri(target):
    """Least integer x >= 0 with x(x+1)/2 >= target."""
    x = 0
    while x * (x + 1) // 2 < target:
        x += 1
    return x


def fibonacci_steps(p):
    """coarse(i, 1) of the Fibonacci scheme, Sec. 3.1: dict row -> step.

    x is the least integer with x(x+1)/2 >= p-1; for row i, y is the least
    integer with i <= y(y+1)/2 + 1 and the step is x - y + 1.
    """
    x = _least_tri(p - 1)
    steps = {}
    for i in range(2, p + 1):
        y = _least_tri(i - 1)  # least y with y(y+1)/2 + 1 >= i
        steps[i] = x - y + 1
    return steps


def fibonacci_coarse(p, q):
    """coarse(i, k) for Fibonacci: column 1 shifted down and +2 per column."""
    _check(p, q)
    c1 = fibonacci_steps(p)
    table = {}
    for k in range(1, min(p, q) + 1):
        for i in range(k + 1, p + 1):
            table[(i, k)] = c1[i - k + 1] + 2 * (k - 1)
    return table


def fibonacci_tree(p, q):
    """Fibonacci list, Sec. 3.1: per column, per step ascending, the z rows
    i0..i0+z-1 zeroed at that step are paired with rows i0-z..i0-1."""
    _check(p, q)
    table = fibonacci_coarse(p, q)
    out = []
    for k in range(1, min(p, q) + 1):
        rows_by_step = {}
        for i in range(k + 1, p + 1):
            rows_by_step.setdefault(table[(i, k)], []).append(i)
        for s in sorted(rows_by_step):
            rows = rows_by_step[s]
            z = len(rows)
            i0 = rows[0]
            assert rows == list(range(i0, i0 + z))
            for j in range(z):
                out.append((i0 + j, i0 + j - z, k))
    return out


def greedy_tree(p, q):
    """Greedy via Algorithm 4.

    Rounds repeat until column q is finished.  In a round, columns are visited
    from q down to 1.  Column j first triangularizes the rows that became
    ready (all p rows for j = 1, otherwise the rows zeroed so far in column
    j-1); then it zeroes floor((nT - nZ)/2) more rows from the bottom, using
    the counters as they stood before this round's triangularization, each
    bottom row paired with the row that many positions above it.
    """
    _check(p, q)
    nT = [0] * (q + 1)
    nZ = [0] * (q + 1)
    out = []

    def finished():
        return nZ[q] == p - q and nT[q] == p - q + 1

    guard = 0
    while not finished():
        guard += 1
        if guard > 4 * (p + q) + 16:
            raise RuntimeError("Greedy did not terminate")
        for j in range(q, 0, -1):
            nT_new = p if j == 1 else nZ[j - 1]
            nZ_new = nZ[j] + (nT[j] - nZ[j]) // 2
            for kk in range(nZ[j], nZ_new):
                row = p - kk
                out.append((row, row - nZ_new + nZ[j], j))
            nT[j] = nT_new
            nZ[j] = nZ_new
    return out


def plasma_tree(p, q, bs):
    """PlasmaTree(BS), Sec. 3.2: flat trees within domains of BS consecutive
    rows starting at row k, then a binary tree over the domain heads."""
    _check(p, q)
    if bs < 1 or bs > p:
        raise ValueError("BS must be in [1, p]")
    out = []
    for k in range(1, min(p, q) + 1):
        heads = list(range(k, p + 1, bs))
        for h in heads:
            for i in range(h + 1, min(h + bs - 1, p) + 1):
                out.append((i, h, k))
        nd = len(heads)
        half = 1
        while half < nd:
            for d in range(half, nd, 2 * half):
                out.append((heads[d], heads[d - half], k))
            half *= 2
    return out


def hadri_tree(p, q, bs):
    """The Semi-Parallel / Fully-Parallel tile CAQR trees of Hadri et al., as
    Sec. 4 describes them: flat trees inside domains of BS rows, then a
    binary tree over the domain heads, as PlasmaTree, except that the
    domains stay where they are (rows 1..BS, BS+1..2BS, ...) so that the top
    domain, not the bottom one, shrinks as the columns advance.  Semi- and
    Fully-Parallel differ only in the kernel family (TS or TT, Sec. 2.1).
    Emission order as PlasmaTree: the flat trees of a column, then its
    merges."""
    _check(p, q)
    if bs < 1 or bs > p:
        raise ValueError("BS must be in [1, p]")
    out = []
    for k in range(1, min(p, q) + 1):
        heads = [k] + [h for h in range(bs + 1, p + 1, bs) if h > k]
        for n, h in enumerate(heads):
            end = heads[n + 1] - 1 if n + 1 < len(heads) else p
            for i in range(h + 1, end + 1):
                out.append((i, h, k))
        nd = len(heads)
        half = 1
        while half < nd:
            for d in range(half, nd, 2 * half):
                out.append((heads[d], heads[d - half], k))
            half *= 2
    return out


def elim_list(p, q, tree, bs=1):
    """Dispatch by tree id (FLAT and SAMEH_KUCK give the same list)."""
    if tree in (FLAT, SAMEH_KUCK):
        return flat_tree(p, q)
    if tree == BINARY:
        return binary_tree(p, q)
    if tree == FIBONACCI:
        return fibonacci_tree(p, q)
    if tree == GREEDY:
        return greedy_tree(p, q)
    if tree == PLASMA:
        return plasma_tree(p, q, bs)
    if tree == HADRI:
        return hadri_tree(p, q, bs)
    if tree in (ASAP, GRASAP):
        from . import dynamic  # the run-time pairings (their own module)
        return dynamic.asap(p, q) if tree == ASAP else dynamic.grasap(p, q, bs)
    raise ValueError("unknown tree %r" % (tree,))


def validate(p, q, elims):
    """Check the conditions of Sec. 2.2 and Lemma 1's normal form.

    Returns a list of error strings (empty when the list is valid):
      * every (i, k) with i > k, k <= min(p,q) is zeroed exactly once;
      * piv < i (Lemma 1);
      * both rows are ready: their tiles left of column k were zeroed earlier;
      * the pivot is a potential annihilator: (piv, k) is zeroed later.
    """
    errs = []
    pos = {}
    for n, (i, piv, k) in enumerate(elims):
        if (i, k) in pos:
            errs.append("tile (%d,%d) zeroed twice" % (i, k))
        pos[(i, k)] = n
    for k in range(1, min(p, q) + 1):
        for i in range(k + 1, p + 1):
            if (i, k) not in pos:
                errs.append("tile (%d,%d) never zeroed" % (i, k))
    for n, (i, piv, k) in enumerate(elims):
        if not (1 <= piv < i <= p and 1 <= k <= min(p, q) and piv >= k):
            errs.append("bad triple (%d,%d,%d)" % (i, piv, k))
            continue
        for kp in range(1, k):
            for r in (i, piv):
                if pos.get((r, kp), n + 1) > n:
                    errs.append("row %d not ready for (%d,%d,%d)" % (r, i, piv, k))
        if piv > k and pos.get((piv, k), -1) < n:
            errs.append("pivot %d already zeroed before (%d,%d,%d)" % (piv, i, piv, k))
    return errs


def coarse_times(p, q, elims):
    """Coarse-grain model of Sec. 3.1: each elimination takes one time-step and
    occupies both of its rows; a row may act in column k once its tile in
    column k-1 has been zeroed.  Returns dict (i, k) -> time-step."""
    _check(p, q)
    zeroed = {}
    busy = {}  # (row, k) -> last step the row was used in column k
    for (i, piv, k) in elims:
        t = 0
        for r in (i, piv):
            if k > 1 and r > k - 1:
                t = max(t, zeroed[(r, k - 1)])
            t = max(t, busy.get((r, k), 0))
        t += 1
        zeroed[(i, k)] = t
        busy[(i, k)] = t
        busy[(piv, k)] = t
    return zeroed
