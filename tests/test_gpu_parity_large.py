"""GPU parity at the full task-graph shapes, the executor's dispatch order,
and the triangular solves.

* Elementwise FP64 parity with the oracle on the tile grids of the tall
  (64 x 8 tiles) and square (40 x 40 tiles) workloads, with tiles of 32 so
  that the oracle finishes in seconds: thousands of subtasks run at once
  across the chip, as at the full sizes.
* At the full sizes (16384 x 2048 and 10240 x 10240, tiles of 256), where the
  oracle is too slow, the factorization bounds ||A - QR||_F / ||A||_F and
  ||Q^T Q - I||_F <= 50 n eps computed on the GPU.
* The executor trace: every subtask became ready only after each of its
  predecessors (its own dependency list, and every edge of the oracle's task
  DAG) had finished.
* R^{-1} X and R^{-T} X against LAPACK's triangular solve on the same R, at
  tile sizes whose solves split a tile row over 1, 2 and 4 workgroups.
"""

import sys

import numpy as np
import pytest
from scipy.linalg import solve_triangular

import tqr_inputs
from oracle import dag, tiled, trees

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _gpu(torch, A):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A, dtype=np.float64).T)).cuda().t()


GRIDS = [
    # (m, n, nb, tree, bs, kernels): tall grid 64 x 8, square grid 40 x 40
    (2048, 256, 32, trees.GREEDY, 1, dag.KERN_TT),
    (2048, 256, 32, trees.FLAT, 1, dag.KERN_TS),
    (2048, 256, 32, trees.PLASMA, 8, dag.KERN_TS),
    (1280, 1280, 32, trees.GREEDY, 1, dag.KERN_TT),
    (1280, 1280, 32, trees.PLASMA, 16, dag.KERN_TS),
]


@pytest.mark.parametrize("case", GRIDS, ids=lambda c: "%dx%d_nb%d_t%d_bs%d_k%d" % c)
def test_large_grid_parity(torch_cuda, case):
    import paper_1104_4475_amd as tqr
    m, n, nb, tree, bs, kern = case
    _say("large grid %s" % (case,))
    A = tqr_inputs.gaussian(m, n, seed=81 + m // nb + n // nb)
    F = tqr.factor(_gpu(torch_cuda, A), nb, tree, bs, kern)
    F.sync()
    O = tiled.tiled_qr(A, nb, tree, bs, kern)
    tol = 50 * n * EPS * np.linalg.norm(A)
    err = np.max(np.abs(F.packed().cpu().numpy() - O.A))
    _say("  max |packed - oracle| %.2e (tol %.2e)" % (err, tol))
    assert err <= tol
    _compare_tau(F, O, nb)


def _compare_tau(F, O, nb):
    """Householder scalars against the oracle.  With the dlarfg convention a
    reflector I - tau [1; v][1; v]^T is orthogonal iff tau = 2 / (1 + v^T v)
    (or tau = 0, v = 0), so tau follows from the stored v with sensitivity
    |d tau| <= tau^2 ||v|| ||dv||: the bound uses the measured difference dv
    of the stored reflector (compared elementwise above)."""
    P = F.packed().cpu().numpy()
    tg, tp = [t.cpu().numpy() for t in F.tau()]

    def vec(M, r, c, j, kind):
        T = M[(r - 1) * nb:r * nb, (c - 1) * nb:c * nb]
        if kind == "ge":
            return T[j + 1:, j]
        if kind == "tt":
            return T[:j + 1, j]
        return T[:, j]

    def check(tau_g, tau_o, r, c, kind):
        for j in range(nb):
            vg, vo = vec(P, r, c, j, kind), vec(O.A, r, c, j, kind)
            if tau_o[j] == 0.0:
                assert tau_g[j] == 0.0, (kind, r, c, j)
                continue
            # rounding of tau, of v and of the sum v^T v (nb terms): about
            # (nb + 16) eps tau
            rnd = (nb + 16) * EPS * tau_o[j]
            # the GPU's own consistency: tau = 2 / (1 + v^T v)
            assert abs(tau_g[j] - 2.0 / (1.0 + vg @ vg)) <= rnd, (kind, r, c, j)
            dv = np.linalg.norm(vg - vo)
            bound = tau_o[j] ** 2 * (2 * np.linalg.norm(vo) * dv + dv ** 2) + 2 * rnd
            assert abs(tau_g[j] - tau_o[j]) <= bound, (kind, r, c, j, tau_g[j] - tau_o[j], bound)

    for (r, c), tau in O.tau_g.items():
        check(tg[c - 1, r - 1], tau, r, c, "ge")
    kinds = {}
    for (kind, i, piv, k, j) in O.tasks:
        if kind in (dag.TSQRT, dag.TTQRT):
            kinds[(i, k)] = "tt" if kind == dag.TTQRT else "ts"
    for (i, c), tau in O.tau_p.items():
        check(tp[c - 1, i - 1], tau, i, c, kinds[(i, c)])


FULL = [
    (16384, 2048, trees.GREEDY, 1, dag.KERN_TT),
    (10240, 10240, trees.PLASMA, 16, dag.KERN_TS),
]


@pytest.mark.parametrize("case", FULL, ids=lambda c: "%dx%d_t%d_bs%d_k%d" % c)
def test_full_size_fp64_bounds(torch_cuda, case):
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    m, n, tree, bs, kern = case
    nb = 256
    _say("full size fp64 %s" % (case,))
    A = tqr_inputs.gaussian_device(m, n, 91, "cuda").t()
    F = tqr.factor(A, nb, tree, bs, kern)
    F.sync()
    R = F.R()
    QR = torch.zeros((n, m), dtype=torch.float64, device="cuda").t()
    QR[:n] = R
    QR = F.apply_q(QR, "N")
    res = (torch.linalg.norm(A - QR) / torch.linalg.norm(A)).item()
    del QR
    Q = F.thin_q()
    G = Q.T @ Q
    G.diagonal().sub_(1.0)
    orth = torch.linalg.norm(G).item()
    del Q, G
    _say("  ||A-QR||/||A|| %.2e  ||Q^TQ-I|| %.2e  (bound %.2e)" % (res, orth, 50 * n * EPS))
    assert res <= 50 * n * EPS
    assert orth <= 50 * n * EPS


def _task_key(kind, i, piv, k, j):
    """Identity of a task of the DAG (0-based tiles, unused fields dropped)."""
    if kind == dag.GEQRT:
        return (kind, i, k)
    if kind == dag.UNMQR:
        return (kind, i, k, j)
    if kind in (dag.TSQRT, dag.TTQRT):
        return (kind, i, piv, k)
    return (kind, i, piv, k, j)


TRACE_CASES = [
    # (m, n, nb, tree, bs, kernels)
    (256, 128, 32, trees.GREEDY, 1, dag.KERN_TT),
    (512, 384, 64, trees.FIBONACCI, 1, dag.KERN_TT),
    (1024, 512, 128, trees.BINARY, 1, dag.KERN_TS),
    (1536, 1024, 256, trees.PLASMA, 2, dag.KERN_TS),
    (2048, 1024, 256, trees.GREEDY, 1, dag.KERN_TT),
    (2560, 2560, 256, trees.FLAT, 1, dag.KERN_TS),
]


@pytest.mark.parametrize("upd", [0, 1])
@pytest.mark.parametrize("case", TRACE_CASES, ids=lambda c: "%dx%d_nb%d_t%d_bs%d_k%d" % c)
def test_executor_trace_respects_dag(torch_cuda, case, upd):
    import paper_1104_4475_amd as tqr
    m, n, nb, tree, bs, kern = case
    _say("trace order %s upd %d" % (case, upd))
    A = _gpu(torch_cuda, tqr_inputs.gaussian(m, n, seed=95))
    F = tqr.factor(A, nb, tree, bs, kern, upd)
    F.sync()
    F.set_trace(True)
    F.refactor(A)
    F.sync()
    tr, _ = F.trace()
    sub, deps = F.exec_plan()
    from paper_1104_4475_amd import _lib
    assert len(tr) == len(sub)
    assert np.array_equal(tr[:, :6], sub[:, :6].astype(np.int64))
    ticket, ready, end = tr[:, 6], tr[:, 7], tr[:, 8]
    assert np.all(ticket > 0) and np.all(ready >= ticket) and np.all(end >= ready)
    # 1. the executor's own subtask dependencies
    streamed = set()  # (predecessor subtask, successor subtask) not waited for in full at the start
    nearly = 0
    for t in range(len(sub)):
        e = deps[sub[t, 6]:sub[t, 7]]
        if len(e):
            d = e & _lib.DEP_INDEX
            stage = (e >> _lib.DEP_STAGE_SHIFT) & 3
            early = (e & _lib.DEP_EARLY) != 0
            assert np.all(d < t) and np.all(stage < 3)
            plain = (stage == 0) & ~early
            late = end[d[plain]] > ready[t]
            assert not late.any(), ("subtask", t, "ready before predecessors", d[plain][late])
            # an early release comes after the predecessor started; a wait
            # inside a panel block subtask makes it end after the predecessor
            assert np.all(ready[d[early]] <= ready[t]), ("subtask", t, "ready before an early predecessor started")
            assert np.all(end[d[stage > 0]] <= end[t]), ("subtask", t, "ended before a predecessor waited inside")
            if (stage > 0).any():
                assert sub[t, 0] in (0, 2, 4) and sub[t, 5] >= 0
            streamed.update((int(u), t) for u in d[~plain])
            nearly += int(early.sum())
    # 1b. streamed predecessors (FP32 / BF16 updates at nb >= 128): an update
    # applies panel block b after that block's flag (or early release), so it
    # ends after every streamed panel block started (and, without early
    # release, after it ended); it ends after its C1 writer started.
    nblk = nb // 32
    for t in range(len(sub)):
        if sub[t, 9] >= 0:
            pe = deps[sub[t, 9]:sub[t, 9] + nblk]
            pb = pe & _lib.DEP_INDEX
            assert np.all(pb < t)
            whole = (pe & _lib.DEP_EARLY) == 0
            assert np.all(end[pb[whole]] <= end[t]), ("subtask", t, "ended before a streamed panel block")
            assert np.all(ready[pb] <= end[t]), ("subtask", t, "ended before a streamed panel block started")
            streamed.update((int(u), t) for u in pb)
        if sub[t, 8] >= 0:
            u = int(sub[t, 8])
            assert u < t and ready[u] <= end[t]
            streamed.add((u, t))
    if nb < 128:
        assert not streamed
    else:
        assert nearly > 0  # panel block subtasks release early at nb >= 128
    if upd == 0:
        assert (sub[:, 8:] < 0).all()  # FP64 updates wait for whole predecessors
    # 2. every edge of the oracle's task DAG: each subtask of a task became
    # ready after some subtask of each predecessor task had finished
    p, q = m // nb, n // nb
    kf = dag.resolve_kernels(tree, kern)
    tasks, preds = dag.build_tasks(p, q, trees.elim_list(p, q, tree, bs), kf)
    subs_of = {}
    for t in range(len(sub)):
        kind, i, piv, k, j = (int(x) for x in sub[t, :5])
        subs_of.setdefault(_task_key(kind, i, piv, k, j), []).append(t)
    keys = []
    for (kind, i, piv, k, j) in tasks:
        keys.append(_task_key(kind, i - 1, piv - 1 if piv else 0, k - 1, j - 1 if j else 0))
    assert set(keys) == set(subs_of), "executor tasks differ from the oracle's DAG"
    first_end = {key: end[v].min() for key, v in subs_of.items()}
    first_ready = {key: ready[v].min() for key, v in subs_of.items()}
    task_of = {}
    for key, v in subs_of.items():
        for t in v:
            task_of[t] = key
    streamed_tasks = {(task_of[u], task_of[t]) for u, t in streamed}
    for v, pv in enumerate(preds):
        rv = ready[subs_of[keys[v]]]
        for u in pv:
            if (keys[u], keys[v]) in streamed_tasks:
                # followed block by block: v cannot end before u has started
                assert first_ready[keys[u]] <= end[subs_of[keys[v]]].max(), ("streamed edge", tasks[u], tasks[v])
                continue
            assert first_end[keys[u]] <= rv.min(), ("DAG edge violated", tasks[u], tasks[v])


SOLVE_CASES = [(1024, 512, 64), (1024, 512, 128), (1024, 768, 256)]


@pytest.mark.parametrize("m,n,nb", SOLVE_CASES)
def test_triangular_solves_match_lapack(torch_cuda, m, n, nb):
    """R^{-1} X and R^{-T} X (one, two and four workgroups per tile row at
    nb 64, 128, 256) against LAPACK's trtrs on the same R: the difference is
    bounded by kappa(R) n eps relative (a backward-stable solve each)."""
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    _say("triangular solves %dx%d nb %d" % (m, n, nb))
    A = tqr_inputs.gaussian(m, n, seed=101 + nb)
    F = tqr.factor(_gpu(torch, A), nb, trees.GREEDY, 1, dag.KERN_TT)
    F.sync()
    R = F.R().cpu().numpy()
    kappa = np.linalg.cond(R)
    Y = tqr_inputs.gaussian(n, 5, seed=102)
    for trans in ("N", "T"):
        got = F.solve_r(_gpu(torch, Y), trans).cpu().numpy()
        want = solve_triangular(R, Y, trans=0 if trans == "N" else 1, lower=False)
        err = np.linalg.norm(got - want) / np.linalg.norm(want)
        _say("  trans %s: rel diff %.2e (kappa %.1e, bound %.2e)" % (trans, err, kappa, 10 * kappa * n * EPS))
        assert err <= 10 * kappa * n * EPS
    # unrefined least squares through the same solves, against the oracle
    B = tqr_inputs.gaussian(m, 3, seed=103)
    X, info = F.lstsq(_gpu(torch, B))
    Xo = tiled.lstsq(tiled.tiled_qr(A, nb, trees.GREEDY, 1), B)
    err = np.linalg.norm(X.cpu().numpy() - Xo) / np.linalg.norm(Xo)
    assert err <= 10 * kappa * n * EPS, err


def test_batch_rerun_refreshes_solve_tables(torch_cuda):
    """A batch replayed on new matrices: least squares on a problem's handle
    (no refinement) must use the new factors' triangular-solve tables."""
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    _say("batch re-run then lstsq")
    shapes, nbs = [(512, 128), (768, 64)], [64, 32]
    bt = tqr.Batch(shapes, nbs)
    for rnd in range(2):
        mats = [tqr_inputs.gaussian(m, n, seed=110 + 10 * rnd + i) for i, (m, n) in enumerate(shapes)]
        bt.run([_gpu(torch, A) for A in mats])
        bt.sync()
        for i, (A, nb) in enumerate(zip(mats, nbs)):
            B = tqr_inputs.gaussian(A.shape[0], 2, seed=120 + 10 * rnd + i)
            X, _ = bt.factors(i).lstsq(_gpu(torch, B))
            Xo = tiled.lstsq(tiled.tiled_qr(A, nb, trees.GREEDY, 1), B)
            err = np.max(np.abs(X.cpu().numpy() - Xo)) / np.max(np.abs(Xo))
            _say("  run %d problem %d: max rel diff %.2e" % (rnd, i, err))
            assert err <= 1e-11


STREAM_CASES = [
    # (m, n, nb, tree, bs, kernels, upd): long TS chains, TT merges, both tile sizes
    (2560, 2560, 256, trees.FLAT, 1, dag.KERN_TS, 1),
    (2048, 1024, 256, trees.PLASMA, 4, dag.KERN_TS, 2),
    (2048, 1280, 256, trees.GREEDY, 1, dag.KERN_TT, 1),
    (1536, 1024, 128, trees.FLAT, 1, dag.KERN_TS, 2),
]


@pytest.mark.parametrize("case", STREAM_CASES, ids=lambda c: "%dx%d_nb%d_t%d_bs%d_k%d_u%d" % c)
def test_streamed_factors_bit_identical(torch_cuda, case, monkeypatch):
    """Updates that follow their reflectors and C1 writers block by block do
    the same arithmetic as updates that wait for whole predecessors, so the
    factors must agree bit for bit (a read of C1 rows or of a reflector block
    before its writer finished would show up here)."""
    import paper_1104_4475_amd as tqr
    m, n, nb, tree, bs, kern, upd = case
    _say("streamed vs whole-predecessor %s" % (case,))
    A = _gpu(torch_cuda, tqr_inputs.gaussian(m, n, seed=97))
    out = []
    for stream in ("0", "1"):
        monkeypatch.setenv("TQR_STREAM", stream)
        F = tqr.factor(A, nb, tree, bs, kern, upd)
        F.sync()
        sub, _ = F.exec_plan()
        assert (sub[:, 8:] >= 0).any() == (stream == "1")
        for _ in range(2):
            F.refactor(A)
            F.sync()
            out.append(F.packed().cpu().numpy())
    for P in out[1:]:
        assert np.array_equal(P.view(np.uint64), out[0].view(np.uint64))


EARLY_CASES = [
    # (m, n, nb, tree, bs, kernels, upd): TS chains, TT merges, GEQRT-only
    # columns, every update precision and both split tile sizes
    (2560, 2560, 256, trees.FLAT, 1, dag.KERN_TS, 1),
    (2048, 1024, 256, trees.PLASMA, 4, dag.KERN_TS, 0),
    (2048, 1280, 256, trees.GREEDY, 1, dag.KERN_TT, 2),
    (1536, 1024, 128, trees.HADRI, 3, dag.KERN_TS, 1),
    (1024, 1024, 128, trees.BINARY, 1, dag.KERN_TT, 0),
]


@pytest.mark.parametrize("case", EARLY_CASES, ids=lambda c: "%dx%d_nb%d_t%d_bs%d_k%d_u%d" % c)
def test_early_release_bit_identical(torch_cuda, case, monkeypatch):
    """Panel block subtasks that release their successors after the
    look-ahead (and wait for the rest of their predecessors inside) do the
    same arithmetic in the same order on every tile element as subtasks
    that wait for whole predecessors: the factors must agree bit for bit.
    So must the plain bottom-level dispatch order and the level-synchronous
    executor (which runs the same plan level by level)."""
    import paper_1104_4475_amd as tqr
    from paper_1104_4475_amd import _lib
    m, n, nb, tree, bs, kern, upd = case
    _say("early release vs whole blocks %s" % (case,))
    A = _gpu(torch_cuda, tqr_inputs.gaussian(m, n, seed=98))
    out = []
    for early, path, order in (("0", "persistent", "sim"), ("1", "persistent", "sim"), ("1", "persistent", "bl"),
                               ("1", "level", "sim")):
        monkeypatch.setenv("TQR_EARLY", early)
        monkeypatch.setenv("TQR_EXEC", path)
        monkeypatch.setenv("TQR_ORDER", order)
        F = tqr.factor(A, nb, tree, bs, kern, upd)
        F.sync()
        sub, deps = F.exec_plan()
        assert ((deps & _lib.DEP_EARLY) != 0).any() == (early == "1")
        for _ in range(2 if path == "persistent" else 1):
            F.refactor(A)
            F.sync()
            out.append(F.packed().cpu().numpy())
        del F
    for P in out[1:]:
        assert np.array_equal(P.view(np.uint64), out[0].view(np.uint64))
