"""GPU: the batched persistent launch (one graph-captured executor over many
problems' task graphs).

Every subtask of the factorization is deterministic (no atomics in the
arithmetic), so a problem factored inside a batch must give bit-identical
tiles and Householder scalars to the same problem factored alone, whatever
the interleaving with other problems.  A few problems are also checked
against the FP64 oracle within 50 n eps ||A||_F elementwise.
"""

import sys

import numpy as np
import pytest

import tqr_inputs
from oracle import tiled, trees

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


def _dev(torch, m, n, seed):
    """Column-major N(0,1) matrix on the GPU (device generator)."""
    return tqr_inputs.gaussian_device(m, n, seed).t()


def _same_as_single(torch, tqr, Fb, A, nb, tree, upd):
    Fs = tqr.factor(A, nb, tree, 1, tqr.KERN_DEFAULT, upd)
    Pb, Ps = Fb.packed(), Fs.packed()
    tb, ts = Fb.tau(), Fs.tau()
    torch.cuda.synchronize()
    return bool(torch.equal(Pb, Ps)) and all(bool(torch.equal(x, y)) for x, y in zip(tb, ts))


SMALL = [(256, 32, 32), (512, 64, 64), (320, 64, 32), (1024, 128, 64), (64, 64, 64), (96, 32, 32),
         (2048, 128, 64), (192, 128, 64), (640, 64, 32), (128, 128, 32), (4096, 32, 32), (256, 128, 64)]


@pytest.mark.parametrize("upd", [0, 1])
def test_small_batch_bit_exact_with_single_calls(torch_cuda, upd):
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    _say("batched small, upd %d" % upd)
    mats = [_dev(torch, m, n, 100 + i) for i, (m, n, nb) in enumerate(SMALL)]
    Fs = tqr.factor_batched(mats, [nb for _, _, nb in SMALL], tqr.TREE_GREEDY, 1, tqr.KERN_DEFAULT, upd)
    for i, ((m, n, nb), A, F) in enumerate(zip(SMALL, mats, Fs)):
        assert _same_as_single(torch, tqr, F, A, nb, tqr.TREE_GREEDY, upd), "problem %d (%d x %d nb %d)" % (i, m, n, nb)


def test_small_batch_matches_oracle(torch_cuda):
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    _say("batched vs oracle")
    shapes = [(256, 64, 32), (320, 128, 64), (512, 32, 32)]
    host = [tqr_inputs.gaussian(m, n, 200 + i) for i, (m, n, nb) in enumerate(shapes)]
    mats = [torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t() for A in host]
    Fs = tqr.factor_batched(mats, [nb for _, _, nb in shapes], tqr.TREE_FIBONACCI)
    for (m, n, nb), A, F in zip(shapes, host, Fs):
        O = tiled.tiled_qr(A, nb, trees.FIBONACCI, 1)
        err = np.max(np.abs(F.packed().cpu().numpy() - O.A))
        assert err <= 50 * n * EPS * np.linalg.norm(A), err


def test_graph_replays(torch_cuda):
    """The captured graph replayed on three different input sets, with eager
    work and synchronization between replays: every replay matches single
    calls bit for bit."""
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    _say("batched graph replays")
    shapes = SMALL[:8]
    B = tqr.Batch([(m, n) for m, n, _ in shapes], [nb for _, _, nb in shapes])
    for rep in range(3):
        mats = [_dev(torch, m, n, 300 + 17 * rep + i) for i, (m, n, nb) in enumerate(shapes)]
        B.run(mats)
        B.sync()
        _ = (mats[0] * 2.0).sum().item()  # eager work between replays
        for i, ((m, n, nb), A) in enumerate(zip(shapes, mats)):
            assert _same_as_single(torch, tqr, B.factors(i), A, nb, tqr.TREE_GREEDY, 0), (rep, i)
    assert B.time_ms() > 0


# (tree, BS, kernel family): the default Greedy/TT and the batch
# autotuner's pick, PlasmaTree BS=16 with TS kernels.
FULL_TREES = [(4, 1, 1), (5, 16, 2)]


@pytest.mark.parametrize("tree,bs,kern", FULL_TREES, ids=["greedy_tt", "plasma16_ts"])
@pytest.mark.parametrize("upd", [0, 1])
def test_full_batch_512(torch_cuda, upd, tree, bs, kern):
    """512 tall-skinny problems: m uniform in [1024, 16384] rounded to nb,
    n in {32, 64, 128}, nb = 32 for n = 32 else 64.  Sampled problems are
    bit-exact with single calls; every problem's R has the column norms of
    A (||R e_j|| = ||A e_j||, orthogonal invariance)."""
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    _say("batched 512, upd %d, tree %d bs %d kernels %d" % (upd, tree, bs, kern))
    shapes = tqr_inputs.batched_shapes(512, tqr_inputs.SEED_BATCH)
    mats = [_dev(torch, m, n, 1000 + i) for i, (m, n, nb) in enumerate(shapes)]
    B = tqr.Batch([(m, n) for m, n, _ in shapes], [nb for _, _, nb in shapes], tree=tree, bs=bs, kernels=kern,
                  upd=upd)
    B.run(mats)
    B.sync()
    _say("  batch run %.2f ms" % B.time_ms())
    for i in range(0, 512, 37):
        m, n, nb = shapes[i]
        b = min(bs, m // nb) if tree == tqr.TREE_PLASMA else bs
        Fs = tqr.factor(mats[i], nb, tree, b, kern, upd)
        Pb, Ps = B.factors(i).packed(), Fs.packed()
        tb, ts = B.factors(i).tau(), Fs.tau()
        torch.cuda.synchronize()
        assert bool(torch.equal(Pb, Ps)) and all(bool(torch.equal(x, y)) for x, y in zip(tb, ts)), i
    tol = 1e-13 if upd == 0 else 1e-5
    for i in range(512):
        R = B.factors(i).R()
        cn = torch.linalg.norm(mats[i], dim=0)
        rel = ((torch.linalg.norm(R, dim=0) - cn).abs() / cn).max().item()
        assert rel <= tol, (i, rel)


def test_batch_trace_respects_each_problems_dag(torch_cuda):
    """Tracing a batch (switched on after the graph was captured): every
    subtask of the merged order is traced once with its problem index, the
    subtasks of problem i are those of its own executor plan, and each became
    ready only after all its predecessors in that plan ended.  Switching the
    trace off again leaves the results unchanged."""
    import paper_1104_4475_amd as tqr
    from paper_1104_4475_amd import _lib
    torch = torch_cuda
    _say("batched trace")
    shapes = SMALL
    B = tqr.Batch([(m, n) for m, n, _ in shapes], [nb for _, _, nb in shapes])
    mats = [_dev(torch, m, n, 700 + i) for i, (m, n, nb) in enumerate(shapes)]
    B.run(mats)
    B.sync()
    B.set_trace(True)
    B.run(mats)
    B.sync()
    tr, rate = B.trace()
    assert rate > 0 and tr.shape[1] == 11
    ticket, ready, end = tr[:, 6], tr[:, 7], tr[:, 8]
    assert np.all(ticket > 0) and np.all(ready >= ticket) and np.all(end >= ready)
    assert np.array_equal(np.sort(np.unique(tr[:, 10])), np.arange(len(shapes)))
    total = 0
    for i in range(len(shapes)):
        rows = np.nonzero(tr[:, 10] == i)[0]
        sub, deps = B.factors(i).exec_plan()
        assert len(rows) == len(sub), i
        total += len(sub)
        where = {tuple(int(x) for x in tr[r, :6]): r for r in rows}
        assert len(where) == len(rows)
        pos = [where[tuple(int(x) for x in sub[t, :6])] for t in range(len(sub))]
        for t in range(len(sub)):
            e = deps[sub[t, 6]:sub[t, 7]]
            assert np.all((e & ~_lib.DEP_INDEX) == 0)  # nb <= 64: whole-task waits only
            for d in e:
                assert end[pos[d]] <= ready[pos[t]], (i, t, int(d))
    assert total == len(tr)
    B.set_trace(False)
    B.run(mats)
    B.sync()
    for i, ((m, n, nb), A) in enumerate(zip(shapes, mats)):
        assert _same_as_single(torch, tqr, B.factors(i), A, nb, tqr.TREE_GREEDY, 0), i


def test_batch_autotuner_picks_its_fastest_and_runs_it(torch_cuda):
    """The batch autotuner times every candidate (tree, BS, kernel family)
    under every tile-size rule; its pick is the fastest entry of its own
    table, and a batch built with the pick factors each problem bit for bit
    as a single call with the same options."""
    import paper_1104_4475_amd as tqr
    from paper_1104_4475_amd.api import batch_nb_rules
    torch = torch_cuda
    _say("batch autotuner")
    shapes = [(512, 64), (1024, 128), (256, 32), (768, 64), (2048, 128), (384, 32)]
    mats = [_dev(torch, m, n, 900 + i) for i, (m, n) in enumerate(shapes)]
    rules = batch_nb_rules(shapes)
    assert rules["nb 32"] == [32] * len(shapes)
    assert rules["nb 64 where it divides"] == [64, 64, 32, 64, 64, 32]
    best, table = tqr.tune_batch(mats, reps=1)
    assert len(table) == len(rules) * len(tqr.BATCH_CANDIDATES)
    assert best[0] == min(t[0] for t in table)
    ms, rule, tree, bs, kern, nbs = best
    B = tqr.Batch(shapes, nbs, tree=tree, bs=bs, kernels=kern)
    B.run(mats)
    B.sync()
    for i in (0, 1, 2):
        m, n = shapes[i]
        Fs = tqr.factor(mats[i], nbs[i], tree, min(bs, m // nbs[i]) if tree == tqr.TREE_PLASMA else bs, kern, 0)
        Pb, Ps = B.factors(i).packed(), Fs.packed()
        torch.cuda.synchronize()
        assert bool(torch.equal(Pb, Ps)), (i, best)
