"""Measurement sweeps on the current GPU, printed as Markdown tables.

  python -m paper_1104_4475_amd.measure trees    [--m 16384 --n 2048 --nb 256 --upd 0 --ts]
      every reduction tree (PlasmaTree with BS 1..64) on an N(0,1) matrix:
      executor time against the critical path of the task graph (Sec. 2.3)
      in Table 1 units and in measured time (each kind weighted by its
      mean measured duration from the executor trace); --upd selects the
      update precision (0 FP64, 1 FP32, 2 BF16), --ts adds every tree with
      TS kernels at its leaves
  python -m paper_1104_4475_amd.measure batched  [--count 512 --tree 5 --bs 16 --kern 2]
      the batched launch of tall-skinny problems, FP64 and FP32 updates,
      with a per-kind breakdown of one traced run of each (default tree:
      PlasmaTree BS=16 with TS kernels)
  python -m paper_1104_4475_amd.measure batched-trees  [--count 512]
      the same batch under each tree and kernel family of BATCH_TREES
  python -m paper_1104_4475_amd.measure batched-tune  [--count 512]
      the batch autotuner (trees x tile-size rules) on the same batch
  python -m paper_1104_4475_amd.measure complex
      the double-complex tiled QR (nb = 32) of square matrices, three trees
"""

import argparse
import sys

import numpy as np

from . import _lib, trace
from .api import Batch, factor

KIND = ["GEQRT", "UNMQR", "TSQRT", "TSMQR", "TTQRT", "TTMQR"]


def _cp(tasks, ptr, idx, w):
    fin = np.zeros(len(tasks))
    for t in range(len(tasks)):
        s = 0.0
        for e in range(ptr[t], ptr[t + 1]):
            s = max(s, fin[idx[e]])
        fin[t] = s + w[tasks[t, 0]]
    return fin.max() if len(fin) else 0.0


def trees(m, n, nb, reps=3, upd=0, ts=False):
    import torch
    p, q = m // nb, n // nb
    g = torch.Generator(device="cuda")
    g.manual_seed(1)
    A = torch.randn((n, m), generator=g, dtype=torch.float64, device="cuda").t()
    cases = [("FlatTree (TS)", _lib.TREE_FLAT, 1, _lib.KERN_TS), ("Sameh-Kuck (TT flat)", _lib.TREE_SAMEH_KUCK, 1,
                                                                  _lib.KERN_TT),
             ("BinaryTree", _lib.TREE_BINARY, 1, _lib.KERN_TT), ("Fibonacci", _lib.TREE_FIBONACCI, 1, _lib.KERN_TT),
             ("Greedy", _lib.TREE_GREEDY, 1, _lib.KERN_TT)]
    cases += [("PlasmaTree BS=%d" % bs, _lib.TREE_PLASMA, bs, _lib.KERN_TT) for bs in (1, 2, 4, 8, 16, 32, 64)
              if bs <= p]
    if ts:
        cases += [(name.replace(" (TT flat)", "") + " + TS", tree, bs, _lib.KERN_TS) for name, tree, bs, kern in cases
                  if kern == _lib.KERN_TT and tree not in (_lib.TREE_FLAT, _lib.TREE_SAMEH_KUCK)]
    flops = 2.0 * m * n * n - 2.0 * n ** 3 / 3.0
    print("| tree | tasks | CP (units) | makespan (ms) | GFLOP/s | CP with measured task times (ms) | makespan / CP |")
    print("|---|---|---|---|---|---|---|")
    for name, tree, bs, kern in cases:
        tasks, cp_units = _lib.schedule(p, q, tree, bs, kern)
        ptr, idx = _lib.task_preds(p, q, tree, bs, kern)
        F = factor(A, nb, tree, bs, kern, upd)
        F.sync()
        best = np.inf
        for _ in range(reps):
            F.refactor(A)
            F.sync()
            best = min(best, F.exec_ms())
        F.set_trace(True)
        F.refactor(A)
        F.sync()
        tr, rate = F.trace()
        tr = np.asarray(tr)
        dur = (tr[:, 8] - tr[:, 7]) * 1e3 / rate  # ms per subtask
        w = np.zeros(6)
        for k in range(6):
            sel = tr[:, 0] == k
            if sel.any():
                # a task's column slabs run side by side: its time is one
                # slab's; a panel task split into inner-block subtasks (slab =
                # block index) takes the sum of its blocks
                w[k] = dur[sel].mean()
                if k in (0, 2, 4) and tr[sel, 5].min() >= 0:
                    w[k] *= tr[sel, 5].max() + 1
        cpt = _cp(tasks, ptr, idx, w)
        print("| %s | %d | %d | %.2f | %.0f | %.2f | %.2f |" % (name, len(tasks), cp_units, best, flops / best / 1e6,
                                                                cpt, best / cpt if cpt > 0 else float("nan")))
        sys.stdout.flush()
        del F


BATCH_TREES = [("Greedy, TT kernels", _lib.TREE_GREEDY, 1, _lib.KERN_TT),
               ("Greedy, TS kernels", _lib.TREE_GREEDY, 1, _lib.KERN_TS),
               ("PlasmaTree BS=4, TS", _lib.TREE_PLASMA, 4, _lib.KERN_TS),
               ("PlasmaTree BS=8, TS", _lib.TREE_PLASMA, 8, _lib.KERN_TS),
               ("PlasmaTree BS=16, TS", _lib.TREE_PLASMA, 16, _lib.KERN_TS),
               ("PlasmaTree BS=16, TT", _lib.TREE_PLASMA, 16, _lib.KERN_TT),
               ("FlatTree, TS", _lib.TREE_FLAT, 1, _lib.KERN_TS)]
# The best tree above again with nb = 32 for every problem (instead of 64
# for n = 64 and 128).
BATCH_NB32 = ("PlasmaTree BS=16, TS, nb = 32 throughout", _lib.TREE_PLASMA, 16, _lib.KERN_TS)


def batched_tune(count, seed=6):
    """The batch autotuner (api.tune_batch) on the batch: every candidate
    tree and tile-size rule, FP64 updates; prints the table and the pick."""
    from .api import tune_batch
    _, mats = _batch_inputs(count, seed)
    names = {v: k for k, v in vars(_lib).items() if k.startswith("TREE_")}
    best, table = tune_batch(mats)
    print("| tile sizes | tree | BS | kernels | graph time (ms) |")
    print("|---|---|---|---|---|")
    for ms, rule, tree, bs, kern in sorted(table):
        print("| %s | %s | %d | %s | %.2f |" % (rule, names.get(tree, tree), bs, "TS" if kern == _lib.KERN_TS else "TT", ms))
    print()
    print("pick: %s, %s BS=%d, %s kernels, %.2f ms" % (best[1], names.get(best[2], best[2]), best[3],
                                                       "TS" if best[4] == _lib.KERN_TS else "TT", best[0]))


def batched_trees(count, seed=6, reps=3):
    """Graph time of the batch for each tree and kernel family of
    BATCH_TREES (FP64 updates)."""
    shapes, mats = _batch_inputs(count, seed)
    flops = sum(2.0 * m * n * n - 2.0 * n ** 3 / 3.0 for m, n, _ in shapes)
    print("| tree | problems | graph time (ms) | GFLOP/s |")
    print("|---|---|---|---|")
    for name, tree, bs, kern in BATCH_TREES + [BATCH_NB32]:
        nbs = [32 if name == BATCH_NB32[0] else nb for _, _, nb in shapes]
        B = Batch([(m, n) for m, n, _ in shapes], nbs, tree=tree, bs=bs, kernels=kern)
        ts = []
        for _ in range(reps + 1):
            B.run(mats)
            B.sync()
            ts.append(B.time_ms())
        t = min(ts[1:])
        print("| %s | %d | %.2f | %.0f |" % (name, count, t, flops / t / 1e6))
        sys.stdout.flush()
        del B


def _batch_inputs(count, seed):
    import torch
    rng = np.random.default_rng(seed)
    shapes = []
    for _ in range(count):
        nn = int(rng.choice([32, 64, 128]))
        nb = 32 if nn == 32 else 64
        u = int(rng.integers(1024, 16385))
        shapes.append((max(nb * int(round(u / nb)), nn), nn, nb))
    mats = []
    for i, (m, n, nb) in enumerate(shapes):
        g = torch.Generator(device="cuda")
        g.manual_seed(1000 + i)
        mats.append(torch.randn((n, m), generator=g, dtype=torch.float64, device="cuda").t())
    return shapes, mats


def batched(count, seed=6, tree=_lib.TREE_PLASMA, bs=16, kern=_lib.KERN_TS):
    shapes, mats = _batch_inputs(count, seed)
    flops = sum(2.0 * m * n * n - 2.0 * n ** 3 / 3.0 for m, n, _ in shapes)
    print("| updates | problems | total flops | graph time (ms) | GFLOP/s |")
    print("|---|---|---|---|---|")
    summaries = []
    for upd, name in ((0, "FP64"), (1, "FP32")):
        B = Batch([(m, n) for m, n, _ in shapes], [nb for _, _, nb in shapes], tree=tree, bs=bs, kernels=kern, upd=upd)
        ts = []
        for _ in range(4):
            B.run(mats)
            B.sync()
            ts.append(B.time_ms())
        t = min(ts[1:])
        print("| %s | %d | %.3e | %.2f | %.0f |" % (name, count, flops, t, flops / t / 1e6))
        sys.stdout.flush()
        # one traced run for the per-kind breakdown (printed after the table)
        B.set_trace(True)
        B.run(mats)
        B.sync()
        tr, rate = B.trace()
        summaries.append((name, B.time_ms(), trace.summarize(tr, rate)))
        del B
    for name, ms, s in summaries:
        print()
        print("%s updates, traced run (%.2f ms graph): %d subtasks on %d workgroups, executor makespan %.2f ms, "
              "workgroups busy %.1f%%, waiting for predecessors %.1f%%"
              % (name, ms, s["subtasks"], s["workgroups"], s["makespan_us"] / 1e3, 100 * s["utilization"],
                 100 * s["wait_us"] / max(1e-9, s["workgroups"] * s["makespan_us"])))
        print()
        print("| kind | subtasks | mean (us) | max (us) | total (ms) | share of busy time | mean wait (us) |")
        print("|---|---|---|---|---|---|---|")
        for k, v in sorted(s["kinds"].items(), key=lambda kv: -kv[1]["total_us"]):
            print("| %s | %d | %.2f | %.2f | %.2f | %.1f%% | %.2f |" % (
                k, v["count"], v["mean_us"], v["max_us"], v["total_us"] / 1e3, 100 * v["total_us"] / s["busy_us"],
                v["mean_wait_us"]))
        sys.stdout.flush()


def complex_qr(sizes=(2048, 4096, 8192), reps=3):
    """Double-complex tiled QR (nb = 32) of square N(0,1) + i N(0,1)
    matrices: pack + factorization time (HIP events, best of reps after one
    warm-up) for three trees; complex flops = 4 (2 m n^2 - 2 n^3 / 3)."""
    import torch
    from .api import zfactor
    cases = [("Greedy, TT", _lib.TREE_GREEDY, 1, _lib.KERN_TT), ("FlatTree, TS", _lib.TREE_FLAT, 1, _lib.KERN_TS),
             ("PlasmaTree BS=16, TS", _lib.TREE_PLASMA, 16, _lib.KERN_TS)]
    print("| n | tree | time (ms) | GFLOP/s (real flops) |")
    print("|---|---|---|---|")
    for n in sizes:
        g = torch.Generator(device="cuda")
        g.manual_seed(3)
        A = torch.complex(torch.randn((n, n), generator=g, dtype=torch.float64, device="cuda"),
                          torch.randn((n, n), generator=g, dtype=torch.float64, device="cuda")).t()
        flops = 4.0 * (2.0 * n ** 3 - 2.0 * n ** 3 / 3.0)
        for name, tree, bs, kern in cases:
            F = zfactor(A, 32, tree, bs, kern)
            F.sync()
            best = float("inf")
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                F.refactor(A)
                e1.record()
                F.sync()
                best = min(best, e0.elapsed_time(e1))
            print("| %d | %s | %.2f | %.0f |" % (n, name, best, flops / best / 1e6))
            sys.stdout.flush()
            del F


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["trees", "batched", "batched-trees", "batched-tune", "complex"])
    ap.add_argument("--m", type=int, default=16384)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--nb", type=int, default=256)
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--upd", type=int, default=0)
    ap.add_argument("--ts", action="store_true")
    ap.add_argument("--tree", type=int, default=_lib.TREE_PLASMA)
    ap.add_argument("--bs", type=int, default=16)
    ap.add_argument("--kern", type=int, default=_lib.KERN_TS)
    a = ap.parse_args(argv)
    if a.what == "trees":
        trees(a.m, a.n, a.nb, upd=a.upd, ts=a.ts)
    elif a.what == "batched-trees":
        batched_trees(a.count)
    elif a.what == "batched-tune":
        batched_tune(a.count)
    elif a.what == "complex":
        complex_qr()
    else:
        batched(a.count, tree=a.tree, bs=a.bs, kern=a.kern)
    return 0


if __name__ == "__main__":
    sys.exit(main())
