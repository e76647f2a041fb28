"""Autotuner and learned selector of the reduction tree, kernel family,
PlasmaTree domain size and tile size.

The paper tunes PlasmaTree's domain size BS by exhaustive search over
measured runs (Sec. 4).  Here the exhaustive autotuner times every candidate
(nb, tree, kernel family, BS) of a shape on the GPU; the learned selector
instead predicts log(makespan) of every candidate with a small multilayer
perceptron (13 -> 64 -> 64 -> 1, trained on timings of the GPU executor) and
picks the argmin, so a shape can be tuned without running its candidates.
The network's forward pass, gradient and Adam step are the library's HIP
kernels (tiledqr_mlp_*); this module only encodes features and drives the
loops.

Trees (feature one-hot order): FlatTree, BinaryTree, Fibonacci, Greedy,
PlasmaTree (with BS).  Kernel family: TT, or TS (TS kernels where the tree
allows them: FlatTree with TS kernels is Sameh-Kuck's TS scheme, the other
trees take TS kernels inside their flat chains and TT at the merges).
"""

import csv
import ctypes
import math
import os
import time

import numpy as np

from . import _lib
from ._lib import check

N_IN = 13
ALGOS = ["flat", "binary", "fibonacci", "greedy", "plasma"]
ALGO_TREE = [_lib.TREE_FLAT, _lib.TREE_BINARY, _lib.TREE_FIBONACCI, _lib.TREE_GREEDY, _lib.TREE_PLASMA]
KERNS = [_lib.KERN_TT, _lib.KERN_TS]  # feature 8: 0 = TT, 1 = TS
PLASMA = 4
PRECS = ["f64", "f32", "bf16"]
NBS = (64, 128, 256)
MAX_TILES = 64  # candidates keep p <= MAX_TILES (the host plan of larger grids takes seconds)
CORPUS_FIELDS = ["p", "q", "nb", "algo", "kern", "bs", "prec", "ms"]


def features(p, q, nb, algo, kern, bs, prec):
    """13 features of a candidate: log2 p, log2 q, log2 nb, one-hot tree
    (5), kernel family (1 = TS), log2 BS for PlasmaTree else 0, one-hot
    update precision (3)."""
    x = np.zeros(N_IN, dtype=np.float32)
    x[0] = math.log2(p)
    x[1] = math.log2(q)
    x[2] = math.log2(nb)
    x[3 + algo] = 1.0
    x[8] = float(kern)
    x[9] = math.log2(bs) if algo == PLASMA else 0.0
    x[10 + prec] = 1.0
    return x


def candidates(m, n, nbs=NBS, max_tiles=MAX_TILES):
    """Every (nb, tree, family, bs) for an m x n matrix: tile sizes dividing
    both dimensions with q <= p <= max_tiles, the four fixed trees and
    PlasmaTree with every power-of-two BS up to p, each with TT and with TS
    kernels."""
    out = []
    for nb in nbs:
        if m % nb or n % nb:
            continue
        p, q = m // nb, n // nb
        if p < q or p > max_tiles:
            continue
        for kern in (0, 1):
            for algo in range(PLASMA):
                out.append((nb, algo, kern, 1))
            bs = 1
            while bs <= p:
                out.append((nb, PLASMA, kern, bs))
                bs *= 2
    return out


def flops(m, n):
    return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0


class Timer:
    """Times factorizations with the executor's own kernel time (HIP events
    around the persistent launch), reusing one input per shape."""

    def __init__(self, seed=0):
        import torch
        self.torch = torch
        self.seed = seed
        self._mats = {}

    def matrix(self, m, n):
        key = (m, n)
        if key not in self._mats:
            if len(self._mats) > 4:
                self._mats.clear()
            g = self.torch.Generator(device="cuda")
            g.manual_seed(self.seed + 7 * m + n)
            self._mats[key] = self.torch.randn((n, m), generator=g, dtype=self.torch.float64, device="cuda").t()
        return self._mats[key]

    def time(self, m, n, nb, algo, kern, bs, prec, reps=1):
        from .api import factor
        A = self.matrix(m, n)
        F = factor(A, nb, ALGO_TREE[algo], bs, KERNS[kern], prec)
        F.sync()
        best = math.inf
        for _ in range(reps):
            F.refactor(A)
            F.sync()
            best = min(best, F.exec_ms())
        del F
        return best


def collect_corpus(path, count, seed=0, flop_cap=6e11, log=None):
    """Time `count` random candidates (p log-uniform in [1, MAX_TILES], q
    log-uniform in [1, p], nb in {64, 128, 256}, tree, family and BS
    uniform, precision uniform) and append them to a CSV file."""
    rng = np.random.default_rng(seed)
    timer = Timer(seed)
    new = not os.path.exists(path)
    with open(path, "a", newline="") as fh:
        w = csv.writer(fh)
        if new:
            w.writerow(CORPUS_FIELDS)
        done = 0
        while done < count:
            p = int(round(2 ** rng.uniform(0, math.log2(MAX_TILES))))
            q = int(round(2 ** rng.uniform(0, math.log2(p)))) if p > 1 else 1
            q = max(1, min(q, p))
            nb = int(rng.choice(NBS))
            if flops(p * nb, q * nb) > flop_cap:
                continue
            algo = int(rng.integers(0, len(ALGOS)))
            kern = int(rng.integers(0, 2))
            bs = int(2 ** rng.integers(0, int(math.log2(p)) + 1)) if algo == PLASMA else 1
            prec = int(rng.integers(0, 3))
            ms = timer.time(p * nb, q * nb, nb, algo, kern, bs, prec)
            w.writerow([p, q, nb, algo, kern, bs, prec, "%.5f" % ms])
            fh.flush()
            done += 1
            if log and done % 100 == 0:
                log("corpus %d / %d" % (done, count))


def exhaustive(m, n, prec, timer, nbs=NBS):
    """The exhaustive autotuner: {(nb, algo, kern, bs): ms} for every
    candidate."""
    return {c: timer.time(m, n, c[0], c[1], c[2], c[3], prec) for c in candidates(m, n, nbs)}


def heldout_shapes(count, seed, step=512, mmax=8192):
    """Held-out (m, n, precision) triples: m, n multiples of step with
    n <= m <= mmax."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        m = step * int(rng.integers(1, mmax // step + 1))
        n = step * int(rng.integers(1, m // step + 1))
        out.append((m, n, int(rng.integers(0, 3))))
    return out


def load_csv(path):
    with open(path) as fh:
        return list(csv.DictReader(fh))


class MakespanModel:
    """The 13 -> 64 -> 64 -> 1 perceptron, parameters and Adam state in FP32
    device memory, trained and evaluated by the library's kernels."""

    def __init__(self, seed=0):
        import torch
        self.torch = torch
        self.nparam = _lib.tiledqr_mlp_nparam()
        rng = np.random.default_rng(seed)
        P = np.zeros(self.nparam, dtype=np.float32)
        # He initialisation; biases zero.
        P[0:832] = rng.standard_normal(832) * math.sqrt(2.0 / 13)
        P[896:4992] = rng.standard_normal(4096) * math.sqrt(2.0 / 64)
        P[5056:5120] = rng.standard_normal(64) * math.sqrt(2.0 / 64)
        self.params = torch.from_numpy(P).cuda()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.step = 0

    @staticmethod
    def _stream():
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def loss_grad(self, X, t):
        check(_lib.tiledqr_mlp_loss_grad(self.params.data_ptr(), X.data_ptr(), t.data_ptr(), X.shape[0],
                                         self.grad.data_ptr(), self.loss.data_ptr(), self._stream()),
              "tiledqr_mlp_loss_grad")
        return self.loss, self.grad

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        check(_lib.tiledqr_mlp_adam(self.params.data_ptr(), self.grad.data_ptr(), self.m.data_ptr(),
                                    self.v.data_ptr(), self.nparam, lr, b1, b2, eps, self.step, self._stream()),
              "tiledqr_mlp_adam")

    def predict(self, X):
        torch = self.torch
        X = torch.as_tensor(X, dtype=torch.float32).cuda().contiguous()
        y = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        check(_lib.tiledqr_mlp_forward(self.params.data_ptr(), X.data_ptr(), X.shape[0], y.data_ptr(),
                                       self._stream()), "tiledqr_mlp_forward")
        return y

    def fit(self, X, t, epochs=2000, lr=3e-3, batch=512, seed=0, log=None):
        """Mini-batch Adam on (X, t); returns the final full-batch loss."""
        torch = self.torch
        X = torch.as_tensor(X, dtype=torch.float32).cuda().contiguous()
        t = torch.as_tensor(t, dtype=torch.float32).cuda().contiguous()
        n = X.shape[0]
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        for ep in range(epochs):
            perm = torch.randperm(n, generator=g, device="cuda")
            for b0 in range(0, n, batch):
                idx = perm[b0:b0 + batch]
                self.loss_grad(X[idx].contiguous(), t[idx].contiguous())
                self.adam(lr=lr)
            if log and (ep + 1) % max(1, epochs // 10) == 0:
                self.loss_grad(X, t)
                log("epoch %d loss %.4f" % (ep + 1, self.loss.item()))
        self.loss_grad(X, t)
        return self.loss.item()


def corpus_arrays(rows):
    X = np.stack([features(int(r["p"]), int(r["q"]), int(r["nb"]), int(r["algo"]), int(r["kern"]), int(r["bs"]),
                           int(r["prec"])) for r in rows])
    t = np.log(np.array([float(r["ms"]) for r in rows], dtype=np.float64)).astype(np.float32)
    return X, t


class Selector:
    """Picks the candidate with the smallest predicted makespan."""

    def __init__(self, model):
        self.model = model

    def choose(self, m, n, prec, nbs=NBS):
        cands = candidates(m, n, nbs)
        X = np.stack([features(m // nb, n // nb, nb, algo, kern, bs, prec) for nb, algo, kern, bs in cands])
        y = self.model.predict(X).cpu().numpy()
        return cands[int(np.argmin(y))]


def regret(table, choice):
    """t(choice) / t(best) - 1 over a measured candidate table."""
    best = min(table.values())
    return table[choice] / best - 1.0


def default_choice(m, n):
    """The choice without a selector: Greedy with TT kernels at the largest
    tile size that divides the matrix."""
    for nb in sorted(NBS, reverse=True):
        if m % nb == 0 and n % nb == 0 and n // nb <= m // nb <= MAX_TILES:
            return (nb, 3, 0, 1)
    raise ValueError("no tile size divides %d x %d" % (m, n))


def now():
    return time.strftime("%H:%M:%S")
