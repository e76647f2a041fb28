"""GPU: the selector's perceptron kernels (forward, loss gradient, Adam)
against the FP64 oracle, and the learned selector against the exhaustive
autotuner on held-out shapes.

Tolerances: the kernels compute in FP32; a dot product of length k carries
a relative error of at most about k 2^-24 of the sum of absolute terms, so
forward values and gradients are compared with a relative bound of 1e-4
against the largest magnitude, and the Adam step with 1e-5.
"""

import os
import sys

import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
DATA = os.path.join(os.path.dirname(HERE), "paper_1104_4475_amd", "data")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


KEYS = [("W1", 0, 832), ("b1", 832, 896), ("W2", 896, 4992), ("b2", 4992, 5056), ("W3", 5056, 5120),
        ("b3", 5120, 5121)]


def _flat(P):
    return np.concatenate([P[k].reshape(-1) for k, _, _ in KEYS]).astype(np.float32)


def _unflat(v):
    shapes = {"W1": (13, 64), "b1": (64,), "W2": (64, 64), "b2": (64,), "W3": (64, 1), "b3": (1,)}
    return {k: np.asarray(v[a:b], dtype=np.float64).reshape(shapes[k]) for k, a, b in KEYS}


def _model_with(torch, P):
    from paper_1104_4475_amd.selector import MakespanModel
    M = MakespanModel(0)
    M.params.copy_(torch.from_numpy(_flat(P)))
    return M


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = np.concatenate([rng.uniform(0, 7, (n, 3)), rng.integers(0, 2, (n, 10))], axis=1)
    t = rng.standard_normal(n)
    return X, t


def _params(seed):
    rng = np.random.default_rng(seed)
    P = omlp.init_params(rng)
    for k in P:
        if k.startswith("b"):
            P[k] = 0.1 * rng.standard_normal(P[k].shape)
    # FP32-representable so both sides start from the same numbers
    return _unflat(_flat(P))


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000])
def test_forward_and_gradient_match_oracle(torch_cuda, n):
    torch = torch_cuda
    _say("mlp gradient n=%d" % n)
    P = _params(3)
    X, t = _data(n, 4)
    X = X.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    M = _model_with(torch, P)
    y = M.predict(X).cpu().numpy()
    yo, _ = omlp.forward(P, X)
    assert np.max(np.abs(y - yo)) <= 1e-4 * max(1.0, np.max(np.abs(yo)))
    loss, grad = M.loss_grad(torch.from_numpy(X.astype(np.float32)).cuda(), torch.from_numpy(t.astype(np.float32)).cuda())
    lo, go = omlp.loss_and_grad(P, X, t)
    assert abs(loss.item() - lo) <= 1e-4 * max(1.0, lo)
    g = _unflat(grad.cpu().numpy())
    for k in go:
        scale = max(1e-6, np.max(np.abs(go[k])))
        assert np.max(np.abs(g[k] - go[k])) <= 1e-4 * scale, k


def test_adam_step_matches_oracle(torch_cuda):
    torch = torch_cuda
    _say("mlp adam")
    P = _params(5)
    X, t = _data(200, 6)
    X = X.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    M = _model_with(torch, P)
    state = {}
    for _ in range(3):
        _, go = omlp.loss_and_grad(P, X, t)
        omlp.adam_step(P, go, state, lr=1e-2)
        M.loss_grad(torch.from_numpy(X.astype(np.float32)).cuda(), torch.from_numpy(t.astype(np.float32)).cuda())
        M.adam(lr=1e-2)
    got = _unflat(M.params.cpu().numpy())
    for k in P:
        assert np.max(np.abs(got[k] - P[k])) <= 1e-5 * max(1.0, np.max(np.abs(P[k]))), k


def test_training_reduces_loss(torch_cuda):
    torch = torch_cuda
    _say("mlp training")
    from paper_1104_4475_amd.selector import MakespanModel
    rng = np.random.default_rng(7)
    X, _ = _data(2000, 8)
    t = 0.5 * X[:, 0] + 0.3 * X[:, 1] * X[:, 2] - X[:, 5] + 0.1 * rng.standard_normal(2000)
    M = MakespanModel(1)
    M.loss_grad(torch.from_numpy(X.astype(np.float32)).cuda(), torch.from_numpy(t.astype(np.float32)).cuda())
    l0 = M.loss.item()
    l1 = M.fit(X, t, epochs=60, lr=3e-3, batch=256)
    _say("  loss %.4f -> %.4f" % (l0, l1))
    assert l1 < 0.05 * l0


def _heldout_tables(path):
    from paper_1104_4475_amd import selector
    tables = {}
    for r in selector.load_csv(path):
        key = (int(r["shape"]), int(r["m"]), int(r["n"]), int(r["prec"]))
        tables.setdefault(key, {})[(int(r["nb"]), int(r["algo"]), int(r["kern"]), int(r["bs"]))] = float(r["ms"])
    return tables


@pytest.mark.skipif(not os.path.exists(os.path.join(DATA, "mi355x_heldout.csv")), reason="no held-out timings")
def test_selector_regret_against_exhaustive_autotuner(torch_cuda):
    """Train the network on the GPU timing corpus with the library's kernels,
    then pick a candidate for every held-out shape: the mean regret
    t(selected) / t(best exhaustive) - 1 must be at most 10%, and below the
    regret of the choice made without the selector (Greedy at the largest
    tile size)."""
    from paper_1104_4475_amd import selector
    _say("selector regret")
    rows = selector.load_csv(os.path.join(DATA, "mi355x_corpus.csv"))
    X, t = selector.corpus_arrays(rows)
    M = selector.MakespanModel(0)
    loss = M.fit(X, t, epochs=300, lr=2e-3, batch=256, seed=0)
    S = selector.Selector(M)
    reg, base = [], []
    for (sid, m, n, prec), table in sorted(_heldout_tables(os.path.join(DATA, "mi355x_heldout.csv")).items()):
        reg.append(selector.regret(table, S.choose(m, n, prec)))
        base.append(selector.regret(table, selector.default_choice(m, n)))
    reg, base = np.array(reg), np.array(base)
    _say("  corpus %d rows, train loss %.4f; %d held-out shapes: regret mean %.3f p90 %.3f max %.3f; "
         "without the selector mean %.3f" % (len(rows), loss, len(reg), reg.mean(), np.percentile(reg, 90),
                                             reg.max(), base.mean()))
    assert reg.mean() <= 0.10
    assert reg.mean() < base.mean()
