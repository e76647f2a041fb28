"""Oracle pins for the FP64 MLP: central finite differences for every
gradient, and the closed form of Adam's first step."""

import numpy as np

from oracle import mlp


def _data(n=17, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, mlp.N_IN))
    t = rng.standard_normal(n)
    return X, t


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    P = mlp.init_params(rng)
    for k in P:  # non-zero biases so every term is exercised
        if k.startswith("b"):
            P[k] = 0.1 * rng.standard_normal(P[k].shape)
    X, t = _data()
    _, g = mlp.loss_and_grad(P, X, t)
    h = 1e-6
    for k in P:
        flat = P[k].reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp, _ = mlp.loss_and_grad(P, X, t)
            flat[i] = old - h
            lm, _ = mlp.loss_and_grad(P, X, t)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].reshape(-1)[i]) <= 1e-6 * max(1.0, abs(fd)), (k, i)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    P = mlp.init_params(rng)
    X, t = _data()
    _, g = mlp.loss_and_grad(P, X, t)
    before = {k: v.copy() for k, v in P.items()}
    state = {}
    lr, eps = 1e-2, 1e-8
    mlp.adam_step(P, g, state, lr=lr, eps=eps)
    for k in P:
        want = before[k] - lr * g[k] / (np.abs(g[k]) + eps)
        assert np.allclose(P[k], want, rtol=1e-12, atol=1e-15)


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    P = mlp.init_params(rng)
    X, _ = _data(200, 4)
    t = np.sin(X[:, 0]) + 0.5 * X[:, 3]
    state = {}
    l0, _ = mlp.loss_and_grad(P, X, t)
    for _ in range(300):
        _, g = mlp.loss_and_grad(P, X, t)
        mlp.adam_step(P, g, state, lr=3e-3)
    l1, _ = mlp.loss_and_grad(P, X, t)
    assert l1 < 0.2 * l0


def test_features_layout():
    x = mlp.features(64, 8, 256, mlp.ALGO_PLASMA, mlp.KERN_TS, 4, 2)
    assert x.shape == (13,)
    assert list(x[:3]) == [6.0, 3.0, 8.0]
    assert x[3 + mlp.ALGO_PLASMA] == 1.0 and x[8] == 1.0 and x[9] == 2.0 and x[12] == 1.0
    assert x.sum() == 6 + 3 + 8 + 1 + 1 + 2 + 1
    y = mlp.features(64, 8, 256, mlp.ALGO_GREEDY, mlp.KERN_TT, 1, 0)
    assert y[3 + mlp.ALGO_GREEDY] == 1.0 and y[8] == 0.0 and y[9] == 0.0 and y[10] == 1.0


def test_selector_features_match_the_oracle():
    """The selector's feature encoding is the oracle's, for every candidate
    of a few shapes."""
    from paper_1104_4475_amd import selector
    for m, n in ((2048, 512), (4096, 4096), (8192, 1024)):
        cands = selector.candidates(m, n)
        assert cands and {c[1] for c in cands} == set(range(5)) and {c[2] for c in cands} == {0, 1}
        for nb, algo, kern, bs in cands:
            assert np.array_equal(selector.features(m // nb, n // nb, nb, algo, kern, bs, 1),
                                  mlp.features(m // nb, n // nb, nb, algo, kern, bs, 1).astype(np.float32))
