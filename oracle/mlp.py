"""FP64 multilayer perceptron for the makespan model of the tree / tile-size
selector (oracle; test infrastructure only).

The paper picks PlasmaTree's domain size by exhaustive search (Sec. 4) and
has no learned model; this is the reference for the project's selector, which
predicts log(makespan) of a candidate (p, q, nb, tree, BS, update precision)
and picks the argmin.

Network: 13 inputs -> 64 -> 64 -> 1, ReLU hidden units, linear output, mean
squared error loss, Adam (Kingma & Ba 2015, with bias correction).

Features (13): log2 p, log2 q, log2 nb; one-hot of five trees (FlatTree,
BinaryTree, Fibonacci, Greedy, PlasmaTree); the kernel family (1 for TS
kernels, 0 for TT); log2 BS for PlasmaTree (0 otherwise); one-hot of three
update precisions (FP64, FP32, BF16).

Parity: gradients pinned by central finite differences; the Adam step by its
closed form on the first iteration (tests/test_oracle_mlp.py).
"""

import numpy as np

N_IN, N_HID = 13, 64
ALGO_FLAT, ALGO_BINARY, ALGO_FIB, ALGO_GREEDY, ALGO_PLASMA = range(5)
KERN_TT, KERN_TS = 0, 1


def features(p, q, nb, algo, kern, bs, prec):
    x = np.zeros(N_IN)
    x[0] = np.log2(p)
    x[1] = np.log2(q)
    x[2] = np.log2(nb)
    x[3 + algo] = 1.0
    x[8] = float(kern)
    x[9] = np.log2(bs) if algo == ALGO_PLASMA else 0.0
    x[10 + prec] = 1.0
    return x


def init_params(rng):
    """He-style initialisation from a numpy Generator."""
    def lin(fan_in, fan_out):
        return rng.standard_normal((fan_in, fan_out)) * np.sqrt(2.0 / fan_in)
    return {"W1": lin(N_IN, N_HID), "b1": np.zeros(N_HID),
            "W2": lin(N_HID, N_HID), "b2": np.zeros(N_HID),
            "W3": lin(N_HID, 1), "b3": np.zeros(1)}


def forward(P, X):
    z1 = X @ P["W1"] + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"] + P["b2"]
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ P["W3"] + P["b3"])[:, 0]
    return y, (X, z1, h1, z2, h2)


def loss_and_grad(P, X, t):
    """MSE loss mean((y - t)^2) and its gradient with respect to every
    parameter."""
    y, (X, z1, h1, z2, h2) = forward(P, X)
    n = X.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = (2.0 / n) * r[:, None]
    g = {"W3": h2.T @ dy, "b3": dy.sum(0)}
    dh2 = dy @ P["W3"].T
    dz2 = dh2 * (z2 > 0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ P["W2"].T
    dz1 = dh1 * (z1 > 0)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(0)
    return loss, g


def adam_step(P, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; state holds m, v and the step count."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in P:
        m = state.setdefault("m_" + k, np.zeros_like(P[k]))
        v = state.setdefault("v_" + k, np.zeros_like(P[k]))
        m *= b1
        m += (1 - b1) * g[k]
        v *= b2
        v += (1 - b2) * g[k] * g[k]
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        P[k] -= lr * mh / (np.sqrt(vh) + eps)
