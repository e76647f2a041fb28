"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.  This module holds none of the factorization's arithmetic: it only
draws matrices and problem-size lists from fixed seeds.

Host generators use numpy.random.default_rng(seed) and return FP64 arrays in
Fortran (column-major) order.  The device generators use a seeded
torch.Generator on the GPU for the large benchmark inputs, where drawing and
orthogonalizing on the host would take minutes; they are never compared
element by element with host draws.

Recipes
-------
gaussian(m, n, seed)            entries i.i.d. N(0, 1).
haar(n, seed)                   Haar-distributed orthogonal matrix: the Q of a
                                QR of an N(0,1) matrix with its columns
                                multiplied by sign(diag R) (Mezzadri 2007).
conditioned(n, kappa, seeds)    A = U diag(s) V^T with U, V Haar and
                                s_i = kappa^{-(i-1)/(n-1)}, so that
                                sigma_max = 1 and sigma_min = 1/kappa.
batched_shapes(count, seed)     tall-skinny batch: n uniform on {32, 64, 128},
                                m = nb * round(U / nb) with U an integer
                                uniform on [1024, 16384], nb = 32 if n = 32
                                else 64.
"""

import numpy as np

SEED_C1, SEED_C2, SEED_C3 = 0, 1, 2
SEED_C3_RHS = 5
SEED_BATCH = 6


def gaussian(m, n, seed):
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((m, n)))


def haar(n, seed):
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def singular_values(n, kappa):
    if n == 1:
        return np.ones(1)
    return kappa ** (-np.arange(n) / (n - 1.0))


def conditioned(n, kappa, seed_u, seed_v):
    U = haar(n, seed_u)
    V = haar(n, seed_v)
    s = singular_values(n, kappa)
    return np.asfortranarray((U * s) @ V.T)


def batched_shapes(count, seed, lo=1024, hi=16384):
    """List of (m, n, nb) for the tall-skinny batch."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice([32, 64, 128]))
        nb = 32 if n == 32 else 64
        u = int(rng.integers(lo, hi + 1))
        m = max(nb * int(round(u / nb)), n)
        out.append((m, n, nb))
    return out


# ---- device generators (large benchmark inputs) -------------------------

def gaussian_device(m, n, seed, device="cuda"):
    """Column-major FP64 N(0,1) matrix on the GPU: returns a torch tensor of
    shape (n, m) whose row c is column c of A (so its storage is A in
    column-major order with lda = m)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return torch.randn((n, m), generator=g, dtype=torch.float64, device=device)


def haar_device(n, seed, device="cuda"):
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    Z = torch.randn((n, n), generator=g, dtype=torch.float64, device=device)
    Q, R = torch.linalg.qr(Z)
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1.0
    return Q * d


def conditioned_device(n, kappa, seed_u, seed_v, device="cuda"):
    """A = U diag(s) V^T on the GPU; returned transposed like gaussian_device
    (row c of the result is column c of A)."""
    import torch
    U = haar_device(n, seed_u, device)
    V = haar_device(n, seed_v, device)
    s = torch.as_tensor(singular_values(n, kappa), device=device)
    A = (U * s) @ V.T
    return A.T.contiguous()
