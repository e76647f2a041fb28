"""GPU: mixed-precision trailing updates (FP32 / BF16 MFMA, FP64 storage and
FP64 panels) and iterative refinement of least squares to FP64 accuracy.

Bounds (u = unit roundoff of the update precision: FP32 2^-24, BF16 2^-8):
* The reflectors are generated in FP64 from the tiles as they are, so the
  computed Q stays orthonormal to FP64 level: ||Q^T Q - I||_F <= 50 n eps.
* Each update C <- C - V T^T V^T C perturbs C by about u ||C|| per rounded
  operand (V, C, W, T, W' and the FP32 accumulation over k rows, which adds
  at most k 2^-24 relative); a column of A meets at most p + q updates, and
  the perturbations are independent roundings, so the backward error
  ||A - QR||_F / ||A||_F stays below 4 sqrt(p + q) (6 u + nb 2^-24).  It must
  also exceed 50 n eps: an FP64 result there would mean the low-precision
  path did not run.
* Refined least squares: backward error eta <= 1e-12.  A backward error
  eta (relative to ||A||_F) moves the solution of a square system by at
  most kappa_2(A) eta ||A||_F / ||A||_2 relative, so two solutions with
  eta <= 1e-12 differ by at most 2 kappa_2 1e-12 ||A||_F / ||A||_2.
"""

import sys

import numpy as np
import pytest

import tqr_inputs
from oracle import dag, tiled, trees

pytestmark = pytest.mark.gpu
EPS = np.finfo(np.float64).eps
U = {1: 2.0 ** -24, 2: 2.0 ** -8}
NAME = {1: "f32", 2: "bf16"}


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


def _bound(upd, p, q, nb):
    return 4.0 * np.sqrt(p + q) * (6 * U[upd] + nb * 2.0 ** -24)


CASES = [
    # (m, n, nb, tree, bs, kernels)
    (256, 128, 32, trees.GREEDY, 1, dag.KERN_TT),
    (256, 128, 32, trees.FLAT, 1, dag.KERN_TS),
    (512, 256, 64, trees.BINARY, 1, dag.KERN_TT),
    (512, 512, 128, trees.FIBONACCI, 1, dag.KERN_TT),
    (1024, 512, 256, trees.GREEDY, 1, dag.KERN_TT),
    (1024, 512, 256, trees.FLAT, 1, dag.KERN_TS),
    (1024, 768, 256, trees.PLASMA, 2, dag.KERN_TT),
]


@pytest.mark.parametrize("upd", [1, 2])
@pytest.mark.parametrize("case", CASES)
def test_mixed_factor_bounds(torch_cuda, case, upd):
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    m, n, nb, tree, bs, kern = case
    _say("mixed %s %dx%d nb %d tree %d bs %d kernels %d" % (NAME[upd], m, n, nb, tree, bs, kern))
    A = tqr_inputs.gaussian(m, n, 40 + m + n)
    F = tqr.factor(_gpu(torch, A), nb, tree, bs, kern, upd)
    R = F.R().cpu().numpy()
    Q = F.thin_q().cpu().numpy()
    orth = np.linalg.norm(Q.T @ Q - np.eye(n))
    back = np.linalg.norm(A - Q @ R) / np.linalg.norm(A)
    p, q = m // nb, n // nb
    bound = _bound(upd, p, q, nb)
    _say("  ||Q^TQ-I|| %.2e  ||A-QR||/||A|| %.2e  (bound %.2e)" % (orth, back, bound))
    assert orth <= 50 * n * EPS
    assert back <= bound
    if q > 1:
        assert back > 50 * n * EPS, "no sign of low-precision updates"
    # R against the FP64 oracle: the same factorization up to the update
    # perturbation, amplified by at most the condition number of A.
    Ro = tiled.tiled_qr(A, nb, tree, bs, kern).R()
    kappa = np.linalg.cond(A)
    dR = np.linalg.norm(R - Ro) / np.linalg.norm(Ro)
    assert dR <= 10 * kappa * bound, dR


# method: 0 auto (semi-normal corrections while they contract fast, then
# classical), 1 classical, 3 semi-normal only.
@pytest.mark.parametrize("upd,kappa,method", [(1, 1e2, 0), (1, 1e6, 0), (2, 1e2, 0), (1, 1e2, 1), (1, 1e6, 1),
                                              (1, 1e2, 3), (2, 1e2, 3)])
def test_mixed_refined_lstsq_matches_oracle(torch_cuda, upd, kappa, method):
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    n, nb, nrhs = 512, 64, 4
    _say("mixed refined lstsq %s n %d kappa %g method %d" % (NAME[upd], n, kappa, method))
    A = tqr_inputs.conditioned(n, kappa, 51, 52)
    rng = np.random.default_rng(53)
    B = A @ rng.standard_normal((n, nrhs))
    F = tqr.factor(_gpu(torch, A), nb, trees.GREEDY, 1, dag.KERN_DEFAULT, upd)
    X, info = F.lstsq(_gpu(torch, B), A0=_gpu(torch, A), tol=1e-12, method=method, raise_on_noconv=True)
    X = X.cpu().numpy()
    eta = tiled.backward_error(A, X, B)
    O = tiled.tiled_qr(A, nb, trees.GREEDY, 1)
    Xo = tiled.lstsq(O, B)
    fwd = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
    _say("  iters %d backward %.2e (oracle's %.2e)  ||x - x_oracle||/||x_oracle|| %.2e"
         % (info["iters"], max(eta), info["backward_err"], fwd))
    assert info["converged"]
    assert max(eta) <= 1e-12
    s = np.linalg.svd(A, compute_uv=False)
    assert fwd <= 2 * (s[0] / s[-1]) * 1e-12 * np.linalg.norm(A) / s[0]


@pytest.mark.parametrize("upd", [1, 2])
def test_mixed_full_size_square(torch_cuda, upd):
    """10240 x 10240 (40 x 40 tiles of 256), kappa 1e2, 4 right-hand sides:
    refined to 1e-12 and agreeing with the FP64 GPU solution (the oracle is
    too slow at this size; both solutions are checked against x_true)."""
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    n, nb, nrhs, kappa = 10240, 256, 4, 1e2
    _say("mixed full size %s n %d" % (NAME[upd], n))
    A = tqr_inputs.conditioned_device(n, kappa, tqr_inputs.SEED_C3, tqr_inputs.SEED_C3 + 1, "cuda").t()
    g = torch.Generator(device="cuda")
    g.manual_seed(tqr_inputs.SEED_C3_RHS)
    Xt = torch.randn((nrhs, n), generator=g, dtype=torch.float64, device="cuda").t()
    B = (A @ Xt).t().contiguous().t()
    F64 = tqr.factor(A, nb, trees.GREEDY, 1, dag.KERN_DEFAULT, 0)
    X64, _ = F64.lstsq(B)
    del F64
    F = tqr.factor(A, nb, trees.GREEDY, 1, dag.KERN_DEFAULT, upd)
    X, info = F.lstsq(B, A0=A, tol=1e-12, raise_on_noconv=True)
    r = B - A @ X
    eta = (torch.linalg.norm(r, dim=0) /
           (torch.linalg.norm(A) * torch.linalg.norm(X, dim=0) + torch.linalg.norm(B, dim=0))).max().item()
    d64 = (torch.linalg.norm(X - X64) / torch.linalg.norm(X64)).item()
    dtrue = (torch.linalg.norm(X - Xt) / torch.linalg.norm(Xt)).item()
    _say("  iters %d backward %.2e  vs fp64 %.2e  vs x_true %.2e" % (info["iters"], eta, d64, dtrue))
    assert info["converged"] and eta <= 1e-12
    # sigma_max = 1 and sigma_min = 1 / kappa by construction
    bound = 2 * kappa * 1e-12 * torch.linalg.norm(A).item()
    assert d64 <= bound and dtrue <= bound


def _tall_conditioned(m, n, kappa, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = kappa ** (-np.arange(n) / (n - 1))
    return (U * s) @ V.T


@pytest.mark.parametrize("upd,kappa", [(0, 1e4), (1, 1e2), (1, 1e4), (2, 1e2)])
def test_tall_augmented_refinement_matches_oracle(torch_cuda, upd, kappa):
    """Tall least squares (2048 x 512, nb 64, an inconsistent right-hand
    side): augmented-system refinement reaches a backward error of 1e-12
    and the solution agrees with the FP64 oracle within the least-squares
    perturbation bound 10 (kappa + kappa^2 ||r|| / (||A|| ||x||)) 1e-12."""
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    m, n, nb, nrhs = 2048, 512, 64, 3
    _say("tall augmented %s kappa %g" % (NAME.get(upd, "f64"), kappa))
    A = _tall_conditioned(m, n, kappa, 61)
    rng = np.random.default_rng(62)
    B = A @ rng.standard_normal((n, nrhs)) + 1e-3 * rng.standard_normal((m, nrhs))
    F = tqr.factor(_gpu(torch, A), nb, trees.GREEDY, 1, dag.KERN_DEFAULT, upd)
    X, info = F.lstsq(_gpu(torch, B), A0=_gpu(torch, A), tol=1e-12, raise_on_noconv=True)
    X = X.cpu().numpy()
    eta = tiled.backward_error(A, X, B)
    Xo = tiled.lstsq(tiled.tiled_qr(A, nb, trees.GREEDY, 1), B)
    fwd = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
    r = B - A @ Xo
    bound = 10 * (kappa + kappa ** 2 * np.linalg.norm(r) / (np.linalg.norm(A, 2) * np.linalg.norm(Xo))) * 1e-12
    _say("  iters %d backward %.2e (ls %.2e)  ||x - x_oracle||/||x_oracle|| %.2e (bound %.2e)"
         % (info["iters"], info["backward_err"], max(eta), fwd, bound))
    assert info["converged"] and info["backward_err"] <= 1e-12
    assert fwd <= bound
