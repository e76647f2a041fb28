"""GPU: mixed-precision trailing updates (FP32 / BF16 MFMA, FP64 storage and
FP64 panels) and iterative refinement of least squares to FP64 accuracy.

Bounds (u = unit roundoff of the update precision: FP32 2^-24, BF16 2^-8):
* The reflectors are generated in FP64 from the tiles as they are, so the
  computed Q stays orthonormal to FP64 level: ||Q^T Q - I||_F <= 50 n eps.
* First-order model of the backward error of the factorization.  Each
  update rounds its operands once (relative error u) and accumulates inner
  products of up to nb terms in FP32 (a random walk of about sqrt(nb) 2^-24
  relative); a column of A meets about p + q updates whose errors are
  independent, so ||A - QR||_F / ||A||_F ~ c u_eff sqrt(p + q) with
  u_eff = u + sqrt(nb) 2^-24 and c of order one.  The tests require c in
  [C_LO, C_HI], a band about ten times wider than the measured spread on
  each side: a wrong precision (an FP64 or FP32 result in the BF16 mode, a
  BF16 one in the FP32 mode) or an operand error of a few u falls outside.
* R against the FP64 oracle, up to row signs (R is unique only up to the
  signs of its rows, and a perturbation of the update precision can flip the
  sign of a pivot that is close to zero): the computed R is the exact R of
  A - E with ||E||_F = back ||A||_F, and the first-order perturbation bound
  of the R factor (Sun 1991) gives ||dR||_F / ||R||_F <= sqrt(2) kappa_2(A)
  back.  C_R = 2 allows for second-order terms.  At BF16 the right-hand side
  is below one, so an update kernel with an error of a few percent fails.
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


def _model(upd, p, q, nb):
    return (U[upd] + np.sqrt(nb) * 2.0 ** -24) * np.sqrt(p + q)


# Band of the model constant c = backward error / model.  Measured on MI355X
# over the cases below: FP32 0.09 - 0.24, BF16 0.22 - 0.66.
C_LO, C_HI = 0.01, 2.5
C_R = 2.0


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
    c = back / _model(upd, p, q, nb)
    # R against the FP64 oracle: the same factorization up to the update
    # perturbation, amplified by at most about the condition number of A.
    Ro = tiled.tiled_qr(A, nb, tree, bs, kern).R()
    kappa = np.linalg.cond(A)
    sgn = np.sign(np.diag(R)) * np.sign(np.diag(Ro))
    flips = int(np.sum(sgn < 0))
    dR = np.linalg.norm(R * sgn[:, None] - Ro) / np.linalg.norm(Ro)
    cr = dR / (kappa * back)
    _say("  ||Q^TQ-I|| %.2e  ||A-QR||/||A|| %.2e  c %.3f  dR %.2e  dR/(kappa back) %.3f (kappa %.1f, "
         "%d row signs flipped)" % (orth, back, c, dR, cr, kappa, flips))
    assert orth <= 50 * n * EPS
    assert C_LO <= c <= C_HI, c
    assert dR <= C_R * kappa * back, cr


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


def test_refinement_six_rhs_reported_error_matches_oracle(torch_cuda):
    """Six right-hand sides (two passes of four through the residual and
    A^T r kernels) on a 384 x 384 system (a column chunk shorter than the
    residual kernel's).  With FP32 updates and a loose tolerance the solve
    stops at its first iterate, whose backward error (about 1e-7) is far
    above rounding level, so the reported error -- built from ||A||_F
    accumulated inside the first residual -- equals the oracle's backward
    error of the returned X to 1e-6 relative (a norm counted twice would be
    off by sqrt(2)); refined to 1e-12 afterwards."""
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    n, nb, nrhs = 384, 64, 6
    _say("refinement with %d right-hand sides, n %d" % (nrhs, n))
    A = tqr_inputs.conditioned(n, 1e2, 61, 62)
    B = A @ np.random.default_rng(63).standard_normal((n, nrhs))
    F = tqr.factor(_gpu(torch, A), nb, trees.GREEDY, 1, dag.KERN_DEFAULT, 1)
    X, info = F.lstsq(_gpu(torch, B), A0=_gpu(torch, A), tol=1e-3, method=3, raise_on_noconv=True)
    eta = max(tiled.backward_error(A, X.cpu().numpy(), B))
    _say("  first iterate: reported %.6e, oracle %.6e" % (info["backward_err"], eta))
    assert info["converged"] and eta > 1e-10
    assert abs(info["backward_err"] - eta) <= 1e-6 * eta
    X, info = F.lstsq(_gpu(torch, B), A0=_gpu(torch, A), tol=1e-12, method=0, raise_on_noconv=True)
    eta = max(tiled.backward_error(A, X.cpu().numpy(), B))
    _say("  refined: iters %d reported %.2e oracle %.2e" % (info["iters"], info["backward_err"], eta))
    assert info["converged"] and eta <= 1e-12


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


def _eta_lib(A, X, B):
    """The library's backward error of X: per column the smaller of the
    square-system value and ||A^T r|| / (||A||_F ||r||) for tall A."""
    nA = np.linalg.norm(A)
    R = B - A @ X
    out = []
    for c in range(X.shape[1]):
        r, x, b = R[:, c], X[:, c], B[:, c]
        e = np.linalg.norm(r) / (nA * np.linalg.norm(x) + np.linalg.norm(b))
        if A.shape[0] != A.shape[1] and np.linalg.norm(r) > 0:
            e = min(e, np.linalg.norm(A.T @ r) / (nA * np.linalg.norm(r)))
        out.append(e)
    return max(out)


# method: 0 auto (semi-normal corrections while they contract fourfold, then
# the augmented system), 2 augmented system only, 3 semi-normal only.
@pytest.mark.parametrize("upd,kappa,method", [(0, 1e4, 0), (1, 1e2, 0), (1, 1e4, 0), (2, 1e2, 0),
                                              (1, 1e2, 2), (1, 1e4, 2), (2, 1e2, 2), (0, 1e4, 3), (1, 1e2, 3)])
def test_tall_refinement_matches_oracle(torch_cuda, upd, kappa, method):
    """Tall least squares (2048 x 512, nb 64, an inconsistent right-hand
    side): refinement reaches a backward error of 1e-12, the solution agrees
    with the FP64 oracle within the least-squares perturbation bound
    10 (kappa + kappa^2 ||r|| / (||A|| ||x||)) 1e-12, and the corrections are
    of the kinds the method asks for."""
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    m, n, nb, nrhs = 2048, 512, 64, 3
    _say("tall refinement %s kappa %g method %d" % (NAME.get(upd, "f64"), kappa, method))
    A = _tall_conditioned(m, n, kappa, 61)
    rng = np.random.default_rng(62)
    B = A @ rng.standard_normal((n, nrhs)) + 1e-3 * rng.standard_normal((m, nrhs))
    F = tqr.factor(_gpu(torch, A), nb, trees.GREEDY, 1, dag.KERN_DEFAULT, upd)
    X, info = F.lstsq(_gpu(torch, B), A0=_gpu(torch, A), tol=1e-12, method=method, raise_on_noconv=True)
    X = X.cpu().numpy()
    eta = tiled.backward_error(A, X, B)
    Xo = tiled.lstsq(tiled.tiled_qr(A, nb, trees.GREEDY, 1), B)
    fwd = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
    r = B - A @ Xo
    bound = 10 * (kappa + kappa ** 2 * np.linalg.norm(r) / (np.linalg.norm(A, 2) * np.linalg.norm(Xo))) * 1e-12
    _say("  iters %d (semi-normal %d, augmented %d) backward %.2e (ls %.2e)  ||x - x_oracle||/||x_oracle|| %.2e "
         "(bound %.2e)" % (info["iters"], info["semi_normal"], info["augmented"], info["backward_err"], max(eta),
                           fwd, bound))
    assert info["converged"] and info["backward_err"] <= 1e-12
    assert fwd <= bound
    assert 0 <= info["semi_normal"] and 0 <= info["augmented"]
    assert info["semi_normal"] + info["augmented"] <= info["iters"] <= 30
    if method == 2:
        assert info["semi_normal"] == 0 and info["augmented"] == info["iters"]
    if method == 3:
        assert info["augmented"] == 0 and info["semi_normal"] == info["iters"]


@pytest.mark.parametrize("case", ["tall_bf16_seminormal", "square_bf16_kappa1e6"])
def test_nonconverged_returns_best_iterate(torch_cuda, case):
    """Where refinement cannot converge (BF16 updates at kappa 1e6: the
    perturbation of the factors exceeds sigma_min, for the semi-normal
    corrections of a tall system and the corrections of a square one), the
    call reports TQR_ENOTCONV and returns the iterate with the smallest
    backward error: the reported error is that of the returned X and is no
    larger than the unrefined solution's."""
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    _say("non-converged refinement %s" % case)
    if case.startswith("tall"):
        A = _tall_conditioned(2048, 512, 1e6, 61)
        rng = np.random.default_rng(62)
        B = A @ rng.standard_normal((512, 3)) + 1e-3 * rng.standard_normal((2048, 3))
        method = 3
    else:
        A = tqr_inputs.conditioned(512, 1e6, 51, 52)
        B = A @ np.random.default_rng(53).standard_normal((512, 3))
        method = 0
    F = tqr.factor(_gpu(torch, A), 64, trees.GREEDY, 1, dag.KERN_DEFAULT, 2)
    X0, _ = F.lstsq(_gpu(torch, B))
    e0 = _eta_lib(A, X0.cpu().numpy(), B)
    X, info = F.lstsq(_gpu(torch, B), A0=_gpu(torch, A), tol=1e-12, method=method)
    e = _eta_lib(A, X.cpu().numpy(), B)
    _say("  status %d iters %d: reported %.3e, of X %.3e, unrefined %.3e"
         % (info["status"], info["iters"], info["backward_err"], e, e0))
    assert info["status"] == tqr.TQR_ENOTCONV and not info["converged"]
    assert e == pytest.approx(info["backward_err"], rel=1e-6)
    assert e <= e0 * (1 + 1e-6)
