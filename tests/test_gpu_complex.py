"""GPU: the double-complex tiled QR (tiledqr_zfactor, nb = 32) against the
double-complex oracle (oracle.ztiled) on the same seeded inputs: the packed
factors (R and the reflectors) elementwise within 50 n eps ||A||_F, R's
diagonal exactly real, and the tau of every panel set (the tau of a short
reflector moves by |d alpha| / ||x||, hence its looser absolute bound)."""

import sys

import numpy as np
import pytest

import tqr_inputs
from oracle import dag, trees, ztiled

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


def _cplx(m, n, seed):
    return tqr_inputs.gaussian(m, n, seed) + 1j * tqr_inputs.gaussian(m, n, seed + 7919)


def _gpu(torch, A):
    return torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()


CASES = [
    # (m, n, tree, bs, kernels)
    (256, 128, trees.GREEDY, 1, dag.KERN_TT),
    (256, 128, trees.FLAT, 1, dag.KERN_TS),
    (320, 192, trees.FIBONACCI, 1, dag.KERN_TT),
    (512, 256, trees.PLASMA, 4, dag.KERN_TS),
    (256, 256, trees.BINARY, 1, dag.KERN_TT),
    (1024, 64, trees.GREEDY, 1, dag.KERN_TS),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%dx%d_t%d_bs%d_k%d" % c)
def test_complex_factors_match_oracle(torch_cuda, case):
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    m, n, tree, bs, kern = case
    _say("complex %s" % (case,))
    A = _cplx(m, n, 61)
    F = tqr.zfactor(_gpu(torch, A), 32, tree, bs, kern)
    F.sync()
    P = F.packed().cpu().numpy()
    O = ztiled.ztiled_qr(A, 32, tree, bs, kern)
    err = np.max(np.abs(P - O.A))
    assert err <= 50 * n * EPS * np.linalg.norm(A), err
    assert np.all(np.diag(P[:n, :n]).imag == 0.0)
    tg, tp = (t.cpu().numpy().reshape(n // 32, m // 32, 32) for t in F.tau())
    for (i, k), t in O.tau_g.items():
        assert np.max(np.abs(tg[k - 1, i - 1] - t)) <= 1e-12, ("taug", i, k)
    for (i, k), t in O.tau_p.items():
        assert np.max(np.abs(tp[k - 1, i - 1] - t)) <= 1e-12, ("taup", i, k)
    # the handle refactors a second matrix into the same storage
    A2 = _cplx(m, n, 64)
    F.refactor(_gpu(torch, A2))
    F.sync()
    O2 = ztiled.ztiled_qr(A2, 32, tree, bs, kern)
    assert np.max(np.abs(F.packed().cpu().numpy() - O2.A)) <= 50 * n * EPS * np.linalg.norm(A2)


def test_complex_real_input_stays_real_and_diagonal_matrix(torch_cuda):
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    _say("complex special cases")
    A = tqr_inputs.gaussian(128, 64, 62).astype(np.complex128)
    F = tqr.zfactor(_gpu(torch, A), 32, tqr.TREE_GREEDY, 1, tqr.KERN_TT)
    F.sync()
    P = F.packed().cpu().numpy()
    assert np.all(P.imag == 0.0)
    # diag(d): R = diag(-sign(Re d) |d|), the reflectors below are zero
    rng = np.random.default_rng(5)
    d = rng.standard_normal(64) + 1j * rng.standard_normal(64)
    d[3] = 2.0
    D = np.diag(d)
    F = tqr.zfactor(_gpu(torch, D), 32, tqr.TREE_FLAT, 1, tqr.KERN_TS)
    F.sync()
    R = F.packed().cpu().numpy()
    beta = -np.where(d.real >= 0.0, 1.0, -1.0) * np.abs(d)
    beta[3] = 2.0
    assert np.max(np.abs(np.diag(R) - beta)) <= 4 * EPS * np.abs(d).max()
    assert np.max(np.abs(R - np.diag(np.diag(R)))) == 0.0


def test_complex_tile_size_other_than_32_is_unsupported(torch_cuda):
    import paper_1104_4475_amd as tqr
    from paper_1104_4475_amd import _lib
    torch = torch_cuda
    A = _gpu(torch, _cplx(128, 64, 63))
    with pytest.raises(_lib.TiledQRError) as e:
        tqr.zfactor(A, 64)
    assert e.value.status == _lib.TQR_EUNSUPPORTED


@pytest.mark.parametrize("case", [(256, 128, trees.GREEDY, 1, dag.KERN_TT), (320, 192, trees.FLAT, 1, dag.KERN_TS),
                                  (512, 256, trees.PLASMA, 4, dag.KERN_TS)],
                         ids=lambda c: "%dx%d_t%d_bs%d_k%d" % c)
def test_complex_apply_q_residual_and_orthogonality(torch_cuda, case):
    """Q^H B and Q B against the complex oracle (5 and 40 right-hand
    sides: one and two 32-column slabs), and the GPU's own Q: ||A - QR||_F /
    ||A||_F and ||Q^H Q - I||_F within 50 n eps."""
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    m, n, tree, bs, kern = case
    _say("complex apply_q %s" % (case,))
    A = _cplx(m, n, 65)
    F = tqr.zfactor(_gpu(torch, A), 32, tree, bs, kern)
    O = ztiled.ztiled_qr(A, 32, tree, bs, kern)
    for nrhs in (5, 40):
        B = _cplx(m, nrhs, 66 + nrhs)
        for trans in ("C", "N"):
            got = F.apply_q(_gpu(torch, B), trans).cpu().numpy()
            want = ztiled.zapply_q(O, B, trans)
            assert np.max(np.abs(got - want)) <= 50 * n * EPS * np.linalg.norm(B), (nrhs, trans)
    E = np.zeros((m, n), dtype=np.complex128)
    E[:n, :n] = np.eye(n)
    Q = F.apply_q(_gpu(torch, E), "N").cpu().numpy()
    R = np.triu(F.packed().cpu().numpy()[:n, :n])
    assert np.linalg.norm(A - Q @ R) / np.linalg.norm(A) <= 50 * n * EPS
    assert np.linalg.norm(Q.conj().T @ Q - np.eye(n)) <= 50 * n * EPS


@pytest.mark.parametrize("case", [(256, 128, trees.GREEDY, 1, dag.KERN_TT), (512, 256, trees.FLAT, 1, dag.KERN_TS),
                                  (320, 320, trees.FIBONACCI, 1, dag.KERN_TT)],
                         ids=lambda c: "%dx%d_t%d_bs%d_k%d" % c)
def test_complex_least_squares_matches_lapack(torch_cuda, case):
    """X = R^{-1} (Q^H B)(1:n) against LAPACK's complex least squares
    (numpy.linalg.lstsq) within 10 kappa n eps relative, and R^{-1} X
    against a dense triangular solve of the GPU's own R."""
    import paper_1104_4475_amd as tqr
    from scipy.linalg import solve_triangular
    torch = torch_cuda
    m, n, tree, bs, kern = case
    _say("complex lstsq %s" % (case,))
    A = _cplx(m, n, 71)
    B = _cplx(m, 3, 72)
    F = tqr.zfactor(_gpu(torch, A), 32, tree, bs, kern)
    X = F.lstsq(_gpu(torch, B)).cpu().numpy()
    Xn = np.linalg.lstsq(A, B, rcond=None)[0]
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(X - Xn) / np.linalg.norm(Xn) <= 10 * kappa * n * EPS
    R = np.triu(F.packed().cpu().numpy()[:n, :n])
    Y = _cplx(n, 2, 73)
    got = F.solve_r(_gpu(torch, Y)).cpu().numpy()
    want = solve_triangular(R, Y, lower=False)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 10 * np.linalg.cond(R) * n * EPS
