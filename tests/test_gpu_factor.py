"""GPU parity: the HIP tiled QR against the oracle, element by element.

Every case prints its name before touching the GPU.  Factors (R, V and the
Householder scalars) are compared with the oracle run on the same input with
the same tree and kernels; the bound is 50 n eps ||A||_F elementwise, and the
residual / orthogonality bounds of the factorization are 50 n eps.
"""

import os
import sys

import numpy as np
import pytest

import tqr_inputs
from oracle import dag, tiled, trees

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


def _gpu(torch, A):
    """Column-major float64 copy of a host matrix on the GPU."""
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A, dtype=np.float64).T)).cuda().t()


def _factor_both(torch, A, nb, tree, bs=1, kern=dag.KERN_DEFAULT, upd=0):
    import paper_1104_4475_amd as tqr
    F = tqr.factor(_gpu(torch, A), nb, tree, bs, kern, upd)
    F.sync()
    O = tiled.tiled_qr(A, nb, tree, bs, kern)
    return F, O


def _compare(torch, F, O, A):
    p, q, nb = O.p, O.q, O.nb
    n = O.n
    tol = 50 * n * EPS * np.linalg.norm(A)
    P = F.packed().cpu().numpy()
    err = np.max(np.abs(P - O.A))
    assert err <= tol, "packed factor differs by %g (tol %g)" % (err, tol)
    tg, tp = [t.cpu().numpy() for t in F.tau()]
    for (r, c), tau in O.tau_g.items():
        assert np.max(np.abs(tg[c - 1, r - 1] - tau)) <= 1e-12, ("tau_geqrt", r, c)
    for (i, c), tau in O.tau_p.items():
        assert np.max(np.abs(tp[c - 1, i - 1] - tau)) <= 1e-12, ("tau_pair", i, c)
    return err


SMALL = [
    # (m, n, nb, tree, bs, kernels)
    (32, 32, 32, trees.GREEDY, 1, dag.KERN_TT),      # GEQRT only
    (32, 64, 32, trees.GREEDY, 1, dag.KERN_TT),      # invalid: m < n (skipped below)
    (64, 32, 32, trees.GREEDY, 1, dag.KERN_TT),      # GEQRT x2 + TTQRT
    (64, 32, 32, trees.FLAT, 1, dag.KERN_TS),        # GEQRT + TSQRT
    (64, 64, 32, trees.GREEDY, 1, dag.KERN_TT),      # + UNMQR, TTMQR
    (64, 64, 32, trees.FLAT, 1, dag.KERN_TS),        # + TSMQR
    (96, 64, 32, trees.BINARY, 1, dag.KERN_TT),
    (128, 64, 64, trees.GREEDY, 1, dag.KERN_TT),
    (128, 128, 64, trees.FLAT, 1, dag.KERN_TS),
    (384, 256, 128, trees.FIBONACCI, 1, dag.KERN_TT),
    (256, 256, 128, trees.FLAT, 1, dag.KERN_TS),
    (512, 256, 256, trees.GREEDY, 1, dag.KERN_TT),
    (512, 256, 256, trees.FLAT, 1, dag.KERN_TS),
    (768, 512, 256, trees.PLASMA, 2, dag.KERN_TT),
    # TS-hybrid trees at nb >= 128 (panel tasks run as inner-block subtasks
    # that pipeline along a pivot: TS leaves, TT merges)
    (1024, 512, 256, trees.PLASMA, 2, dag.KERN_TS),
    (768, 768, 128, trees.GREEDY, 1, dag.KERN_TS),
    (1024, 768, 256, trees.ASAP, 1, dag.KERN_TT),
    (1280, 768, 256, trees.HADRI, 2, dag.KERN_TS),
]


@pytest.mark.parametrize("case", SMALL, ids=lambda c: "%dx%d_nb%d_t%d_bs%d_k%d" % c)
def test_small_shapes_match_oracle(torch_cuda, case):
    m, n, nb, tree, bs, kern = case
    if m < n:
        pytest.skip("m < n is rejected by the library")
    _say("case %s" % (case,))
    A = tqr_inputs.gaussian(m, n, seed=m + 7 * n + nb)
    F, O = _factor_both(torch_cuda, A, nb, tree, bs, kern)
    _compare(torch_cuda, F, O, A)


C1 = [(trees.GREEDY, 1, dag.KERN_TT), (trees.FLAT, 1, dag.KERN_TS), (trees.SAMEH_KUCK, 1, dag.KERN_TT),
      (trees.BINARY, 1, dag.KERN_TT), (trees.FIBONACCI, 1, dag.KERN_TT), (trees.PLASMA, 2, dag.KERN_TT),
      (trees.PLASMA, 3, dag.KERN_TS), (trees.GREEDY, 1, dag.KERN_TS),
      # run-time pairings (Sec. 3.2) and Hadri's Semi/Fully-Parallel trees (Sec. 4)
      (trees.ASAP, 1, dag.KERN_TT), (trees.GRASAP, 2, dag.KERN_TT), (trees.HADRI, 3, dag.KERN_TS),
      (trees.HADRI, 3, dag.KERN_TT)]


@pytest.mark.parametrize("tree,bs,kern", C1)
def test_config1_parity_and_bounds(torch_cuda, tree, bs, kern):
    # 256 x 128 at nb = 32 (p = 8, q = 4), N(0,1) from seed 0.
    _say("config1 tree=%d bs=%d kern=%d" % (tree, bs, kern))
    torch = torch_cuda
    A = tqr_inputs.gaussian(256, 128, seed=tqr_inputs.SEED_C1)
    F, O = _factor_both(torch, A, 32, tree, bs, kern)
    _compare(torch, F, O, A)
    Ag = _gpu(torch, A)
    Q = F.thin_q()
    R = F.R()
    n = 128
    res = (torch.linalg.norm(Ag - Q @ R) / torch.linalg.norm(Ag)).item()
    orth = torch.linalg.norm(Q.T @ Q - torch.eye(n, dtype=torch.float64, device="cuda")).item()
    assert res <= 50 * n * EPS, res
    assert orth <= 50 * n * EPS, orth


def test_level_executor_matches_persistent(torch_cuda, monkeypatch):
    _say("level executor")
    A = tqr_inputs.gaussian(256, 128, seed=3)
    monkeypatch.setenv("TQR_EXEC", "level")
    F, O = _factor_both(torch_cuda, A, 32, trees.GREEDY, 1, dag.KERN_TT)
    _compare(torch_cuda, F, O, A)
    monkeypatch.setenv("TQR_EXEC", "persistent")


@pytest.mark.parametrize("order", ["asap", "alap", "bl"])
def test_other_dispatch_orders_match(torch_cuda, monkeypatch, order):
    """The default dispatch order is the start order of a simulated list
    schedule; the ASAP, ALAP and plain bottom-level orders must give the
    same factors."""
    _say("%s order" % order)
    A = tqr_inputs.gaussian(512, 256, seed=4)
    monkeypatch.setenv("TQR_ORDER", order)
    F, O = _factor_both(torch_cuda, A, 64, trees.FIBONACCI, 1, dag.KERN_TT)
    monkeypatch.delenv("TQR_ORDER")
    _compare(torch_cuda, F, O, A)


def test_apply_q_matches_oracle(torch_cuda):
    _say("apply_q")
    torch = torch_cuda
    A = tqr_inputs.gaussian(320, 192, seed=11)
    B = tqr_inputs.gaussian(320, 5, seed=12)
    for tree, kern in ((trees.GREEDY, dag.KERN_TT), (trees.FLAT, dag.KERN_TS)):
        F, O = _factor_both(torch, A, 64, tree, 1, kern)
        for trans in ("T", "N"):
            got = F.apply_q(_gpu(torch, B), trans).cpu().numpy()
            want = tiled.apply_q(O, B, trans)
            assert np.max(np.abs(got - want)) <= 50 * 192 * EPS * np.linalg.norm(B), (tree, trans)
        # more than 16 right-hand sides (four column groups per slab)
        Bw = tqr_inputs.gaussian(320, 21, seed=13)
        got = F.apply_q(_gpu(torch, Bw), "T").cpu().numpy()
        assert np.max(np.abs(got - tiled.apply_q(O, Bw, "T"))) <= 50 * 192 * EPS * np.linalg.norm(Bw), tree
        # empty right-hand side is a no-op
        E = torch.zeros((320, 0), dtype=torch.float64, device="cuda")
        assert F.apply_q(E, "T").shape == (320, 0)


def test_lstsq_matches_oracle(torch_cuda):
    _say("lstsq")
    torch = torch_cuda
    A = tqr_inputs.gaussian(384, 128, seed=21)
    B = tqr_inputs.gaussian(384, 3, seed=22)
    F, O = _factor_both(torch, A, 64, trees.GREEDY, 1, dag.KERN_TT)
    X, info = F.lstsq(_gpu(torch, B))
    want = tiled.lstsq(O, B)
    assert np.max(np.abs(X.cpu().numpy() - want)) <= 1e-10


@pytest.mark.parametrize("upd", [0, 1])
def test_panel_block_subtasks_bit_identical(torch_cuda, upd):
    """Panel tasks run as inner-block subtasks (the default at nb >= 128) or
    whole (TQR_PANEL_SPLIT=0): every tile sees the same operations in the
    same order, so the factors are bit-identical."""
    import os
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    _say("panel block subtasks vs whole panel tasks, upd %d" % upd)
    A = _gpu(torch, tqr_inputs.gaussian(1024, 768, seed=41))
    out = []
    for split in ("1", "0"):
        os.environ["TQR_PANEL_SPLIT"] = split
        try:
            F = tqr.factor(A, 256, trees.PLASMA, 2, dag.KERN_TS, upd)
            F.sync()
            out.append(F.packed().cpu().numpy())
        finally:
            del os.environ["TQR_PANEL_SPLIT"]
    assert np.array_equal(out[0], out[1])


def test_trsm_inverse_and_substitution_agree(torch_cuda):
    """Triangular solves with the diagonal-tile inverses and coupling tiles
    (default) against substitution inside the diagonal tiles
    (TQR_TRSM_SUBST=1), through lstsq and the R^-T solve of the augmented
    refinement; both against the oracle."""
    import os
    torch = torch_cuda
    _say("trsm inverse vs substitution")
    A = tqr_inputs.gaussian(1024, 512, seed=43)
    B = tqr_inputs.gaussian(1024, 5, seed=44)
    F, O = _factor_both(torch, A, 128, trees.GREEDY, 1, dag.KERN_TT)
    want = tiled.lstsq(O, B)
    sols = []
    for sub in ("0", "1"):
        os.environ["TQR_TRSM_SUBST"] = sub
        try:
            X, info = F.lstsq(_gpu(torch, B), A0=_gpu(torch, A), tol=1e-13)
            sols.append(X.cpu().numpy())
        finally:
            del os.environ["TQR_TRSM_SUBST"]
        assert info["converged"]
    scale = np.max(np.abs(want))
    for X in sols:
        assert np.max(np.abs(X - want)) <= 1e-10 * scale
    assert np.max(np.abs(sols[0] - sols[1])) <= 1e-10 * scale


def test_square_refinement_fp64(torch_cuda):
    _say("square refinement fp64")
    torch = torch_cuda
    n = 256
    A = tqr_inputs.conditioned(n, 1e6, 31, 32)
    Xt = tqr_inputs.gaussian(n, 4, seed=33)
    B = A @ Xt
    F, O = _factor_both(torch, A, 64, trees.GREEDY, 1, dag.KERN_TT)
    X, info = F.lstsq(_gpu(torch, B), A0=_gpu(torch, A), tol=1e-12)
    assert info["converged"] and info["backward_err"] <= 1e-12
    eta = tiled.backward_error(A, X.cpu().numpy(), B)
    assert np.max(eta) <= 1e-12


@pytest.mark.parametrize("upd", [0, 1])
def test_joint_factor_and_qtb(torch_cuda, upd):
    """tiledqr_refactor_qtb: the factors are bit-identical to a plain
    factorization (every subtask is deterministic) and Q^T B matches the
    separate application within 50 n eps ||B||; the least-squares solution
    from the joint Q^T B matches the plain one."""
    import paper_1104_4475_amd as tqr
    torch = torch_cuda
    _say("joint factor + Q^T B, upd %d" % upd)
    m, n, nb, nrhs = 1024, 768, 256, 4
    A = tqr_inputs.gaussian(m, n, 71)
    B = np.random.default_rng(72).standard_normal((m, nrhs))
    Ad, Bd = _gpu(torch, A), _gpu(torch, B)
    F = tqr.factor(Ad, nb, trees.GREEDY, 1, dag.KERN_DEFAULT, upd)
    P0 = F.packed().clone()
    Y0 = F.apply_q(Bd, "T")
    QtB = F.refactor_qtb(Ad, Bd)
    torch.cuda.synchronize()
    assert torch.equal(F.packed(), P0)
    err = (QtB - Y0).abs().max().item()
    assert err <= 50 * m * EPS * np.linalg.norm(B), err
    X1, _ = F.lstsq(Bd)
    X2, _ = F.lstsq(Bd, QtB=QtB)
    assert (X1 - X2).abs().max().item() <= 1e-10 * X1.abs().max().item()
