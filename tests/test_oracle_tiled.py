"""Oracle pins for the tiled driver, apply_q, least squares and refinement."""

import numpy as np
import pytest

import tqr_inputs
from oracle import brute, dag, tiled, trees

EPS = np.finfo(np.float64).eps
CASES = [
    (trees.GREEDY, 1, dag.KERN_TT), (trees.FLAT, 1, dag.KERN_TS),
    (trees.SAMEH_KUCK, 1, dag.KERN_TT), (trees.BINARY, 1, dag.KERN_TT),
    (trees.FIBONACCI, 1, dag.KERN_TT), (trees.PLASMA, 3, dag.KERN_TT),
    (trees.GREEDY, 1, dag.KERN_TS), (trees.PLASMA, 2, dag.KERN_TS),
]


def _rows_equal_up_to_sign(R1, R2, tol):
    s = np.sign(np.diag(R1)) * np.sign(np.diag(R2))
    return np.allclose(R1 * s[:, None], R2, atol=tol, rtol=0)


@pytest.mark.parametrize("tree,bs,kern", CASES)
def test_tiled_r_matches_brute_force(tree, bs, kern):
    A = tqr_inputs.gaussian(48, 24, seed=4)
    F = tiled.tiled_qr(A, 6, tree, bs, kern)
    R0, _, _ = brute.householder_qr(A)
    assert _rows_equal_up_to_sign(F.R(), R0, 1e-12)


@pytest.mark.parametrize("tree,bs,kern", CASES[:3])
def test_config1_bounds(tree, bs, kern):
    # 256 x 128 at nb = 32 (p = 8, q = 4), N(0,1) from a seed.
    A = tqr_inputs.gaussian(256, 128, seed=tqr_inputs.SEED_C1)
    F = tiled.tiled_qr(A, 32, tree, bs, kern)
    n = A.shape[1]
    Q = tiled.thin_q(F)
    R = F.R()
    res = np.linalg.norm(A - Q @ R) / np.linalg.norm(A)
    orth = np.linalg.norm(Q.T @ Q - np.eye(n))
    assert res <= 50 * n * EPS
    assert orth <= 50 * n * EPS
    Rn = np.linalg.qr(A, mode="r")
    assert np.allclose(np.abs(R), np.abs(Rn), atol=1e-11)


def test_square_and_single_column():
    for (m, n, nb) in ((30, 30, 5), (20, 5, 5), (5, 5, 5)):
        A = tqr_inputs.gaussian(m, n, seed=m + n)
        for tree in (trees.GREEDY, trees.FLAT):
            F = tiled.tiled_qr(A, nb, tree)
            R0, _, _ = brute.householder_qr(A)
            assert _rows_equal_up_to_sign(F.R(), R0, 1e-12)


def test_apply_q_roundtrip_and_orthogonality():
    A = tqr_inputs.gaussian(40, 16, seed=9)
    F = tiled.tiled_qr(A, 4, trees.GREEDY)
    B = tqr_inputs.gaussian(40, 3, seed=10)
    Y = tiled.apply_q(F, B, "T")
    Z = tiled.apply_q(F, Y, "N")
    assert np.allclose(Z, B, atol=1e-13)
    assert np.isclose(np.linalg.norm(Y), np.linalg.norm(B), rtol=1e-13)
    # Q^T A = [R; 0]
    QA = tiled.apply_q(F, A, "T")
    assert np.allclose(QA[:16], F.R(), atol=1e-12)
    assert np.allclose(QA[16:], 0.0, atol=1e-12)


def test_lstsq_tall_matches_numpy():
    A = tqr_inputs.gaussian(60, 20, seed=12)
    B = tqr_inputs.gaussian(60, 2, seed=13)
    F = tiled.tiled_qr(A, 5, trees.FIBONACCI)
    X = tiled.lstsq(F, B)
    Xn = np.linalg.lstsq(A, B, rcond=None)[0]
    assert np.allclose(X, Xn, atol=1e-12)
    assert np.max(tiled.backward_error(A, X, B)) < 1e-14


def test_conditioned_generator():
    A = tqr_inputs.conditioned(64, 1e6, 2, 3)
    s = np.linalg.svd(A, compute_uv=False)
    assert np.isclose(s[0], 1.0, rtol=1e-12)
    assert np.isclose(s[-1], 1e-6, rtol=1e-8)


def test_refinement_recovers_from_perturbed_factors():
    # Plant an error in the oracle: solve with factors of A + E, |E| ~ 1e-6,
    # and check that FP64-residual refinement reaches backward error 1e-12.
    n = 48
    A = tqr_inputs.conditioned(n, 1e2, 21, 22)
    Xt = tqr_inputs.gaussian(n, 4, seed=23)
    B = A @ Xt
    E = 1e-6 * tqr_inputs.gaussian(n, n, seed=24)
    F = tiled.tiled_qr(A + E, 8, trees.GREEDY)
    X, iters, ok, eta = tiled.refine(A, B, lambda rhs: tiled.lstsq(F, rhs))
    assert ok and eta <= 1e-12 and 1 <= iters <= 6
    X64 = tiled.lstsq(tiled.tiled_qr(A, 8, trees.GREEDY), B)
    assert np.allclose(X, X64, atol=1e-11)


def test_refinement_reports_stagnation():
    n = 32
    A = tqr_inputs.conditioned(n, 1e10, 31, 32)
    B = A @ tqr_inputs.gaussian(n, 1, seed=33)
    E = 1e-3 * tqr_inputs.gaussian(n, n, seed=34)
    F = tiled.tiled_qr(A + E, 8, trees.GREEDY)
    X, iters, ok, eta = tiled.refine(A, B, lambda rhs: tiled.lstsq(F, rhs), max_iter=30)
    assert not ok and iters < 30


# ---- pins of the backward error -----------------------------------------
# Square systems: eta(x) = ||b - A x|| / (||A||_F ||x|| + ||b||) is the
# normwise backward error of Rigal and Gaches (Higham, Accuracy and Stability
# of Numerical Algorithms, Thm. 7.1): the smallest eps with (A + dA) x = b +
# db, ||dA||_F <= eps ||A||_F, ||db|| <= eps ||b||.  Tall systems: eta(x) =
# ||A^T r|| / (||A||_F ||r||), zero exactly at the least-squares solution.

def test_backward_error_square_hand_values():
    # A = diag(3, 4): ||A||_F = 5 while ||A||_2 = 4, so a 2-norm in place of
    # the Frobenius norm, or a dropped ||b|| term, changes the value.
    A = np.diag([3.0, 4.0])
    b = np.array([[3.0], [4.0]])
    x = np.array([[1.0], [0.0]])       # r = (0, 4)
    assert tiled.backward_error(A, x, b)[0] == pytest.approx(4.0 / (5.0 * 1.0 + 5.0), rel=1e-15)
    x = np.array([[1.0], [1.0]])       # exact solution
    assert tiled.backward_error(A, x, b)[0] == 0.0
    x = np.zeros((2, 1))               # r = b: eta = ||b|| / ||b|| = 1
    assert tiled.backward_error(A, x, b)[0] == pytest.approx(1.0, rel=1e-15)


def test_backward_error_square_is_attained():
    """The perturbations dA = a r x^T / ||x||^2 and db = -c r with
    relative sizes exactly eta (a ||r|| / ||x|| = eta ||A||_F, c ||r|| = eta
    ||b||) make x exact: (A + dA) x = b + db holds iff a + c = 1, i.e. iff
    eta is the value of the theorem."""
    rng = np.random.default_rng(71)
    for n in (1, 5, 17):
        A = rng.standard_normal((n, n))
        b = rng.standard_normal((n, 1))
        x = np.linalg.solve(A, b) + 1e-3 * rng.standard_normal((n, 1))
        eta = tiled.backward_error(A, x, b)[0]
        r = b - A @ x
        nr, nx = np.linalg.norm(r), np.linalg.norm(x)
        a = eta * np.linalg.norm(A, "fro") * nx / nr
        c = eta * np.linalg.norm(b) / nr
        dA = a * (r @ x.T) / nx ** 2
        db = -c * r
        assert np.linalg.norm(dA, "fro") == pytest.approx(eta * np.linalg.norm(A, "fro"), rel=1e-12)
        assert np.allclose((A + dA) @ x, b + db, rtol=0, atol=1e-12 * np.linalg.norm(b))


def test_backward_error_tall_hand_values():
    A = np.array([[3.0, 0.0], [0.0, 4.0], [0.0, 0.0]])   # ||A||_F = 5, ||A||_2 = 4
    b = np.array([[1.0], [1.0], [1.0]])
    x = np.zeros((2, 1))   # r = b, A^T r = (3, 4): eta = 5 / (5 sqrt 3)
    assert tiled.backward_error(A, x, b)[0] == pytest.approx(1.0 / np.sqrt(3.0), rel=1e-15)
    x = np.array([[1.0 / 3.0], [0.25]])  # least-squares solution: A^T r = 0
    assert tiled.backward_error(A, x, b)[0] == pytest.approx(0.0, abs=1e-16)
    # b orthogonal to range(A) and x = 0: r = b != 0 and A^T r = 0
    b = np.array([[0.0], [0.0], [2.0]])
    assert tiled.backward_error(A, np.zeros((2, 1)), b)[0] == 0.0
    # consistent system solved exactly: r = 0
    b = A @ np.array([[1.0], [-2.0]])
    assert tiled.backward_error(A, np.array([[1.0], [-2.0]]), b)[0] == 0.0


def test_backward_error_scale_invariant_and_per_column():
    rng = np.random.default_rng(72)
    for (m, n) in ((9, 9), (12, 5)):
        A = rng.standard_normal((m, n))
        X = rng.standard_normal((n, 3))
        B = rng.standard_normal((m, 3))
        e = tiled.backward_error(A, X, B)
        assert e.shape == (3,)
        assert np.allclose(tiled.backward_error(1e5 * A, X, 1e5 * B), e, rtol=1e-12)
        for c in range(3):
            assert tiled.backward_error(A, X[:, c:c + 1], B[:, c:c + 1])[0] == pytest.approx(e[c], rel=1e-15)
