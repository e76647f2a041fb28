"""The double-complex oracle (oracle.zkernels / oracle.ztiled) against what
fixes it from outside: the pinned real oracle on real input, LAPACK's
zgeqrf through numpy.linalg.qr (R up to the signs of its rows: both keep
the diagonal real), the residual and orthogonality bounds of the tiled QR,
and the closed form of a diagonal complex matrix."""

import numpy as np
import pytest

import tqr_inputs
from oracle import dag, tiled, trees, ztiled, zkernels

EPS = np.finfo(np.float64).eps

CASES = [
    # (m, n, nb, tree, bs, kernels)
    (64, 32, 8, trees.GREEDY, 1, dag.KERN_TT),
    (64, 32, 8, trees.FLAT, 1, dag.KERN_TS),
    (96, 48, 16, trees.FIBONACCI, 1, dag.KERN_TT),
    (128, 64, 16, trees.PLASMA, 2, dag.KERN_TS),
    (64, 64, 16, trees.BINARY, 1, dag.KERN_TT),
]


def _cplx(m, n, seed):
    return tqr_inputs.gaussian(m, n, seed) + 1j * tqr_inputs.gaussian(m, n, seed + 7919)


@pytest.mark.parametrize("case", CASES)
def test_real_input_reduces_to_the_real_oracle(case):
    m, n, nb, tree, bs, kern = case
    A = tqr_inputs.gaussian(m, n, 31)
    Z = ztiled.ztiled_qr(A.astype(np.complex128), nb, tree, bs, kern)
    F = tiled.tiled_qr(A, nb, tree, bs, kern)
    # the imaginary parts stay exactly zero; the real parts differ from the
    # real oracle only by the summation order of the dot products
    assert np.all(Z.A.imag == 0.0)
    assert np.max(np.abs(Z.A.real - F.A)) <= 4 * EPS * np.linalg.norm(A)
    for ztau, rtau in ((Z.tau_g, F.tau_g), (Z.tau_p, F.tau_p)):
        assert set(ztau) == set(rtau)
        for key, t in rtau.items():
            assert np.all(ztau[key].imag == 0.0)
            # tau = (beta - alpha) / beta moves by |d alpha| / ||x|| when x
            # is short: a loose absolute bound (R and V are held to 4 eps above)
            assert np.max(np.abs(ztau[key].real - t)) <= 1e-12


@pytest.mark.parametrize("case", CASES)
def test_r_matches_lapack_up_to_row_signs(case):
    m, n, nb, tree, bs, kern = case
    A = _cplx(m, n, 41)
    Z = ztiled.ztiled_qr(A, nb, tree, bs, kern)
    R = Z.R()
    Rn = np.linalg.qr(A, mode="r")[:n, :n]
    assert np.all(np.diag(R).imag == 0.0)
    d = np.sign(np.diag(R).real) * np.sign(np.diag(Rn).real)
    assert np.all(np.abs(d) == 1.0)
    assert np.max(np.abs(R - d[:, None] * Rn)) <= 50 * n * EPS * np.linalg.norm(A)


@pytest.mark.parametrize("case", CASES)
def test_residual_and_orthogonality(case):
    m, n, nb, tree, bs, kern = case
    A = _cplx(m, n, 43)
    Z = ztiled.ztiled_qr(A, nb, tree, bs, kern)
    Q = ztiled.zthin_q(Z)
    res = np.linalg.norm(A - Q @ Z.R()) / np.linalg.norm(A)
    orth = np.linalg.norm(Q.conj().T @ Q - np.eye(n))
    assert res <= 50 * n * EPS and orth <= 50 * n * EPS, (res, orth)
    # Q^H B from the reflectors equals the conjugate transpose of Q [I; 0]
    # on the first n rows (square factor: all of Q)
    if m == n:
        B = _cplx(m, 3, 47)
        assert np.max(np.abs(ztiled.zapply_q(Z, B, "C") - Q.conj().T @ B)) <= 50 * n * EPS * np.linalg.norm(B)


def test_diagonal_complex_matrix_closed_form():
    """A = diag(d), complex d: every reflector acts on a zero vector below a
    complex pivot, so R = diag(beta) with beta = -sign(Re d) |d| real, and
    Q = diag(d / beta)."""
    n, nb = 32, 8
    rng = np.random.default_rng(5)
    d = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    d[3] = 2.0  # a real pivot: no reflector (tau = 0)
    d[4] = -1.5j  # Re d = 0: sign(+0) = +1, beta = -|d|
    A = np.diag(d)
    for tree, kern in ((trees.GREEDY, dag.KERN_TT), (trees.FLAT, dag.KERN_TS)):
        Z = ztiled.ztiled_qr(A, nb, tree, 1, kern)
        beta = -np.where(d.real >= 0.0, 1.0, -1.0) * np.abs(d)
        beta[3] = 2.0
        assert np.max(np.abs(np.diag(Z.R()) - beta)) <= 4 * EPS * np.abs(d).max()
        assert np.max(np.abs(np.triu(Z.R(), 1))) == 0.0
        Q = ztiled.zthin_q(Z)
        assert np.max(np.abs(np.diag(Q) - d / beta)) <= 8 * EPS
        assert Z.tau_g[(1, 1)][3] == 0.0


def test_reflector_annihilates_and_is_unitary():
    rng = np.random.default_rng(9)
    for _ in range(20):
        x = rng.standard_normal(6) + 1j * rng.standard_normal(6)
        alpha = complex(rng.standard_normal(), rng.standard_normal())
        beta, tau, v = zkernels.zhouse(alpha, x)
        u = np.concatenate(([1.0], v))
        H = np.eye(7) - tau * np.outer(u, u.conj())
        y = H.conj().T @ np.concatenate(([alpha], x))
        assert abs(y[0] - beta) <= 8 * EPS * abs(beta) and np.max(np.abs(y[1:])) <= 8 * EPS * abs(beta)
        assert np.linalg.norm(H.conj().T @ H - np.eye(7)) <= 16 * EPS
        assert beta.imag == 0.0
