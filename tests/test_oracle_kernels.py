"""Oracle kernel pins against LAPACK (through SciPy).

Each tile kernel is a special case of a LAPACK routine: GEQRT is dgeqrf of the
tile; TSQRT / TTQRT are dgeqrf of the stacked pair [R; A2] / [R1; R2] (whose
reflectors vanish on the top block below its diagonal); the updates are
dormqr with those reflectors.  LAPACK rounds differently (scaled norms,
blocking), so agreement is to a few ulps scaled by the data.
"""

import numpy as np
import pytest
from scipy.linalg import lapack

from oracle import brute, kernels

TOL = 1e-12


def _dgeqrf(A):
    qr, tau, work, info = lapack.dgeqrf(np.asfortranarray(A))
    assert info == 0
    return qr, tau


def _dormqr_t(qr, tau, C):
    lwork = max(1, C.shape[1]) * 64
    cq, work, info = lapack.dormqr("L", "T", qr, tau, np.asfortranarray(C), lwork)
    assert info == 0
    return cq


@pytest.mark.parametrize("nb", [4, 16, 33])
def test_geqrt_unmqr_vs_lapack(nb):
    rng = np.random.default_rng(nb)
    A = rng.standard_normal((nb, nb))
    C = rng.standard_normal((nb, nb + 3))
    F = A.copy()
    tau = kernels.geqrt(F)
    qr, ltau = _dgeqrf(A)
    assert np.allclose(np.triu(F), np.triu(qr), atol=TOL, rtol=0)
    assert np.allclose(np.tril(F, -1), np.tril(qr, -1), atol=TOL, rtol=0)
    assert np.allclose(tau, ltau, atol=TOL, rtol=0)
    C1 = C.copy()
    kernels.unmqr(F, tau, C1)
    assert np.allclose(C1, _dormqr_t(qr, ltau, C), atol=TOL, rtol=0)


@pytest.mark.parametrize("nb", [4, 16, 33])
def test_tsqrt_tsmqr_vs_lapack(nb):
    rng = np.random.default_rng(100 + nb)
    R = np.triu(rng.standard_normal((nb, nb)))
    A2 = rng.standard_normal((nb, nb))
    S = np.vstack([R, A2])
    qr, ltau = _dgeqrf(S)
    R1, V2 = R.copy(), A2.copy()
    tau = kernels.tsqrt(R1, V2)
    assert np.allclose(np.triu(R1), np.triu(qr[:nb]), atol=TOL, rtol=0)
    assert np.allclose(np.tril(qr[:nb], -1), 0.0, atol=TOL)
    assert np.allclose(V2, qr[nb:], atol=TOL, rtol=0)
    assert np.allclose(tau, ltau, atol=TOL, rtol=0)
    C1 = rng.standard_normal((nb, 5))
    C2 = rng.standard_normal((nb, 5))
    want = _dormqr_t(qr, ltau, np.vstack([C1, C2]))
    kernels.tsmqr(V2, tau, C1, C2)
    assert np.allclose(np.vstack([C1, C2]), want, atol=TOL, rtol=0)


@pytest.mark.parametrize("nb", [4, 16, 33])
def test_ttqrt_ttmqr_vs_lapack(nb):
    rng = np.random.default_rng(200 + nb)
    R1 = np.triu(rng.standard_normal((nb, nb)))
    R2u = np.triu(rng.standard_normal((nb, nb)))
    lower = np.tril(rng.standard_normal((nb, nb)), -1)  # must stay untouched
    qr, ltau = _dgeqrf(np.vstack([R1, R2u]))
    A1, A2 = R1.copy(), R2u + lower
    tau = kernels.ttqrt(A1, A2)
    assert np.allclose(np.triu(A1), np.triu(qr[:nb]), atol=TOL, rtol=0)
    assert np.allclose(np.triu(A2), np.triu(qr[nb:]), atol=TOL, rtol=0)
    assert np.allclose(np.tril(qr[nb:], -1), 0.0, atol=TOL)
    assert np.array_equal(np.tril(A2, -1), lower)
    assert np.allclose(tau, ltau, atol=TOL, rtol=0)
    C1 = rng.standard_normal((nb, 4))
    C2 = rng.standard_normal((nb, 4))
    want = _dormqr_t(qr, ltau, np.vstack([C1, C2]))
    kernels.ttmqr(A2, tau, C1, C2)
    assert np.allclose(np.vstack([C1, C2]), want, atol=TOL, rtol=0)


def test_updates_transpose_inverse():
    rng = np.random.default_rng(3)
    nb = 12
    V = rng.standard_normal((nb, nb))
    tau = kernels.geqrt(V)
    C = rng.standard_normal((nb, 3))
    D = C.copy()
    kernels.unmqr(V, tau, D, "T")
    kernels.unmqr(V, tau, D, "N")
    assert np.allclose(D, C, atol=1e-13)


def test_house_conventions():
    beta, tau, v = kernels.house(3.0, np.zeros(4))
    assert (beta, tau) == (3.0, 0.0) and not v.any()
    beta, tau, v = kernels.house(3.0, np.array([4.0]))
    assert beta == -5.0 and abs(tau - 1.6) < 1e-15 and abs(v[0] - 0.5) < 1e-15
    beta, tau, v = kernels.house(0.0, np.array([2.0]))
    assert beta == -2.0 and tau == 1.0
    # H (alpha, x)^T = (beta, 0)^T
    x = np.array([1.0, -2.0, 0.5])
    beta, tau, v = kernels.house(-0.7, x)
    u = np.concatenate([[1.0], v])
    y = np.concatenate([[-0.7], x])
    hy = y - tau * u * (u @ y)
    assert np.allclose(hy, [beta, 0, 0, 0], atol=1e-15)


def test_brute_vs_lapack_and_numpy():
    rng = np.random.default_rng(11)
    A = rng.standard_normal((40, 17))
    R, V, tau = brute.householder_qr(A)
    qr, ltau = _dgeqrf(A)
    assert np.allclose(R, np.triu(qr[:17]), atol=TOL, rtol=0)
    assert np.allclose(tau, ltau, atol=TOL, rtol=0)
    Rn = np.linalg.qr(A, mode="r")
    assert np.allclose(np.abs(R), np.abs(Rn), atol=1e-12)
