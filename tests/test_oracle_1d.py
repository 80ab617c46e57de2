"""Pins of the oracle's 1D tables (GLL nodes/weights, M, K) and of the 1D
generalized eigenproblem, against closed forms, exact integration in mpmath,
and invariants fixed by the mathematics (Sec. 3 and the fast diagonalization of
Sec. 5)."""

import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import gll

PS = [2, 3, 4, 5, 6, 8, 12, 16]


def test_p2_closed_form():
    t = gll.tables(2)
    np.testing.assert_allclose(t["x"], [-1.0, 0.0, 1.0], atol=1e-16)
    np.testing.assert_allclose(t["w"], [1 / 3, 4 / 3, 1 / 3], rtol=1e-15)
    K = np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 6.0
    np.testing.assert_allclose(t["K"], K, rtol=0, atol=4e-16)


def test_p3_closed_form():
    t = gll.tables(3)
    s = 1 / math.sqrt(5)
    np.testing.assert_allclose(t["x"], [-1, -s, s, 1], atol=2e-16)
    np.testing.assert_allclose(t["w"], [1 / 6, 5 / 6, 5 / 6, 1 / 6], rtol=1e-15)


@pytest.mark.parametrize("p", [2, 3, 4, 6, 8, 12, 16, 24, 32])
def test_tables_vs_exact_integration(p):
    """Nodes, weights and K agree with exact polynomial integration in mpmath."""
    t = gll.tables(p)
    x, w, K = gll.mp_to_numpy(gll.tables_mp(p, dps=50))
    np.testing.assert_allclose(t["x"], x, rtol=0, atol=2e-16)
    np.testing.assert_allclose(t["w"], w, rtol=4e-16, atol=0)
    assert np.abs(t["K"] - K).max() <= 2.5e-16 * np.abs(K).max()


@pytest.mark.parametrize("p", PS + [32])
def test_quadrature_exactness(p):
    """GLL quadrature with p+1 points is exact up to degree 2p-1 and not at 2p."""
    t = gll.tables(p)
    for m in range(0, 2 * p):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.sum(t["w"] * t["x"] ** m) - exact) < 1e-14
    if p <= 16:   # the degree-2p error shrinks like 4^-p; beyond p=16 it is rounding-level
        m = 2 * p
        assert abs(np.sum(t["w"] * t["x"] ** m) - 2.0 / (m + 1)) > 1e-11


@pytest.mark.parametrize("p", PS + [24, 32])
def test_K_invariants(p):
    t = gll.tables(p)
    K = t["K"]
    np.testing.assert_array_equal(K, K.T)
    # constants are in the null space
    assert np.abs(K.sum(axis=1)).max() < 1e-13 * np.abs(K).max()
    ev = np.linalg.eigvalsh(K)
    assert ev[0] > -1e-12 * ev[-1]
    assert ev[1] > 1e-3       # one-dimensional null space
    # K x = e_p - e_0 for the linear function x (int phi_i' * 1)
    Kx = K @ t["x"]
    ref = np.zeros(p + 1)
    ref[0], ref[p] = -1.0, 1.0
    np.testing.assert_allclose(Kx, ref, atol=2e-13 * p)


@pytest.mark.parametrize("p", list(range(2, 33)))
def test_1d_schur_complement(p):
    """1D harmonic extension is linear: K_BB - K_BI K_II^-1 K_IB = 1/2 [[1,-1],[-1,1]]."""
    K = gll.tables(p)["K"]
    B = [0, p]
    I = list(range(1, p))
    S = K[np.ix_(B, B)] - K[np.ix_(B, I)] @ np.linalg.solve(K[np.ix_(I, I)], K[np.ix_(I, B)])
    np.testing.assert_allclose(S, 0.5 * np.array([[1, -1], [-1, 1]]), atol=1e-13)


def _geneig(p):
    t = gll.tables(p)
    I = slice(1, p)
    return sla.eigh(t["K"][I, I], t["M"][I, I]), t


def test_generalized_eigenvalues_small_p():
    (lam2, _), _ = _geneig(2)
    np.testing.assert_allclose(lam2, [2.0], rtol=1e-14)
    (lam3, _), _ = _geneig(3)
    np.testing.assert_allclose(lam3, [2.5, 7.5], rtol=1e-14)


@pytest.mark.parametrize("p", [8, 16, 32])
def test_generalized_eigen_invariants(p):
    """S^T M_II S = I, S^T K_II S = Lambda; the smallest eigenvalue approaches the
    1D Dirichlet Laplacian's pi^2/4 on [-1,1]; in the transformed basis the
    boundary rows reproduce the 1D Schur complement exactly."""
    (lam, S), t = _geneig(p)
    I = slice(1, p)
    M, K = t["M"], t["K"]
    np.testing.assert_allclose(S.T @ M[I, I] @ S, np.eye(p - 1), atol=1e-13)
    np.testing.assert_allclose(S.T @ K[I, I] @ S, np.diag(lam), atol=1e-12 * lam.max())
    assert abs(lam[0] - math.pi ** 2 / 4) < 1e-6
    a = S.T @ K[I, 0]
    b = S.T @ K[I, p]
    # the sums cancel K_00 ~ p^2/6 down to 1/2: allow rounding relative to K_00
    assert abs(K[0, 0] - np.sum(a * a / lam) - 0.5) < 1e-14 * K[0, 0] * p
    assert abs(K[0, p] - np.sum(a * b / lam) + 0.5) < 1e-14 * K[0, 0] * p
