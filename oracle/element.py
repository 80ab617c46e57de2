"""Element-level oracle: metric, explicit element operator, static condensation.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Index convention: element arrays u[k][j][i], flattened with i fastest, so a
Kronecker product A (x) B (x) C = np.kron(A, np.kron(B, C)) acts with C on i
(direction x1), B on j (x2) and A on k (x3).
"""

import numpy as np
import scipy.linalg as sla

from . import gll


def metric(h, lam):
    """Metric coefficients d_e = (h1 h2 h3 / 8) (lam, 4/h1^2, 4/h2^2, 4/h3^2).

    Sec. 3, eq. "metriccoeffelement": d_{e,0} carries the Helmholtz parameter,
    d_{e,1..3} the metric terms of a Cartesian element of extents h1, h2, h3.
    """
    h1, h2, h3 = (float(v) for v in h)
    J = h1 * h2 * h3 / 8.0
    return np.array([J * lam, J * 4.0 / h1**2, J * 4.0 / h2**2, J * 4.0 / h3**2])


def kron3(A, B, C):
    """A (x) B (x) C with C acting on the fastest index i."""
    return np.kron(A, np.kron(B, C))


def element_operator(p, d, tab=None):
    """Explicit element Helmholtz operator H_e ((p+1)^3 square, dense).

    Sec. 3, eq. "helmholtz_operator":
    H_e = d0 M(x)M(x)M + d1 M(x)M(x)K + d2 M(x)K(x)M + d3 K(x)M(x)M.
    """
    tab = tab or gll.tables(p)
    M, K = tab["M"], tab["K"]
    return (d[0] * kron3(M, M, M) + d[1] * kron3(M, M, K)
            + d[2] * kron3(M, K, M) + d[3] * kron3(K, M, M))


def stiffness_terms(p, tab=None):
    """The four tensor terms A_0..A_3 with H_e = sum_m d_m A_m (Sec. 3)."""
    tab = tab or gll.tables(p)
    M, K = tab["M"], tab["K"]
    return [kron3(M, M, M), kron3(M, M, K), kron3(M, K, M), kron3(K, M, M)]


def boundary_interior(p):
    """Index sets of the element's boundary nodes B and interior nodes I.

    Sec. 4: B holds every node with some local index in {0, p}, I the rest.
    Returned in element order (i fastest), plus the (k, j, i) triples of B.
    """
    n = p + 1
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    kk, jj, ii = kk.ravel(), jj.ravel(), ii.ravel()
    on_b = ((kk == 0) | (kk == p) | (jj == 0) | (jj == p) | (ii == 0) | (ii == p))
    B = np.nonzero(on_b)[0]
    I = np.nonzero(~on_b)[0]
    return B, I, np.stack([kk[B], jj[B], ii[B]], axis=1)


def condense(H, B, I):
    """Condensed operator H_BB - H_BI H_II^-1 H_IB (Sec. 4, eq. condensation_system).

    H_II^-1 H_IB is evaluated with a dense Cholesky factorisation of H_II, which
    is symmetric positive definite (it is the homogeneous Dirichlet operator of
    the element interior).
    """
    HBB = H[np.ix_(B, B)]
    HBI = H[np.ix_(B, I)]
    HIB = H[np.ix_(I, B)]
    if len(I) == 0:
        return HBB.copy()
    HII = H[np.ix_(I, I)]
    c = sla.cho_factor(HII, lower=True)
    X = sla.cho_solve(c, HIB)
    S = HBB - HBI @ X
    return 0.5 * (S + S.T)


def condensed_element_operator(p, d, tab=None):
    """H_hat_e for one element with metric d, with the B index set."""
    B, I, _ = boundary_interior(p)
    H = element_operator(p, d, tab)
    return condense(H, B, I), B, I


def condensed_rhs_element(H, B, I, F):
    """F_hat = F_B - H_BI H_II^-1 F_I for one element (Sec. 4, Algorithm 1)."""
    if len(I) == 0:
        return F[B].copy()
    HII = H[np.ix_(I, I)]
    c = sla.cho_factor(HII, lower=True)
    return F[B] - H[np.ix_(B, I)] @ sla.cho_solve(c, F[I])


def recover_interior_element(H, B, I, F, uB):
    """u_I = H_II^-1 (F_I - H_IB u_B) (Sec. 4, eq. condensation_inner)."""
    HII = H[np.ix_(I, I)]
    c = sla.cho_factor(HII, lower=True)
    return sla.cho_solve(c, F[I] - H[np.ix_(I, B)] @ uB)
