"""Element-level oracle: metric, explicit element operator, static condensation.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Index convention: element arrays u[k][j][i], flattened with i fastest, so a
Kronecker product A (x) B (x) C = np.kron(A, np.kron(B, C)) acts with C on i
(direction x1), B on j (x2) and A on k (x3).

Two routes to the Schur complement H_BB - H_BI H_II^-1 H_IB (Sec. 4):
* dense (p <= 16, n_I^3 <= 3375): H_e formed densely, H_II factored by
  Cholesky (``condense``, ``ElementBlocks`` with route "dense");
* separable (p > 16): H_e formed as a sparse sum of Kronecker products, H_II^-1
  applied through LAPACK's generalized symmetric eigendecomposition of the 1D
  interior matrices (``SeparableInteriorSolve``), the Schur complement only
  applied to vectors (or formed column block by column block on request).
  Sparse LU is no alternative: H_II's factors fill in almost completely (at
  p = 24 about 1.2e8 nonzeros and a factor time of minutes).
The separable route is pinned against the dense one at p = 8..16 and, at any
p, by the residual of H_II x = b with the explicit sparse H_II.
"""

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

# Largest degree whose element operator the oracle forms densely.
DENSE_MAX_P = 16

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


# ----------------------------------------------------------------------------
# Large-p route: sparse Kronecker blocks and a separable interior inverse
# ----------------------------------------------------------------------------

def kron3_sparse(A, B, C):
    """A (x) B (x) C as a sparse CSR matrix (C acting on the fastest index i)."""
    return sp.kron(sp.csr_matrix(A), sp.kron(sp.csr_matrix(B), sp.csr_matrix(C), format="csr"), format="csr")


def element_operator_sparse(p, d, tab=None):
    """The element operator of Sec. 3, eq. "helmholtz_operator", as a sparse
    matrix: d0 M(x)M(x)M + d1 M(x)M(x)K + d2 M(x)K(x)M + d3 K(x)M(x)M."""
    tab = tab or gll.tables(p)
    M, K = tab["M"], tab["K"]
    return (d[0] * kron3_sparse(M, M, M) + d[1] * kron3_sparse(M, M, K)
            + d[2] * kron3_sparse(M, K, M) + d[3] * kron3_sparse(K, M, M)).tocsr()


class SeparableInteriorSolve:
    """x = H_II^-1 b for the interior block of one element operator.

    Sec. 5 (fast diagonalisation): the 1D interior matrices satisfy
    K_II V = M_II V Lambda with V^T M_II V = I (here from LAPACK's generalized
    symmetric-definite eigensolver).  Then M_II = V^-T V^-1 and
    K_II = V^-T Lambda V^-1, so every Kronecker term of H_II has the factors
    V^-T (x) V^-T (x) V^-T on the left and V^-1 (x) V^-1 (x) V^-1 on the right,
    and H_II^-1 = (V (x) V (x) V) D^-1 (V^T (x) V^T (x) V^T) with
    D(k, j, i) = d0 + d1 Lambda_i + d2 Lambda_j + d3 Lambda_k.
    """

    def __init__(self, p, d, tab=None):
        tab = tab or gll.tables(p)
        n = p - 1
        self.n = n
        if n == 0:
            self.V = np.zeros((0, 0))
            self.D = np.zeros((0, 0, 0))
            return
        lam, V = sla.eigh(tab["K"][1:p, 1:p], tab["M"][1:p, 1:p])
        self.V = V
        L = lam
        self.D = (d[0] + d[1] * L[None, None, :] + d[2] * L[None, :, None] + d[3] * L[:, None, None])

    def _each_axis(self, X, A):
        """Apply the n x n matrix A along each of the three element axes of X (n, n, n, m)."""
        X = np.tensordot(A, X, axes=([1], [0]))                    # along k
        X = np.tensordot(A, X, axes=([1], [1])).transpose(1, 0, 2, 3)  # along j
        X = np.tensordot(A, X, axes=([1], [2])).transpose(1, 2, 0, 3)  # along i
        return X

    def apply(self, B):
        """H_II^-1 B for B of shape (n_I^3,) or (n_I^3, m)."""
        B = np.asarray(B, dtype=np.float64)
        squeeze = B.ndim == 1
        n = self.n
        X = B.reshape(n, n, n, -1)
        Y = self._each_axis(X, self.V.T) / self.D[..., None]
        Z = self._each_axis(Y, self.V).reshape(n ** 3, -1)
        return Z[:, 0] if squeeze else Z


class ElementBlocks:
    """The blocks H_BB, H_BI, H_IB, H_II of one element operator and its Schur
    complement H_BB - H_BI H_II^-1 H_IB (Sec. 4, eq. condensation_system).

    route "dense": dense H_e and a Cholesky factorisation of H_II (default for
    p <= DENSE_MAX_P); route "separable": sparse H_e blocks and
    ``SeparableInteriorSolve`` (default above).
    """

    def __init__(self, p, d, tab=None, route=None):
        tab = tab or gll.tables(p)
        self.p = p
        self.d = np.asarray(d, dtype=np.float64)
        self.route = route or ("dense" if p <= DENSE_MAX_P else "separable")
        B, I, _ = boundary_interior(p)
        self.B, self.I = B, I
        if self.route == "dense":
            H = element_operator(p, d, tab)
            self.H = H
            self.HBB = H[np.ix_(B, B)]
            self.HBI = H[np.ix_(B, I)]
            self.HIB = H[np.ix_(I, B)]
            self.HII = H[np.ix_(I, I)]
            self._ch = sla.cho_factor(self.HII, lower=True) if len(I) else None
        elif self.route == "separable":
            H = element_operator_sparse(p, d, tab)
            self.H = H
            self.HBB = H[B][:, B].tocsr()
            self.HBI = H[B][:, I].tocsr()
            self.HIB = H[I][:, B].tocsr()
            self.HII = H[I][:, I].tocsr()
            self._sep = SeparableInteriorSolve(p, d, tab)
        else:
            raise ValueError("route must be 'dense' or 'separable'")

    def interior_solve(self, X):
        """H_II^-1 X, X of shape (n_I^3,) or (n_I^3, m)."""
        if len(self.I) == 0:
            return np.zeros_like(np.asarray(X, dtype=np.float64))
        if self.route == "dense":
            return sla.cho_solve(self._ch, X)
        return self._sep.apply(X)

    def schur_apply(self, UB):
        """(H_BB - H_BI H_II^-1 H_IB) U_B for U_B of shape (n_B,) or (n_B, m)."""
        UB = np.asarray(UB, dtype=np.float64)
        out = self.HBB @ UB
        if len(self.I):
            out = out - self.HBI @ self.interior_solve(self.HIB @ UB)
        return np.asarray(out)

    def schur_matrix(self, chunk=256):
        """The Schur complement as a dense symmetric n_B x n_B matrix."""
        if self.route == "dense":
            return condense(self.H, self.B, self.I)
        nB = len(self.B)
        S = np.empty((nB, nB))
        HBBd = self.HBB.toarray()
        for c0 in range(0, nB, chunk):
            c1 = min(nB, c0 + chunk)
            S[:, c0:c1] = HBBd[:, c0:c1]
            if len(self.I):
                X = self.interior_solve(self.HIB[:, c0:c1].toarray())
                S[:, c0:c1] -= self.HBI @ X
        return 0.5 * (S + S.T)
