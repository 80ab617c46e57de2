"""1D spectral basis of the oracle: GLL nodes and weights, M and K.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper passages followed (Sec. 3, "The spectral-element method for cuboidal
elements"):
* the 1D nodal basis is the set of Lagrange polynomials through the
  Gauss-Lobatto-Legendre (GLL) points of degree p, so GLL points are the
  degrees of freedom;
* M_ij = int_{-1}^{1} phi_i phi_j, approximated by GLL quadrature, which makes
  M diagonal with the GLL weights on the diagonal;
* K_ij = int_{-1}^{1} phi_i' phi_j'.

Two independent evaluations live here:
* ``tables(p)``      -- numpy, evaluated in x87 extended precision and rounded
                        to FP64: Legendre-series root finding for the nodes,
                        barycentric Lagrange differentiation, and K from exact
                        GLL quadrature of phi_i' phi_j' (degree 2p-2);
* ``tables_mp(p)``   -- mpmath at high precision with a different algorithm:
                        exact rational Legendre coefficients, polynomial roots,
                        and K/weights by exact term-wise integration of the
                        Lagrange polynomials' coefficient expansions.  Used only
                        as a pin for ``tables``.
"""

from fractions import Fraction

import numpy as np
from numpy.polynomial import legendre as npleg


# ----------------------------------------------------------------------------
# FP64 tables (the oracle proper)
# ----------------------------------------------------------------------------

def gll_nodes_weights(p, dtype=np.float64):
    """GLL nodes x_0 < ... < x_p on [-1, 1] and weights w_i.

    Nodes: -1, +1 and the p-1 roots of P_p' (Sec. 3, GLL paragraph).
    Weights: w_i = 2 / (p (p+1) P_p(x_i)^2), the Lobatto quadrature weights,
    which are the diagonal of the GLL-lumped mass matrix.  ``dtype`` may be
    np.longdouble (x87 extended precision), used by ``tables`` internally.
    """
    if p < 1:
        raise ValueError("p must be >= 1")
    c = np.zeros(p + 1)
    c[p] = 1.0
    dc = npleg.legder(c)
    d2c = npleg.legder(dc)
    cl, dcl, d2cl = (a.astype(dtype) for a in (c, dc, d2c))
    if p >= 2:
        r = np.sort(np.real(npleg.legroots(dc))).astype(dtype)
        # Newton polish of the interior roots on P_p'(x) = 0.
        for _ in range(4):
            r = r - npleg.legval(r, dcl) / npleg.legval(r, d2cl)
        x = np.concatenate((np.array([-1.0], dtype=dtype), r, np.array([1.0], dtype=dtype)))
    else:
        x = np.array([-1.0, 1.0], dtype=dtype)
    Pp = npleg.legval(x, cl)
    w = 2.0 / (p * (p + 1) * Pp * Pp)
    return x, w


def diff_matrix(x):
    """Lagrange differentiation matrix D_ij = phi_j'(x_i) for nodes x.

    Textbook barycentric form: D_ij = (b_j / b_i) / (x_i - x_j) with
    barycentric weights b_i = 1 / prod_{m != i} (x_i - x_m); the diagonal is the
    negative row sum (derivative of the constant function is zero).  Works in
    the dtype of ``x``.
    """
    n = len(x)
    diffs = x[:, None] - x[None, :]
    np.fill_diagonal(diffs, 1.0)
    b = 1.0 / np.prod(diffs, axis=1)
    D = (b[None, :] / b[:, None]) / diffs
    np.fill_diagonal(D, 0.0)
    D[np.arange(n), np.arange(n)] = -D.sum(axis=1)
    return D


def tables(p):
    """FP64 1D tables for degree p: dict with x, w, D, M, K.

    K = D^T W D is exact: phi_i' phi_j' has degree 2p-2 <= 2p-1, which GLL
    quadrature integrates exactly.  Nodes, weights, D and K are evaluated in
    x87 extended precision and rounded once to FP64, so K is correctly rounded
    up to about one unit in the last place even at p = 32.
    """
    xl, wl = gll_nodes_weights(p, dtype=np.longdouble)
    Dl = diff_matrix(xl)
    Kl = Dl.T @ (wl[:, None] * Dl)
    Kl = 0.5 * (Kl + Kl.T)
    x = xl.astype(np.float64)
    w = wl.astype(np.float64)
    return {"p": p, "x": x, "w": w, "D": Dl.astype(np.float64), "M": np.diag(w),
            "K": Kl.astype(np.float64)}


# ----------------------------------------------------------------------------
# High-precision pin (independent algorithm)
# ----------------------------------------------------------------------------

def _legendre_coeffs_exact(n):
    """Monomial coefficients (low to high) of P_n as exact Fractions.

    Bonnet recurrence (m+1) P_{m+1} = (2m+1) x P_m - m P_{m-1}.
    """
    P0 = [Fraction(1)]
    if n == 0:
        return P0
    P1 = [Fraction(0), Fraction(1)]
    for m in range(1, n):
        nxt = [Fraction(0)] * (m + 2)
        for a, c in enumerate(P1):
            nxt[a + 1] += Fraction(2 * m + 1, m + 1) * c
        for a, c in enumerate(P0):
            nxt[a] -= Fraction(m, m + 1) * c
        P0, P1 = P1, nxt
    return P1


def tables_mp(p, dps=50):
    """High-precision 1D tables (x, w, K as mpmath matrices / lists).

    Nodes: -1, +1 and the roots of P_p' from the exact rational coefficients.
    Weights: w_i = int_{-1}^{1} phi_i (GLL quadrature is exact for phi_i).
    K_ij = int_{-1}^{1} phi_i' phi_j' by exact term-wise integration.
    """
    import mpmath as mp

    with mp.workdps(dps):
        P = _legendre_coeffs_exact(p)
        dP = [a * P[a] for a in range(1, len(P))]  # low -> high
        if p >= 2:
            # mpmath.polyroots wants high -> low coefficients
            roots = mp.polyroots([mp.mpf(c.numerator) / c.denominator for c in dP[::-1]],
                                 maxsteps=400, extraprec=4 * dps)
            roots = sorted(mp.re(r) for r in roots)
            x = [mp.mpf(-1)] + list(roots) + [mp.mpf(1)]
        else:
            x = [mp.mpf(-1), mp.mpf(1)]
        n = p + 1

        def polymul(a, b):
            out = [mp.mpf(0)] * (len(a) + len(b) - 1)
            for i, ai in enumerate(a):
                if ai == 0:
                    continue
                for j, bj in enumerate(b):
                    out[i + j] += ai * bj
            return out

        def integrate(c):
            return sum(2 * c[m] / (m + 1) for m in range(0, len(c), 2))

        phis = []
        for i in range(n):
            poly = [mp.mpf(1)]
            for m in range(n):
                if m == i:
                    continue
                den = x[i] - x[m]
                poly = polymul(poly, [-x[m] / den, 1 / den])
            phis.append(poly)
        dphis = [[a * c[a] for a in range(1, len(c))] for c in phis]
        w = [integrate(c) for c in phis]
        K = mp.matrix(n, n)
        for i in range(n):
            for j in range(i, n):
                v = integrate(polymul(dphis[i], dphis[j]))
                K[i, j] = v
                K[j, i] = v
        return {"p": p, "x": x, "w": w, "K": K}


def mp_to_numpy(tab):
    """Round an mpmath table (from ``tables_mp``) to float64 numpy arrays."""
    x = np.array([float(v) for v in tab["x"]])
    w = np.array([float(v) for v in tab["w"]])
    n = len(x)
    K = np.array([[float(tab["K"][i, j]) for j in range(n)] for i in range(n)])
    return x, w, K
