"""Oracle rows of the assembled condensed operator at single nodes, for
meshes too large for the oracle's assembled operator (test helper).

For a global node, every incident element's condensed operator is formed from
its definitions (explicit element matrix, Schur complement by Cholesky,
Sec. 4), applied to that element's boundary values, and the node's rows are
summed (the assembly R of Sec. 3).  Values on Dirichlet faces are read as 0.
"""

import itertools

import numpy as np
import scipy.linalg as sla

from oracle import element as OE
from oracle import gll


class SampledOracle:
    """Rows of R_B blockdiag(H^_e) R_B^T u at chosen global nodes."""

    def __init__(self, wmesh):
        self.m = wmesh
        self.p = wmesh["p"]
        self.n = wmesh["n"]
        self.tab = gll.tables(self.p)
        self.B, self.I, _ = OE.boundary_interior(self.p)
        self.cache = {}
        self.N1, self.N2, self.N3 = (a * self.p + 1 for a in self.n)

    def constrained(self, I):
        Nax = (self.N1, self.N2, self.N3)
        bits = self.m["dirichlet"]
        for a in range(3):
            if (bits >> (2 * a)) & 1 and I[a] == 0:
                return True
            if (bits >> (2 * a + 1)) & 1 and I[a] == Nax[a] - 1:
                return True
        return False

    def elements_of(self, I):
        cands = []
        for a in range(3):
            q, r = divmod(I[a], self.p)
            c = [q] if r else [q - 1, q]
            cands.append([e for e in c if 0 <= e < self.n[a]])
        return list(itertools.product(*cands))

    def element_out(self, e, u_of_node):
        """H^_e u_B for element e = (e1, e2, e3): full boundary vector (element order of B)."""
        e1, e2, e3 = e
        w = self.m["widths"]
        lam = self.m["lam"]
        d = OE.metric((w[0][e1], w[1][e2], w[2][e3]), lam)
        key = tuple(d)
        if key not in self.cache:
            if len(self.cache) >= 8:          # bounded host memory at large p
                self.cache.pop(next(iter(self.cache)))
            H = OE.element_operator(self.p, d, self.tab)
            c = sla.cho_factor(H[np.ix_(self.I, self.I)], lower=True) if len(self.I) else None
            self.cache[key] = (H, c)
        H, c = self.cache[key]
        p1 = self.p + 1
        kk, rem = np.divmod(self.B, p1 * p1)
        jj, ii = np.divmod(rem, p1)
        I1, I2, I3 = e1 * self.p + ii, e2 * self.p + jj, e3 * self.p + kk
        uB = np.array([0.0 if self.constrained((a, b, cc)) else u_of_node(a, b, cc)
                       for a, b, cc in zip(I1, I2, I3)])
        out = H[np.ix_(self.B, self.B)] @ uB
        if c is not None:
            out -= H[np.ix_(self.B, self.I)] @ sla.cho_solve(c, H[np.ix_(self.I, self.B)] @ uB)
        return out, (I1, I2, I3)

    def row(self, I, u_of_node, memo):
        total = 0.0
        for e in self.elements_of(I):
            if e not in memo:
                memo[e] = self.element_out(e, u_of_node)
            out, (I1, I2, I3) = memo[e]
            pos = np.nonzero((I1 == I[0]) & (I2 == I[1]) & (I3 == I[2]))[0]
            assert len(pos) == 1
            total += out[pos[0]]
        return total
