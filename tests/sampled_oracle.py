"""Oracle rows of the assembled condensed operator at single nodes, for
meshes too large for the oracle's assembled operator (test helper).

For a global node, every incident element's condensed operator is formed from
its definitions (explicit element matrix and the Schur complement of Sec. 4:
dense Cholesky for p <= 16, sparse Kronecker blocks with the separable interior
inverse above), applied to that element's boundary values, and the node's rows
are summed (the assembly R of Sec. 3).  Values on Dirichlet faces are read as 0.
Per-element lambda (``lam_e``, element order e1 fastest) is honoured.
"""

import itertools

import numpy as np

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
        lam_e = self.m.get("lam_e")
        lam = self.m["lam"] if lam_e is None else lam_e[e1 + self.n[0] * (e2 + self.n[1] * e3)]
        d = OE.metric((w[0][e1], w[1][e2], w[2][e3]), lam)
        key = tuple(d)
        if key not in self.cache:
            if len(self.cache) >= 8:          # bounded host memory at large p
                self.cache.pop(next(iter(self.cache)))
            self.cache[key] = OE.ElementBlocks(self.p, d, self.tab)
        blk = self.cache[key]
        p1 = self.p + 1
        kk, rem = np.divmod(self.B, p1 * p1)
        jj, ii = np.divmod(rem, p1)
        I1, I2, I3 = e1 * self.p + ii, e2 * self.p + jj, e3 * self.p + kk
        uB = np.array([0.0 if self.constrained((a, b, cc)) else u_of_node(a, b, cc)
                       for a, b, cc in zip(I1, I2, I3)])
        return blk.schur_apply(uB), (I1, I2, I3)

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
