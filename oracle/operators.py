"""Global oracle operations on the condensed system.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything is in the physical (nodal GLL) basis and FP64.  Global vectors are
full nodal arrays of length N in lexicographic order; skeleton operations read
and write only the free skeleton entries and leave every other entry zero.

Paper passages:
* assembly R H_L R^T (Sec. 3, the discrete system);
* condensed operator and right-hand side, interior recovery (Sec. 4,
  eqs. condensation_inner / condensation_system, Algorithm 1);
* conjugate gradients with the block-Jacobi "block preconditioner" of Sec. 8:
  exact inverses of the self-blocks of faces, edges and vertices of the
  assembled condensed operator (the BC solver of Sec. 8).
"""

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import element, gll, mesh as meshmod


# ----------------------------------------------------------------------------
# Per-class element data
# ----------------------------------------------------------------------------

def element_classes(mesh):
    """Group elements by identical metric vector d_e.

    Returns (metrics (n_e,4), class_of_element (n_e,), unique metrics (n_c,4)).
    On a uniform mesh there is a single class.
    """
    d = meshmod.element_metrics(mesh)
    uniq, inv = np.unique(d, axis=0, return_inverse=True)
    return d, inv.ravel(), uniq


class CondensedOperator:
    """The assembled condensed operator sum_e R_B,e H_hat_e R_B,e^T on free nodes.

    Element operators are the explicit Schur complements of ``element.condense``
    (Sec. 4), computed once per class of identical metric.
    """

    def __init__(self, mesh, max_classes=4096):
        self.mesh = mesh
        self.p = mesh["p"]
        self.tab = gll.tables(self.p)
        self.sizes = meshmod.sizes(mesh)
        self.B, self.I, self.Bkji = element.boundary_interior(self.p)
        self.gmap = meshmod.gather_map(mesh)
        self.gB = self.gmap[:, self.B]
        self.gI = self.gmap[:, self.I]
        self.d, self.cls, self.uniq = element_classes(mesh)
        if len(self.uniq) > max_classes:
            raise MemoryError("%d element classes exceed the oracle limit" % len(self.uniq))
        # per class: the element operator's blocks (dense Cholesky route for
        # p <= 16, sparse Kronecker blocks with the separable interior inverse
        # above), and for the dense route the explicit Schur complement
        self.blocks = [element.ElementBlocks(self.p, dc, self.tab) for dc in self.uniq]
        self.H = [b.H for b in self.blocks]
        self.Hhat = [b.schur_matrix() if b.route == "dense" else None for b in self.blocks]
        self.skel = meshmod.skeleton_mask(mesh)
        self.cons = meshmod.constrained_mask(mesh)
        self.free_skel = self.skel & ~self.cons

    # -- apply ---------------------------------------------------------------
    def apply(self, u):
        """v = R Hhat_L R^T u on the free skeleton (Sec. 4).

        Face-to-face form with one dense matrix product per element class, the
        "MMC" variant of Sec. 7 (Algorithm 2 with primary part included).

        u: (N,) or (N, k); constrained and interior entries of u are ignored.
        """
        u = np.asarray(u, dtype=np.float64)
        squeeze = u.ndim == 1
        U = u[:, None] if squeeze else u
        Um = np.where(self.free_skel[:, None], U, 0.0)
        V = np.zeros_like(Um)
        for c, Hh in enumerate(self.Hhat):
            els = np.nonzero(self.cls == c)[0]
            if len(els) == 0:
                continue
            idx = self.gB[els]                              # (ne_c, nB)
            k = Um.shape[1]
            UL = Um[idx].transpose(1, 0, 2).reshape(len(self.B), -1)   # (nB, ne_c*k)
            if Hh is not None:
                VL = (Hh @ UL).reshape(len(self.B), len(els), k)      # one GEMM per class
            else:
                VL = self._schur_apply_chunked(c, UL).reshape(len(self.B), len(els), k)
            for r in range(k):
                V[:, r] += np.bincount(idx.T.ravel(), weights=VL[:, :, r].ravel(),
                                       minlength=len(V))
        V[~self.free_skel] = 0.0
        return V[:, 0] if squeeze else V

    def _schur_apply_chunked(self, c, UL, chunk=512):
        """Schur complement of class c applied to the columns of UL (large-p route)."""
        out = np.empty_like(UL)
        for c0 in range(0, UL.shape[1], chunk):
            out[:, c0:c0 + chunk] = self.blocks[c].schur_apply(UL[:, c0:c0 + chunk])
        return out

    def schur(self, c):
        """Explicit Schur complement of class c (formed on first use for p > 16)."""
        if self.Hhat[c] is None:
            self.Hhat[c] = self.blocks[c].schur_matrix()
        return self.Hhat[c]

    @staticmethod
    def _local_coo(H):
        """Local (row, col, value) triples of a dense or sparse element matrix."""
        if sp.issparse(H):
            h = H.tocoo()
            return h.row, h.col, h.data
        n = H.shape[0]
        return np.repeat(np.arange(n), n), np.tile(np.arange(n), n), H.ravel()

    # -- sparse assembled matrices -------------------------------------------
    def assembled_condensed(self):
        """Sparse Hhat_G restricted to free skeleton nodes, with their numbers."""
        rows, cols, vals = [], [], []
        for e in range(len(self.gB)):
            Hh = self.schur(self.cls[e])
            g = self.gB[e]
            rows.append(np.repeat(g, len(g)))
            cols.append(np.tile(g, len(g)))
            vals.append(Hh.ravel())
        N = self.sizes["N"]
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(N, N)).tocsr()
        fs = np.nonzero(self.free_skel)[0]
        return A[fs][:, fs].tocsc(), fs

    def assembled_full(self):
        """Sparse full uncondensed H_G = R H_L R^T restricted to free nodes."""
        rows, cols, vals = [], [], []
        for e in range(len(self.gmap)):
            lr, lc, lv = self._local_coo(self.H[self.cls[e]])
            g = self.gmap[e]
            rows.append(g[lr])
            cols.append(g[lc])
            vals.append(lv)
        N = self.sizes["N"]
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(N, N)).tocsr()
        fr = np.nonzero(~self.cons)[0]
        return A[fr][:, fr].tocsc(), fr

    # -- right-hand side -------------------------------------------------------
    def element_rhs(self, f):
        """Element-local F_e = J_e (W (x) W (x) W) f_e, shape (n_e, (p+1)^3[, k]).

        The GLL-lumped mass matrix of element e is J_e W(x)W(x)W with
        J_e = h1 h2 h3 / 8 (Sec. 3); F_L = M_L f is the discretised RHS of the
        discrete system R H_L R^T u_G = R F_L.
        """
        w = self.tab["w"]
        W3 = element.kron3(np.diag(w), np.diag(w), np.diag(w)).diagonal()
        J = meshmod.element_jacobians(self.mesh)
        f = np.asarray(f, dtype=np.float64)
        fe = f[self.gmap]
        if f.ndim == 1:
            return J[:, None] * W3[None, :] * fe
        return J[:, None, None] * W3[None, :, None] * fe

    def condensed_rhs(self, f):
        """F_hat = R (F_B - H_BI H_II^-1 F_I) on the free skeleton (Sec. 4, Alg. 1)."""
        f = np.asarray(f, dtype=np.float64)
        squeeze = f.ndim == 1
        F = self.element_rhs(f)
        if squeeze:
            F = F[:, :, None]
        N = self.sizes["N"]
        out = np.zeros((N, F.shape[2]))
        for c, blk in enumerate(self.blocks):
            els = np.nonzero(self.cls == c)[0]
            if len(els) == 0:
                continue
            for r in range(F.shape[2]):
                FI = F[els][:, self.I, r].T                  # (nI, ne_c)
                corr = blk.HBI @ blk.interior_solve(FI)      # (nB, ne_c)
                FB = F[els][:, self.B, r].T - corr
                out[:, r] += np.bincount(self.gB[els].ravel(), weights=FB.T.ravel(), minlength=N)
        out[~self.free_skel] = 0.0
        return out[:, 0] if squeeze else out

    def assembled_rhs(self, f):
        """R F_L (full, uncondensed) on free nodes."""
        F = self.element_rhs(f)
        N = self.sizes["N"]
        out = np.bincount(self.gmap.ravel(), weights=F.ravel(), minlength=N)
        out[self.cons] = 0.0
        return out

    # -- solves ----------------------------------------------------------------
    def solve_condensed(self, f):
        """Skeleton solution Hhat_G^-1 F_hat by sparse LU; returns (N,) with skeleton entries."""
        A, fs = self.assembled_condensed()
        rhs = self.condensed_rhs(f)
        lu = spla.splu(A)
        out = np.zeros(self.sizes["N"])
        out[fs] = lu.solve(rhs[fs])
        return out

    def solve_full_dirichlet(self, f, g):
        """Full uncondensed direct solve with prescribed values on the Dirichlet nodes.

        u = g on the nodes of the Dirichlet domain faces; on the free nodes
        (R H_L R^T)_FF u_F = (R F_L)_F - (R H_L R^T)_FD g_D, i.e. the discrete
        system of Sec. 3 with the known values moved to the right-hand side.
        f, g: nodal arrays (N,); returns the full nodal solution (N,).
        """
        rows, cols, vals = [], [], []
        for e in range(len(self.gmap)):
            lr, lc, lv = self._local_coo(self.H[self.cls[e]])
            gm = self.gmap[e]
            rows.append(gm[lr])
            cols.append(gm[lc])
            vals.append(lv)
        N = self.sizes["N"]
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(N, N)).tocsr()
        F = np.bincount(self.gmap.ravel(), weights=self.element_rhs(f).ravel(), minlength=N)
        fr = np.nonzero(~self.cons)[0]
        dn = np.nonzero(self.cons)[0]
        u = np.zeros(N)
        u[dn] = np.asarray(g, dtype=np.float64)[dn]
        rhs = F[fr] - A[fr][:, dn] @ u[dn]
        u[fr] = spla.splu(A[fr][:, fr].tocsc()).solve(rhs)
        return u

    def solve_full(self, f):
        """Full uncondensed direct solve of R H_L R^T u = R F_L on free nodes."""
        A, fr = self.assembled_full()
        rhs = self.assembled_rhs(f)
        lu = spla.splu(A)
        out = np.zeros(self.sizes["N"])
        out[fr] = lu.solve(rhs[fr])
        return out

    def recover_interior(self, f, u_skel):
        """Fill interior nodes: u_I = H_II^-1 (F_I - H_IB u_B) per element (Alg. 1)."""
        F = self.element_rhs(f)
        u = np.array(u_skel, dtype=np.float64)
        um = np.where(self.free_skel, u, 0.0)
        for c, blk in enumerate(self.blocks):
            els = np.nonzero(self.cls == c)[0]
            if len(els) == 0:
                continue
            uB = um[self.gB[els]].T                          # (nB, ne_c)
            uI = blk.interior_solve(F[els][:, self.I].T - blk.HIB @ uB)
            u[self.gI[els]] = uI.T
        u[self.cons] = 0.0
        return u

    # -- entities and the block preconditioner -------------------------------
    def entity_ids(self):
        """Entity id of every free skeleton node (global faces, edges, vertices).

        A skeleton node lies on a vertex if all three global indices are
        multiples of p, on an edge if two are, on a face if one is.  Nodes of
        one entity share the pattern and the integer parts of I_a / p.
        """
        p = self.p
        G = meshmod.global_ijk(self.mesh)
        fs = np.nonzero(self.free_skel)[0]
        Gs = G[fs]
        pat = (Gs % p == 0).astype(np.int64)
        # nodes with I_a % p == 0 lie on the entity plane I_a / p, the others in
        # the element slab I_a // p: either way the key is I_a // p.
        key = np.concatenate([pat, Gs // p], axis=1)
        _, ids = np.unique(key, axis=0, return_inverse=True)
        return fs, ids.ravel()

    def block_jacobi(self):
        """Dense inverses of each entity's self-block of Hhat_G (Sec. 8, BC)."""
        A, fs = self.assembled_condensed()
        fs2, ids = self.entity_ids()
        assert np.array_equal(fs, fs2)
        A = A.tocsr()
        blocks = []
        for ent in range(ids.max() + 1 if len(ids) else 0):
            loc = np.nonzero(ids == ent)[0]
            blk = A[loc][:, loc].toarray()
            blocks.append((loc, np.linalg.inv(blk)))
        return blocks

    def bc_pcg(self, f=None, rhs=None, tol=1e-10, maxit=10000, fixed_iters=None):
        """Block-Jacobi PCG on the condensed system in the physical basis (Sec. 8).

        Conjugate gradients with x0 = 0; stops when ||r||_2 <= tol ||b||_2 (the
        Euclidean residual reduced by 1/tol, Sec. 8), or after ``fixed_iters``
        iterations if given.  Returns (x (N,), info) with the alpha and beta
        sequences, the residual norms and the iteration count.
        """
        A, fs = self.assembled_condensed()
        b = (self.condensed_rhs(f) if rhs is None else np.asarray(rhs))[fs]
        blocks = self.block_jacobi()

        def prec(r):
            z = np.zeros_like(r)
            for loc, inv in blocks:
                z[loc] = inv @ r[loc]
            return z

        x = np.zeros_like(b)
        r = b.copy()
        z = prec(r)
        pvec = z.copy()
        rho = r @ z
        bnorm = np.linalg.norm(b)
        alphas, betas, res = [], [], [np.linalg.norm(r)]
        it = 0
        while True:
            if fixed_iters is None and (res[-1] <= tol * bnorm or it >= maxit):
                break
            if fixed_iters is not None and it >= fixed_iters:
                break
            q = A @ pvec
            alpha = rho / (pvec @ q)
            x += alpha * pvec
            r -= alpha * q
            z = prec(r)
            rho_new = r @ z
            beta = rho_new / rho
            pvec = z + beta * pvec
            rho = rho_new
            alphas.append(alpha)
            betas.append(beta)
            res.append(np.linalg.norm(r))
            it += 1
        out = np.zeros(self.sizes["N"])
        out[fs] = x
        return out, {"alpha": np.array(alphas), "beta": np.array(betas),
                     "res": np.array(res), "iters": it, "bnorm": bnorm}
