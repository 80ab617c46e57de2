"""Gradient oracle for the loss L = 1/2 sum_k ||u_k - t_k||^2 over free skeleton nodes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The forward map is the discrete system of Sec. 3, H_G u = M_G f with
H_G = R H_L R^T and H_e = sum_m d_{e,m} A_m (eq. helmholtz_operator); the
skeleton part of u is what static condensation returns (Sec. 4).  The adjoint
of the full uncondensed system gives, for any parameter theta,

    dL/dtheta = -a^T (dH_G/dtheta) u + a^T d(M_G f)/dtheta,   H_G a = dL/du,

with dL/du = u - t on free skeleton nodes and 0 elsewhere.  Parameters:
* the per-element metric coefficients d_{e,m} (taken as independent inputs,
  right-hand side held fixed): dL/dd_{e,m} = -a_e^T A_m u_e;
* the per-element Helmholtz parameter lambda_e, d_{e,0} = J_e lambda_e:
  dL/dlambda_e = J_e dL/dd_{e,0};
* the nodal right-hand side f: dL/df = M_G a on free nodes.
"""

import numpy as np
import scipy.sparse.linalg as spla

from . import element, mesh as meshmod
from .operators import CondensedOperator


def loss_and_grads(mesh, f, t):
    """Direct-solve loss and gradients.

    f: (N, k) nodal right-hand sides; t: (N, k) targets (only free skeleton
    entries are used).  Returns dict with u (N,k), a (N,k), loss, g_d (n_e,4),
    g_lam (n_e,), g_f (N,k).
    """
    op = CondensedOperator(mesh)
    f = np.asarray(f, dtype=np.float64)
    if f.ndim == 1:
        f = f[:, None]
    t = np.asarray(t, dtype=np.float64).reshape(f.shape)
    A, fr = op.assembled_full()
    lu = spla.splu(A)
    N = op.sizes["N"]
    k = f.shape[1]
    u = np.zeros((N, k))
    a = np.zeros((N, k))
    loss = 0.0
    fs = op.free_skel
    for r in range(k):
        rhs = op.assembled_rhs(f[:, r])
        u[fr, r] = lu.solve(rhs[fr])
        g = np.where(fs, u[:, r] - t[:, r], 0.0)
        loss += 0.5 * float(g @ g)
        a[fr, r] = lu.solve(g[fr])       # H_G is symmetric
    terms = element.stiffness_terms(mesh["p"], op.tab)
    gmap = op.gmap
    n_e = len(gmap)
    g_d = np.zeros((n_e, 4))
    for e in range(n_e):
        ue = u[gmap[e]]
        ae = a[gmap[e]]
        for m in range(4):
            g_d[e, m] = -np.sum(ae * (terms[m] @ ue))
    J = meshmod.element_jacobians(mesh)
    g_lam = J * g_d[:, 0]
    w = op.tab["w"]
    W3 = element.kron3(np.diag(w), np.diag(w), np.diag(w)).diagonal()
    MG = np.bincount(gmap.ravel(), weights=(J[:, None] * W3[None, :]).ravel(), minlength=N)
    g_f = MG[:, None] * a
    g_f[op.cons] = 0.0
    return {"u": u, "a": a, "loss": loss, "g_d": g_d, "g_lam": g_lam, "g_f": g_f}


def loss_only(mesh, f, t):
    """Loss of the direct solve (for central finite differences)."""
    op = CondensedOperator(mesh)
    f = np.asarray(f, dtype=np.float64)
    if f.ndim == 1:
        f = f[:, None]
    t = np.asarray(t, dtype=np.float64).reshape(f.shape)
    A, fr = op.assembled_full()
    lu = spla.splu(A)
    loss = 0.0
    for r in range(f.shape[1]):
        rhs = op.assembled_rhs(f[:, r])
        u = np.zeros(op.sizes["N"])
        u[fr] = lu.solve(rhs[fr])
        g = np.where(op.free_skel, u - t[:, r], 0.0)
        loss += 0.5 * float(g @ g)
    return loss
