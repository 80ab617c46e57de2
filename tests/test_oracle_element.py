"""Pins of the oracle's element operator and static condensation (Secs. 3-6).

Pins used (none re-types the oracle's own formula):
* closed-form action of H_e on trilinear functions: for lambda = 0 these are
  discretely harmonic, so the Schur complement must reproduce H_e u on B;
* Schur complement as energy minimiser over interior values;
* symmetry / definiteness / null space of the condensed operator;
* an independent route to H_II^-1 (fast diagonalisation, Sec. 5) and the
  transformed-basis factorisation of Sec. 6 (Table 2, diagonal face blocks).
"""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import element, gll


def _kji(p):
    n = p + 1
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return kk.ravel(), jj.ravel(), ii.ravel()


def test_metric_reference_element():
    # a 2x2x2 element is the reference element: J = 1, d = (lam, 1, 1, 1)
    np.testing.assert_allclose(element.metric((2, 2, 2), 3.0), [3.0, 1.0, 1.0, 1.0])
    # h = (1, 2, 4): J = 1, d1 = 4, d2 = 1, d3 = 1/4
    np.testing.assert_allclose(element.metric((1, 2, 4), 0.5), [0.5, 4.0, 1.0, 0.25])


@pytest.mark.parametrize("p", [2, 3, 4, 6, 8])
def test_trilinear_modes_closed_form(p):
    """lambda = 0: H_hat u_B = (H u)_B, with (H u) in closed form.

    For u = f3(xi3) f2(xi2) f1(xi1), f in {1, xi}: the GLL quadrature of
    phi_i' * f' gives K 1 = 0 and K xi = e_p - e_0, so e.g.
    (H xi1)_{kji} = d1 w_k w_j (delta_ip - delta_i0).
    """
    t = gll.tables(p)
    x, w = t["x"], t["w"]
    d = np.array([0.0, 1.7, 0.6, 2.3])
    H = element.element_operator(p, d, t)
    B, I, _ = element.boundary_interior(p)
    Hh = element.condense(H, B, I)
    kk, jj, ii = _kji(p)
    ends = lambda idx: (idx == p).astype(float) - (idx == 0).astype(float)
    for e3 in (0, 1):
        for e2 in (0, 1):
            for e1 in (0, 1):
                f1 = x[ii] if e1 else np.ones_like(x[ii])
                f2 = x[jj] if e2 else np.ones_like(x[jj])
                f3 = x[kk] if e3 else np.ones_like(x[kk])
                u = f1 * f2 * f3
                Hu = np.zeros_like(u)
                if e1:
                    Hu += d[1] * w[kk] * f3 * w[jj] * f2 * ends(ii)
                if e2:
                    Hu += d[2] * w[kk] * f3 * ends(jj) * w[ii] * f1
                if e3:
                    Hu += d[3] * ends(kk) * w[jj] * f2 * w[ii] * f1
                # closed form has no interior part: the mode is discretely harmonic
                assert np.abs(Hu[I]).max() == 0.0
                np.testing.assert_allclose(H @ u, Hu, atol=1e-12)
                np.testing.assert_allclose(Hh @ u[B], Hu[B], atol=1e-12)


@pytest.mark.parametrize("p", [2, 3, 5, 8])
def test_condensed_is_energy_minimum(p):
    rng = np.random.default_rng(p)
    d = np.array([0.3, 1.1, 0.9, 2.0])
    t = gll.tables(p)
    H = element.element_operator(p, d, t)
    B, I, _ = element.boundary_interior(p)
    Hh = element.condense(H, B, I)
    uB = rng.standard_normal(len(B))
    u = np.zeros(H.shape[0])
    u[B] = uB
    u[I] = element.recover_interior_element(H, B, I, np.zeros(H.shape[0]), uB)
    e0 = u @ H @ u
    np.testing.assert_allclose(uB @ Hh @ uB, e0, rtol=1e-12)
    for _ in range(5):
        v = u.copy()
        v[I] += 1e-3 * rng.standard_normal(len(I))
        assert v @ H @ v > e0


@pytest.mark.parametrize("p", [2, 3, 4, 6])
@pytest.mark.parametrize("lam", [0.0, 1.0])
def test_condensed_symmetry_and_nullspace(p, lam):
    d = element.metric((0.5, 0.25, 1.0), lam)
    Hh, B, _ = element.condensed_element_operator(p, d)
    np.testing.assert_array_equal(Hh, Hh.T)
    ev = np.linalg.eigvalsh(Hh)
    if lam == 0.0:
        assert abs(ev[0]) < 1e-12 * ev[-1]
        assert ev[1] > 1e-8 * ev[-1]
        assert np.abs(Hh @ np.ones(len(B))).max() < 1e-12 * ev[-1]
    else:
        assert ev[0] > 1e-10 * ev[-1]


def _fast_diag(p, t):
    Ii = slice(1, p)
    lam, S = sla.eigh(t["K"][Ii, Ii], t["M"][Ii, Ii])
    return lam, S


@pytest.mark.parametrize("p", [3, 5, 8])
def test_fast_diagonalisation_inverse(p):
    """H_II^-1 = (S(x)S(x)S) D^-1 (S(x)S(x)S)^T, D = d0 + d1 L_i + d2 L_j + d3 L_k (Sec. 5)."""
    t = gll.tables(p)
    lam, S = _fast_diag(p, t)
    d = np.array([0.7, 1.3, 0.4, 2.2])
    H = element.element_operator(p, d, t)
    _, I, _ = element.boundary_interior(p)
    HII = H[np.ix_(I, I)]
    one = np.ones(p - 1)
    D = (d[0] + d[1] * np.kron(one, np.kron(one, lam)) + d[2] * np.kron(one, np.kron(lam, one))
         + d[3] * np.kron(lam, np.kron(one, one)))
    S3 = element.kron3(S, S, S)
    inv_fd = S3 @ np.diag(1.0 / D) @ S3.T
    np.testing.assert_allclose(inv_fd @ HII, np.eye(len(I)), atol=1e-11)


def _transformed_apply(p, t, d, U):
    """Transformed condensed apply of one element, written from Sec. 6 / Table 2.

    U is the element's transformed boundary vector laid out on the full
    (p+1)^3 cube (interior entries ignored).  Returns V on the cube (interior 0).
    """
    lam, S = _fast_diag(p, t)
    Ii = slice(1, p)
    a = S.T @ t["K"][Ii, 0]
    b = S.T @ t["K"][Ii, p]
    m0, K00, K0p = t["w"][0], t["K"][0, 0], t["K"][0, p]
    n = p + 1
    # 1D transformed matrices
    Mt = np.diag(np.concatenate(([m0], np.ones(p - 1), [m0])))
    Kt = np.zeros((n, n))
    Kt[0, 0] = Kt[p, p] = K00
    Kt[0, p] = Kt[p, 0] = K0p
    Kt[Ii, Ii] = np.diag(lam)
    Kt[Ii, 0] = Kt[0, Ii] = a
    Kt[Ii, p] = Kt[p, Ii] = b
    U = U.reshape(n, n, n).copy()
    isI = np.zeros(n, bool)
    isI[1:p] = True
    interior = isI[:, None, None] & isI[None, :, None] & isI[None, None, :]
    U[interior] = 0.0
    # primary part: restriction of sum_m d_m (x)-products to B x B
    V = (d[0] * np.einsum("a,b,c,abc->abc", np.diag(Mt), np.diag(Mt), np.diag(Mt), U)
         + d[1] * np.einsum("a,b,cz,abz->abc", np.diag(Mt), np.diag(Mt), Kt, U)
         + d[2] * np.einsum("a,by,c,ayc->abc", np.diag(Mt), Kt, np.diag(Mt), U)
         + d[3] * np.einsum("ax,b,c,xbc->abc", Kt, np.diag(Mt), np.diag(Mt), U))
    V[interior] = 0.0
    # condensed part (Table 2): face -> eigenspace, D^-1, eigenspace -> face
    Uw, Ue = U[1:p, 1:p, 0], U[1:p, 1:p, p]
    Us, Un = U[1:p, 0, 1:p], U[1:p, p, 1:p]
    Ub, Ut = U[0, 1:p, 1:p], U[p, 1:p, 1:p]
    uc = (d[1] * (Uw[:, :, None] * a[None, None, :] + Ue[:, :, None] * b[None, None, :])
          + d[2] * (Us[:, None, :] * a[None, :, None] + Un[:, None, :] * b[None, :, None])
          + d[3] * (Ub[None, :, :] * a[:, None, None] + Ut[None, :, :] * b[:, None, None]))
    Dd = (d[0] + d[1] * lam[None, None, :] + d[2] * lam[None, :, None] + d[3] * lam[:, None, None])
    vc = uc / Dd
    V[1:p, 1:p, 0] -= d[1] * vc @ a
    V[1:p, 1:p, p] -= d[1] * vc @ b
    V[1:p, 0, 1:p] -= d[2] * np.einsum("kji,j->ki", vc, a)
    V[1:p, p, 1:p] -= d[2] * np.einsum("kji,j->ki", vc, b)
    V[0, 1:p, 1:p] -= d[3] * np.einsum("kji,k->ji", vc, a)
    V[p, 1:p, 1:p] -= d[3] * np.einsum("kji,k->ji", vc, b)
    return V.ravel(), S


@pytest.mark.parametrize("p", [2, 3, 4, 7])
def test_transformed_factorisation_matches_schur(p):
    """T^T H_hat T (oracle Schur complement) equals the factorised transformed
    operator of Sec. 6 (primary part from M~, K~; condensed part from Table 2),
    with T = S1(x)S1(x)S1, S1 = diag(1, S, 1), S^T M_II S = I."""
    t = gll.tables(p)
    d = np.array([0.8, 1.9, 0.35, 1.2])
    H = element.element_operator(p, d, t)
    B, I, _ = element.boundary_interior(p)
    Hh = element.condense(H, B, I)
    _, S = _fast_diag(p, t)
    S1 = np.eye(p + 1)
    S1[1:p, 1:p] = S
    T = element.kron3(S1, S1, S1)
    TB = T[np.ix_(B, B)]
    assert np.abs(T[np.ix_(B, I)]).max() == 0.0     # T does not mix B and I
    Ht = TB.T @ Hh @ TB
    rng = np.random.default_rng(1)
    for _ in range(3):
        u = rng.standard_normal((p + 1) ** 3)
        v, _ = _transformed_apply(p, t, d, u)
        np.testing.assert_allclose(v[B], Ht @ u[B], atol=1e-12 * np.abs(Ht).max())
    # face self-blocks of the transformed condensed operator are diagonal
    kk, jj, ii = _kji(p)
    isI = lambda q: (q > 0) & (q < p)
    w_face = np.nonzero((ii[B] == 0) & isI(jj[B]) & isI(kk[B]))[0]
    blk = Ht[np.ix_(w_face, w_face)]
    assert np.abs(blk - np.diag(np.diag(blk))).max() < 1e-12 * np.abs(blk).max()


# ---------------------------------------------------------------------------
# Large-p route (sparse Kronecker blocks, separable interior inverse)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("p", [8, 12, 16])
def test_separable_route_matches_dense_cholesky(p):
    """The separable route's Schur complement equals the dense Cholesky one
    for general metrics (lambda > 0, anisotropic), at every p the dense route
    reaches."""
    t = gll.tables(p)
    for d in (np.array([0.8, 1.7, 0.6, 2.3]), element.metric((0.01, 0.5, 1.28), 3.0)):
        dense = element.ElementBlocks(p, d, t, route="dense")
        sep = element.ElementBlocks(p, d, t, route="separable")
        S_d = dense.schur_matrix()
        S_s = sep.schur_matrix()
        assert np.abs(S_s - S_d).max() <= 1e-12 * np.abs(S_d).max()
        U = np.random.default_rng(p).standard_normal((len(dense.B), 3))
        a, b = dense.schur_apply(U), sep.schur_apply(U)
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)


@pytest.mark.parametrize("p", [18, 24, 32])
def test_separable_route_against_explicit_operator(p):
    """At large p, against the explicit sparse element operator: the interior
    values u_I = -H_II^-1 H_IB u_B make (H u)_I vanish (energy minimum over the
    interior), and the Schur complement applied to u_B equals (H u)_B."""
    t = gll.tables(p)
    d = element.metric((0.02, 0.7, 2.56), 1.0)
    blk = element.ElementBlocks(p, d, t)
    assert blk.route == "separable"
    H = element.element_operator_sparse(p, d, t)
    B, I = blk.B, blk.I
    uB = np.random.default_rng(100 + p).standard_normal((len(B), 2))
    uI = -blk.interior_solve(blk.HIB @ uB)
    u = np.zeros(((p + 1) ** 3, 2))
    u[B] = uB
    u[I] = uI
    Hu = H @ u
    scale = np.abs(H).max() * np.abs(u).max()
    assert np.abs(Hu[I]).max() <= 1e-12 * scale
    SuB = blk.schur_apply(uB)
    assert np.linalg.norm(SuB - Hu[B]) <= 1e-12 * np.linalg.norm(Hu[B])
    # the interior solve itself, on a general right-hand side
    b = np.random.default_rng(200 + p).standard_normal(len(I))
    x = blk.interior_solve(b)
    assert np.linalg.norm(blk.HII @ x - b) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("p", [24])
def test_separable_route_trilinear_closed_form(p):
    """lambda = 0 at p = 24 on the separable route: the Schur complement
    reproduces the closed-form H u on B for the eight trilinear modes."""
    t = gll.tables(p)
    x, w = t["x"], t["w"]
    d = np.array([0.0, 1.7, 0.6, 2.3])
    blk = element.ElementBlocks(p, d, t)
    assert blk.route == "separable"
    B = blk.B
    kk, jj, ii = _kji(p)
    ends = lambda idx: (idx == p).astype(float) - (idx == 0).astype(float)
    for e3 in (0, 1):
        for e2 in (0, 1):
            for e1 in (0, 1):
                f1 = x[ii] if e1 else np.ones_like(x[ii])
                f2 = x[jj] if e2 else np.ones_like(x[jj])
                f3 = x[kk] if e3 else np.ones_like(x[kk])
                Hu = np.zeros(len(ii))
                if e1:
                    Hu += d[1] * w[kk] * f3 * w[jj] * f2 * ends(ii)
                if e2:
                    Hu += d[2] * w[kk] * f3 * ends(jj) * w[ii] * f1
                if e3:
                    Hu += d[3] * ends(kk) * w[jj] * f2 * w[ii] * f1
                got = blk.schur_apply((f1 * f2 * f3)[B])
                assert np.abs(got - Hu[B]).max() <= 1e-12 * max(1.0, np.abs(Hu).max())


def test_separable_schur_matrix_symmetric_p20():
    """The column-block Schur complement of the separable route is symmetric
    before symmetrisation (p = 20, lambda > 0)."""
    p = 20
    t = gll.tables(p)
    blk = element.ElementBlocks(p, element.metric((0.05, 0.3, 1.0), 2.0), t)
    nB = len(blk.B)
    cols = np.random.default_rng(5).choice(nB, 40, replace=False)
    E = np.zeros((nB, 40))
    E[cols, np.arange(40)] = 1.0
    S = blk.schur_apply(E)                 # columns cols of the Schur complement
    # entry (cols[a], cols[b]) against (cols[b], cols[a]) for the sampled pairs
    sub = S[cols]
    assert np.abs(sub - sub.T).max() <= 1e-12 * np.abs(sub).max()
