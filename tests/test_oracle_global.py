"""Pins of the oracle's assembled system: condensed = full solve, interior
recovery, manufactured-solution convergence, operator symmetry, and the
block-Jacobi PCG (the paper's BC solver) against the same PCG run in the
fast-diagonalisation basis with a diagonal preconditioner (the BT solver):
Sec. 8 states both give the same iteration count; in exact arithmetic they
give identical alpha/beta sequences."""

import math

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import gll, mesh as M
from oracle.operators import CondensedOperator


def _mesh(p, n=(2, 2, 2), widths=None, lam=1.0, lam_e=None, dirichlet=0x3F):
    return M.make_mesh(**W.mesh(p, n, widths=widths, lam=lam, lam_e=lam_e, dirichlet=dirichlet))


MESHES = {
    "uniform2": lambda p: _mesh(p),
    "stretched": lambda p: _mesh(p, (3, 2, 2), widths=[[0.2, 0.3, 0.5], [0.7, 0.3], [0.1, 0.9]],
                                 lam=0.5),
    "lam_e": lambda p: _mesh(p, (2, 2, 3), lam=None,
                             lam_e=np.array([0.1, 3.0, 7.0, 0.5, 1.0, 2.0, 9.0, 0.2, 4.0, 0.3, 5.0, 6.0])),
    "partial_dirichlet": lambda p: _mesh(p, (2, 3, 2), lam=2.0, dirichlet=0b010011),
}


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("p", [2, 3, 5])
def test_condensed_equals_full_solve(name, p):
    mesh = MESHES[name](p)
    op = CondensedOperator(mesh)
    f = np.random.default_rng(p).uniform(-1, 1, op.sizes["N"])
    u_full = op.solve_full(f)
    u_skel = op.solve_condensed(f)
    fs = op.free_skel
    np.testing.assert_allclose(u_skel[fs], u_full[fs], rtol=0, atol=1e-12 * np.abs(u_full).max())
    u_rec = op.recover_interior(f, u_skel)
    np.testing.assert_allclose(u_rec, u_full, rtol=0, atol=1e-12 * np.abs(u_full).max())


@pytest.mark.parametrize("name", list(MESHES))
def test_apply_symmetric_and_matches_assembled(name):
    mesh = MESHES[name](4)
    op = CondensedOperator(mesh)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(op.sizes["N"])
    v = rng.standard_normal(op.sizes["N"])
    Au, Av = op.apply(u), op.apply(v)
    fs = op.free_skel
    assert abs(v[fs] @ Au[fs] - u[fs] @ Av[fs]) < 1e-12 * np.abs(Au).max() * np.abs(v).sum()
    A, idx = op.assembled_condensed()
    np.testing.assert_allclose(Au[idx], A @ u[idx], atol=1e-13 * np.abs(Au).max())
    # interior and constrained entries of the input are ignored
    u2 = u.copy()
    u2[~fs] = 1e6
    np.testing.assert_array_equal(op.apply(u2), Au)


def test_manufactured_convergence():
    """u = sin(pi x) sin(pi y) sin(pi z), lambda = 1 on the unit cube, 2^3 elements:
    spectral convergence of the skeleton error (Sec. 3 discretisation)."""
    errs = {}
    for p in (2, 4, 6, 8):
        mesh = _mesh(p)
        op = CondensedOperator(mesh)
        X = M.node_coordinates(mesh)
        uex = np.prod(np.sin(math.pi * X), axis=1)
        f = (1.0 + 3 * math.pi ** 2) * uex
        u = op.solve_condensed(f)
        fs = op.free_skel
        errs[p] = np.abs(u[fs] - uex[fs]).max()
    assert errs[2] < 5e-2 and errs[4] < 1e-4 and errs[6] < 1e-6 and errs[8] < 1e-9
    assert errs[2] > errs[4] > errs[6] > errs[8]


@pytest.mark.parametrize("p", [2, 4, 6])
def test_bc_pcg_converges_to_direct(p):
    mesh = MESHES["stretched"](p)
    op = CondensedOperator(mesh)
    f = np.random.default_rng(11).uniform(-1, 1, op.sizes["N"])
    x, info = op.bc_pcg(f, tol=1e-12)
    ref = op.solve_condensed(f)
    assert info["res"][-1] <= 1e-12 * info["bnorm"]
    np.testing.assert_allclose(x, ref, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("p", [3, 5])
def test_bc_equals_bt_alpha_beta(p):
    """Block-Jacobi PCG in the physical basis and diagonal PCG in the transformed
    basis produce the same alpha_k, beta_k (Sec. 8: BC and BT need the same
    iterations)."""
    mesh = MESHES["stretched"](p)
    op = CondensedOperator(mesh)
    f = np.random.default_rng(3).uniform(-1, 1, op.sizes["N"])
    _, info = op.bc_pcg(f, fixed_iters=12)
    # transformed system built here from the assembled matrix: each entity
    # transforms with S along its interior directions
    A, fs = op.assembled_condensed()
    A = A.toarray()
    t = gll.tables(p)
    lam, S = sla.eigh(t["K"][1:p, 1:p], t["M"][1:p, 1:p])
    G = M.global_ijk(mesh)[fs]
    fs_ids, ids = op.entity_ids()
    T = np.zeros_like(A)
    for ent in range(ids.max() + 1):
        loc = np.nonzero(ids == ent)[0]
        g = G[loc]
        interior_axes = [ax for ax in range(3) if np.any(g[:, ax] % p != 0)]
        # the entity's nodes in lexicographic order (I1 fastest) are the tensor grid
        # of its interior axes; the transform is S along each of them
        Tl = np.ones((1, 1))
        for ax in interior_axes[::-1]:
            Tl = np.kron(Tl, S)
        order = np.lexsort([g[:, ax] for ax in range(3)])
        T[np.ix_(loc[order], loc[order])] = Tl
    At = T.T @ A @ T
    b = T.T @ op.condensed_rhs(f)[fs]
    Pd = np.diag(At)
    offd = At.copy()
    for ent in range(ids.max() + 1):
        loc = np.nonzero(ids == ent)[0]
        blk = At[np.ix_(loc, loc)]
        assert np.abs(blk - np.diag(np.diag(blk))).max() < 1e-11 * np.abs(At).max()
    x = np.zeros_like(b)
    r = b.copy()
    z = r / Pd
    pv = z.copy()
    rho = r @ z
    al, be = [], []
    for _ in range(12):
        q = At @ pv
        a = rho / (pv @ q)
        x += a * pv
        r -= a * q
        z = r / Pd
        rn = r @ z
        be.append(rn / rho)
        al.append(a)
        pv = z + be[-1] * pv
        rho = rn
    np.testing.assert_allclose(al, info["alpha"], rtol=1e-9)
    np.testing.assert_allclose(be, info["beta"], rtol=1e-9)
