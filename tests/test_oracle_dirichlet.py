"""Pins of the oracle's solve with prescribed (inhomogeneous) Dirichlet values
and of the manufactured solution of the solver experiment (Sec. 8)."""

import numpy as np

import workloads as W
from oracle import gll
from oracle import mesh as M
from oracle.operators import CondensedOperator


def _coords(wm):
    return W.nodal_coordinates(wm["p"], wm["n"], wm["widths"], gll.tables(wm["p"])["x"])


def test_manufactured_laplacian_matches_finite_differences():
    rng = np.random.default_rng(0)
    X = rng.uniform(0.0, 2 * np.pi, (40, 3))
    k, h = 0.9, 1e-4
    lap = W.manufactured_laplacian(X, k)
    fd = sum((W.manufactured_u(X + h * e, k) - 2 * W.manufactured_u(X, k) + W.manufactured_u(X - h * e, k)) / h**2
             for e in np.eye(3))
    assert np.abs(lap - fd).max() <= 1e-5 * max(1.0, np.abs(lap).max())


def test_coordinates_match_oracle_nodes():
    wm = W.mesh(3, (2, 3, 2), widths=[[0.3, 0.7], W.geometric_widths(3, 4), [0.5, 0.5]])
    assert np.allclose(_coords(wm), M.node_coordinates(M.make_mesh(**wm)), atol=1e-15)


def test_harmonic_quadratic_is_reproduced():
    """lambda = 0, u = x1 x2 x3 + x1^2 - x2^2 (harmonic, in the element space): the
    discrete solution with u on the Dirichlet faces is u itself."""
    wm = W.mesh(3, (3, 2, 2), widths=[W.geometric_widths(3, 8), [0.4, 0.6], [0.7, 0.3]], lam=0.0)
    X = _coords(wm)
    u = X[:, 0] * X[:, 1] * X[:, 2] + X[:, 0] ** 2 - X[:, 1] ** 2
    op = CondensedOperator(M.make_mesh(**wm))
    sol = op.solve_full_dirichlet(np.zeros(len(X)), u)
    assert np.abs(sol - u).max() <= 1e-12 * np.abs(u).max()


def test_zero_boundary_values_give_the_homogeneous_solve():
    wm = W.mesh(4, (2, 2, 2), lam=0.6)
    op = CondensedOperator(M.make_mesh(**wm))
    f = np.random.default_rng(1).standard_normal(op.sizes["N"])
    assert np.allclose(op.solve_full_dirichlet(f, np.zeros_like(f)), op.solve_full(f), rtol=0, atol=1e-13)


def test_manufactured_solution_converges_spectrally():
    """lambda = 0 on (0, 2 pi)^3, 2^3 stretched elements, k = 0.5: the nodal error
    falls with p at an accelerating rate (spectral convergence), by more than
    500x from p = 4 to p = 10."""
    errs = []
    for p in (4, 6, 8, 10):
        wm = W.mesh(p, (2, 2, 2), widths=[W.one_sided_widths(2, 1.5, 2 * np.pi)] * 3, lam=0.0)
        X = _coords(wm)
        u = W.manufactured_u(X, 0.5)
        f = -W.manufactured_laplacian(X, 0.5)
        op = CondensedOperator(M.make_mesh(**wm))
        errs.append(np.abs(op.solve_full_dirichlet(f, u) - u).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(r > 4 for r in ratios) and ratios[0] < ratios[1] < ratios[2], errs
    assert errs[3] < errs[0] / 500, errs
