"""Prescribed (inhomogeneous) Dirichlet values through the C ABI against the
oracle's full direct solve with the known values eliminated: all nodes
(skeleton and recovered interiors) <= 1e-10 relative, for FP64, k > 1 (the
RHS-major CG), partial Dirichlet masks and mixed precision; harmonic
polynomials are reproduced; the initial guess's Dirichlet entries are ignored."""

import numpy as np
import pytest

import workloads as W
from oracle import gll
from oracle import mesh as M
from oracle.operators import CondensedOperator

pytestmark = pytest.mark.gpu


def _coords(wm):
    return W.nodal_coordinates(wm["p"], wm["n"], wm["widths"], gll.tables(wm["p"])["x"])


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


MESHES = {
    "stretched_p4_lam05": W.mesh(4, (3, 2, 2), widths=[W.geometric_widths(3, 8), [0.4, 0.6], [0.7, 0.3]], lam=0.5),
    "stretched_p5_lam0": W.mesh(5, (2, 3, 2), widths=[[0.3, 0.7], W.geometric_widths(3, 16), [0.5, 0.5]], lam=0.0),
    "partial_mask_p3": W.mesh(3, (2, 2, 3), lam=0.2, dirichlet=0b011001),
    "p16_one_element": W.mesh(16, (1, 1, 2), widths=[[1.0], [1.0], [0.3, 0.7]], lam=0.0),
}


@pytest.mark.parametrize("name", list(MESHES))
@pytest.mark.parametrize("k", [1, 3])
def test_prescribed_values_match_oracle(lib, name, k):
    print("case", name, k, flush=True)
    wm = MESHES[name]
    ctx = lib.Context(wm)
    op = CondensedOperator(M.make_mesh(**wm))
    rng = np.random.default_rng(60 + k)
    f = rng.standard_normal((k, op.sizes["N"]))
    g = rng.standard_normal((k, op.sizes["N"]))
    u, info = ctx.solve(_t(f), tol=1e-13, g=_t(g))
    u = u.cpu().numpy()
    for r in range(k):
        ref = op.solve_full_dirichlet(f[r], g[r])
        assert info[r]["status"] == 0
        assert np.abs(u[r] - ref).max() <= 1e-10 * np.abs(ref).max(), (name, r)
    ctx.close()


def test_mixed_precision_with_prescribed_values(lib):
    wm = MESHES["stretched_p4_lam05"]
    ctx = lib.Context(wm)
    op = CondensedOperator(M.make_mesh(**wm))
    rng = np.random.default_rng(70)
    f, g = rng.standard_normal(op.sizes["N"]), rng.standard_normal(op.sizes["N"])
    u, info = ctx.solve(_t(f), tol=1e-13, g=_t(g), precision=lib.PREC_MIXED_IR, inner_tol=1e-5)
    ref = op.solve_full_dirichlet(f, g)
    assert np.abs(u.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()


def test_harmonic_quadratic_reproduced(lib):
    wm = MESHES["stretched_p5_lam0"]
    X = _coords(wm)
    uex = X[:, 0] * X[:, 1] * X[:, 2] + X[:, 0] ** 2 - X[:, 1] ** 2
    ctx = lib.Context(wm)
    u, _ = ctx.solve(_t(np.zeros_like(uex)), tol=1e-14, g=_t(uex))
    assert np.abs(u.cpu().numpy() - uex).max() <= 1e-11 * np.abs(uex).max()


def test_initial_guess_dirichlet_entries_ignored(lib):
    import torch
    wm = MESHES["partial_mask_p3"]
    ctx = lib.Context(wm)
    op = CondensedOperator(M.make_mesh(**wm))
    rng = np.random.default_rng(71)
    f, g = rng.standard_normal(op.sizes["N"]), rng.standard_normal(op.sizes["N"])
    x0 = torch.as_tensor(rng.standard_normal(ctx.N_s), device="cuda")   # garbage everywhere
    u, info = ctx.solve(_t(f), tol=1e-13, g=_t(g), x0=x0)
    ref = op.solve_full_dirichlet(f, g)
    assert np.abs(u.cpu().numpy() - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("p,paper_iters", [(8, 166), (16, 196)])
def test_solver_experiment_iteration_counts(lib, p, paper_iters):
    """Sec. 8's solver test with expansion factor 2 (aspect ratio 128): the BT
    iteration count to a 1e-12 residual reduction matches the count implied by
    the paper's iteration-times table (Sec. 8: solution time per DOF / iteration
    time per DOF) within 3."""
    import torch
    wm = W.solver_experiment_mesh(p, 2.0)
    X = _coords(wm)
    ctx = lib.Context(wm)
    f = torch.as_tensor(-W.manufactured_laplacian(X, 5.0), device="cuda")
    g = torch.as_tensor(W.manufactured_u(X, 5.0), device="cuda")
    _, info = ctx.solve(f, tol=1e-12, g=g)
    print("iterations", p, info[0]["iters"], "paper", paper_iters)
    assert abs(info[0]["iters"] - paper_iters) <= 3


def test_solver_experiment_uniform_mesh_converges(lib):
    """Expansion factor 1: the error against the exact solution at p = 24 is below 1e-6."""
    import torch
    wm = W.solver_experiment_mesh(24, 1.0)
    X = _coords(wm)
    uex = W.manufactured_u(X, 5.0)
    ctx = lib.Context(wm)
    u, _ = ctx.solve(torch.as_tensor(-W.manufactured_laplacian(X, 5.0), device="cuda"), tol=1e-12,
                     g=torch.as_tensor(uex, device="cuda"))
    assert np.abs(u.cpu().numpy() - uex).max() <= 1e-6 * np.abs(uex).max()


@pytest.mark.parametrize("p", [17, 24, 32])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_harmonic_quadratics_high_order(lib, p, precision):
    """The k-plane element path (n_I >= 16, every line-sum split it uses):
    two harmonic quadratics prescribed on the boundary of a stretched 2x1x2 mesh
    come back at every node to rounding, in FP64 and with the FP32 inner solve of
    the mixed iterative refinement.  Exact at any p (the GLL quadrature
    integrates the stiffness of a quadratic exactly), so it needs no oracle."""
    print("case", p, precision, flush=True)
    wm = W.mesh(p, (2, 1, 2), widths=[[0.3, 0.7], [1.0], [0.6, 0.4]], lam=0.0)
    X = _coords(wm)
    u1 = X[:, 0] * X[:, 1] * X[:, 2] + X[:, 0] ** 2 - X[:, 1] ** 2
    u2 = 2.0 * X[:, 2] ** 2 - X[:, 0] ** 2 - X[:, 1] ** 2 + 3.0 * X[:, 1] + 1.0
    uex = np.stack([u1, u2])
    ctx = lib.Context(wm)
    kw = dict(precision=lib.PREC_MIXED_IR, inner_tol=1e-5) if precision == "mixed" else {}
    u, info = ctx.solve(_t(np.zeros_like(uex)), tol=1e-13, g=_t(uex), **kw)
    err = np.abs(u.cpu().numpy() - uex).max() / np.abs(uex).max()
    print("p", p, precision, "iters", [i["iters"] for i in info], "max rel err", err, flush=True)
    assert err <= 1e-10
    ctx.close()
