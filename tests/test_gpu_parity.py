"""GPU parity of the HIP path against the FP64 CPU oracle, through the C ABI.

Tolerances: the FP64 apply matches the oracle's explicit Schur complement to
1e-12 relative (2-norm over free skeleton nodes); the solve's forward error vs
the oracle's direct solve is <= 1e-10 when run to a 1e-13 residual.
"""

import numpy as np
import pytest

import workloads as W
from gpu_helpers import MESHES, both, check_layout, oracle_transform, rel_err

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype or torch.float64)


@pytest.mark.parametrize("name", list(MESHES))
def test_layout_bijection(lib, name):
    ctx, op, g, free = both(MESHES[name]())
    check_layout(op, g, free)
    assert ctx.N == op.sizes["N"]
    assert ctx.N_free == int(op.free_skel.sum())


@pytest.mark.parametrize("name", list(MESHES))
def test_apply_physical_fp64(lib, name):
    print("case", name, flush=True)
    ctx, op, g, free = both(MESHES[name]())
    u = W.random_skeleton_input(op.sizes["N"], k=2, seed=1)      # (2, N)
    ref = op.apply(u.T)                                            # (N, 2)
    us = _t(u.T[g])                                                # (N_s, 2)
    v = lib.PHYSICAL
    out = ctx.apply(us, basis=v).cpu().numpy()
    for r in range(2):
        e = rel_err(out[free, r], ref[g[free], r])
        assert e <= 1e-12, (name, r, e)
        # entry by entry too: no single face, edge or vertex row may be off
        m = np.max(np.abs(out[free, r] - ref[g[free], r])) / np.max(np.abs(ref[g[free], r]))
        assert m <= 1e-12, (name, r, m)
    assert np.all(out[~free] == 0.0)


@pytest.mark.parametrize("name", ["config1", "stretched3_p5", "stretched3_p8", "lam_e_p8_classes", "p17_planes"])
def test_apply_fp32_reported(lib, name):
    """FP32 operator vs FP64 oracle: reported, loosely bounded."""
    import torch
    ctx, op, g, free = both(MESHES[name]())
    u = W.random_skeleton_input(op.sizes["N"], k=1, seed=2)[0]
    ref = op.apply(u)
    out = ctx.apply(_t(u[g], torch.float32), basis=lib.PHYSICAL).double().cpu().numpy()
    e = rel_err(out[free], ref[g[free]])
    print("fp32 apply rel err", name, e)
    assert e < 1e-5


@pytest.mark.parametrize("name", ["config1", "stretched3_p5", "neumann_p6"])
def test_transforms_inverse_and_dual(lib, name):
    ctx, op, g, free = both(MESHES[name]())
    rng = np.random.default_rng(4)
    u = _t(rng.standard_normal((ctx.N_s, 3)))
    r = _t(rng.standard_normal((ctx.N_s, 3)))
    ut = ctx.transform(u, lib.COEF_TO_TRANSFORMED)
    back = ctx.transform(ut, lib.COEF_TO_PHYSICAL)
    assert rel_err(back.cpu().numpy(), u.cpu().numpy()) < 1e-13
    rt = ctx.transform(r, lib.DUAL_TO_TRANSFORMED)
    rb = ctx.transform(rt, lib.DUAL_TO_PHYSICAL)
    assert rel_err(rb.cpu().numpy(), r.cpu().numpy()) < 1e-13
    # duality: (T^-1 u) . (T^T r) = u . r
    lhs = (ut * rt).sum(0).cpu().numpy()
    rhs = (u * r).sum(0).cpu().numpy()
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


@pytest.mark.parametrize("name", ["config1", "stretched3_p2", "stretched3_p5", "lam_e_p3", "partial_dirichlet_p4",
                                  "neumann_p6"])
def test_precond_diag_matches_transformed_oracle(lib, name):
    """diag(T^T H^ T), with T built from the oracle's assembled matrix and its own
    eigenvectors (diagonal entries do not depend on eigenvector signs), against
    the library's preconditioner diagonal."""
    ctx, op, g, free = both(MESHES[name]())
    A, fs, T = oracle_transform(op)
    ref = np.einsum("ij,ij->j", T, A @ T)
    pos = np.searchsorted(fs, g[free])
    diag = ctx.precond_diag().cpu().numpy()
    assert np.all(diag[~free] == 0.0)
    assert np.abs(diag[free] - ref[pos]).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["config1", "stretched3_p5", "lam_e_p3", "partial_dirichlet_p4", "p17_planes"])
def test_condensed_rhs(lib, name):
    ctx, op, g, free = both(MESHES[name]())
    f = W.random_skeleton_input(op.sizes["N"], k=2, seed=5)       # nodal (2, N)
    ref = op.condensed_rhs(f.T)                                     # physical (N, 2)
    fhat_t = ctx.condense_rhs(_t(f))                                # transformed (N_s, 2)
    fhat = ctx.transform(fhat_t, lib.DUAL_TO_PHYSICAL).cpu().numpy()
    for r in range(2):
        assert rel_err(fhat[free, r], ref[g[free], r]) <= 1e-12
    assert np.all(fhat[~free] == 0.0)


@pytest.mark.parametrize("name", ["config1", "stretched3_p2", "stretched3_p5", "lam_e_p3", "partial_dirichlet_p4",
                                  "neumann_p6", "p17_planes"])
def test_solve_fp64_matches_direct(lib, name):
    print("case", name, flush=True)
    ctx, op, g, free = both(MESHES[name]())
    f = W.random_skeleton_input(op.sizes["N"], k=2, seed=6)
    u, info = ctx.solve(_t(f), tol=1e-13)
    u = u.cpu().numpy()
    for r in range(2):
        ref = op.recover_interior(f[r], op.solve_condensed(f[r]))
        assert info[r]["status"] == 0 and info[r]["rel_res"] <= 1e-13
        e = np.abs(u[r] - ref).max() / np.abs(ref).max()
        assert e <= 1e-10, (name, r, e, info[r])


def test_manufactured_solution(lib):
    """u = sin(pi x) sin(pi y) sin(pi z), lambda = 1, config-1 mesh: the GPU
    solution equals the oracle's direct solve and shows the discretisation error
    of degree 4."""
    import math
    from oracle import mesh as M
    wm = W.config1()[0]
    ctx, op, g, free = both(wm)
    X = M.node_coordinates(op.mesh)
    uex = np.prod(np.sin(math.pi * X), axis=1)
    f = (1 + 3 * math.pi ** 2) * uex
    u, info = ctx.solve(_t(f), tol=1e-13)
    u = u.cpu().numpy()
    ref = op.recover_interior(f, op.solve_condensed(f))
    assert np.abs(u - ref).max() <= 1e-10 * np.abs(ref).max()
    err = np.abs(u - uex).max()
    assert 1e-6 < err < 1e-4


@pytest.mark.parametrize("basis", ["PHYSICAL", "TRANSFORMED"])
@pytest.mark.parametrize("dtype", ["float64", "float32"])
def test_apply_batched_equals_single_columns(lib, basis, dtype):
    """k = 5 right-hand sides in one call (RHS-major kernels behind the [N_s][k]
    interface) equal five single-RHS applies, up to the scatter's rounding order."""
    import torch
    ctx, op, g, free = both(MESHES["stretched3_p5"]())
    dt = getattr(torch, dtype)
    u = torch.as_tensor(np.random.default_rng(8).standard_normal((ctx.N_s, 5)), device="cuda").to(dt)
    b = getattr(lib, basis)
    out = ctx.apply(u, basis=b).double().cpu().numpy()
    tol = 1e-13 if dtype == "float64" else 1e-5
    for r in range(5):
        one = ctx.apply(u[:, r].contiguous(), basis=b).double().cpu().numpy()
        assert np.abs(out[:, r] - one).max() <= tol * np.abs(one).max(), (basis, dtype, r)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_dinv_table_matches_recompute(lib, dtype):
    """The cube apply reads D^-1 from per-class tables when the mesh has few
    metric classes and recomputes it otherwise: the same operator once with one
    class per element width pair (25) and once with 75 classes (lambda_e = 1 + e
    ulp, equal to 1 within 75 units in the last place) gives the same result to
    rounding."""
    import torch
    from paper_1601_08179_amd import semcond
    p, n = 10, (5, 5, 3)
    ne = n[0] * n[1] * n[2]
    widths = [W.geometric_widths(n[0], 8), W.geometric_widths(n[1], 3), W.uniform_widths(n[2])]
    one = semcond.Context(W.mesh(p, n, widths=widths, lam=1.0, dirichlet=0b010101))
    many = semcond.Context(W.mesh(p, n, widths=widths, lam=None,
                                  lam_e=1.0 + np.arange(ne) * np.finfo(float).eps, dirichlet=0b010101))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    u = torch.as_tensor(np.random.default_rng(5).standard_normal((one.N_s, 3)), device="cuda", dtype=tdt)
    a = one.apply(u).double().cpu().numpy()
    b = many.apply(u).double().cpu().numpy()
    tol = 1e-13 if dtype == "f64" else 2e-6
    assert rel_err(a, b) <= tol, rel_err(a, b)
