"""Deterministic assembly (fixed-order slot sums instead of atomics, the
assembly R of Sec. 3): bit-identical results between runs, agreement with
the atomic mode and with the oracle; per-right-hand-side element gradients
against the oracle's adjoint gradients."""

import numpy as np
import pytest

import workloads as W
from gpu_helpers import MESHES, both, rel_err

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


@pytest.mark.parametrize("name", ["config1", "stretched3_p2", "stretched3_p8", "lam_e_p3", "neumann_p6",
                                  "p17_planes"])
def test_deterministic_apply_bitwise_and_oracle(lib, name):
    import torch
    print("case", name, flush=True)
    ctx, op, g, free = both(MESHES[name]())
    u = W.random_skeleton_input(op.sizes["N"], k=3, seed=31)
    ut = _t(u[:, g].T)
    v_atomic = ctx.apply(ut, basis=lib.PHYSICAL).cpu().numpy()
    ctx.set_deterministic(True)
    v1 = ctx.apply(ut, basis=lib.PHYSICAL).cpu().numpy()
    v2 = ctx.apply(ut, basis=lib.PHYSICAL).cpu().numpy()
    ctx.set_deterministic(False)
    assert np.array_equal(v1, v2)
    ref = op.apply(u.T)[g]
    for r in range(3):
        assert rel_err(v1[free, r], ref[free, r]) <= 1e-12
        assert rel_err(v1[:, r], v_atomic[:, r]) <= 1e-14
        assert np.all(v1[~free, r] == 0.0)
    # transformed basis, one right-hand side (the node-major k = 1 path)
    x = torch.randn(ctx.N_s, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    ctx.set_deterministic(True)
    y1 = ctx.apply(x).cpu().numpy()
    y2 = ctx.apply(x).cpu().numpy()
    ctx.set_deterministic(False)
    assert np.array_equal(y1, y2)
    assert rel_err(y1, ctx.apply(x).cpu().numpy()) <= 1e-14


@pytest.mark.parametrize("name", ["config1", "stretched3_p5", "p17_planes"])
def test_deterministic_condensed_rhs(lib, name):
    print("case", name, flush=True)
    ctx, op, g, free = both(MESHES[name]())
    f = W.random_skeleton_input(op.sizes["N"], k=2, seed=32)
    ctx.set_deterministic(True)
    a = ctx.condense_rhs(_t(f))
    b = ctx.condense_rhs(_t(f))
    ctx.set_deterministic(False)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    c = ctx.condense_rhs(_t(f))
    assert rel_err(a.cpu().numpy(), c.cpu().numpy()) <= 1e-14
    # to the physical basis (dual transform) and against the oracle
    phys = ctx.transform(a, lib.DUAL_TO_PHYSICAL).cpu().numpy()
    ref = op.condensed_rhs(f.T)[g]
    for r in range(2):
        assert rel_err(phys[free, r], ref[free, r]) <= 1e-12


@pytest.mark.parametrize("precision", ["PREC_F64", "PREC_MIXED_IR"])
@pytest.mark.parametrize("name", ["config1", "stretched3_p8", "lam_e_p3"])
def test_deterministic_solve_bitwise(lib, name, precision):
    """Two deterministic solves return the same bits (solution, iterations,
    residual) and agree with the atomic-mode solve and the direct solve."""
    print("case", name, precision, flush=True)
    ctx, op, g, free = both(MESHES[name]())
    f = W.random_skeleton_input(op.sizes["N"], k=3, seed=33)
    prec = getattr(lib, precision)
    u1, i1 = ctx.solve(_t(f), tol=1e-12, precision=prec, deterministic=True)
    u2, i2 = ctx.solve(_t(f), tol=1e-12, precision=prec, deterministic=True)
    ua, ia = ctx.solve(_t(f), tol=1e-12, precision=prec)
    u1, u2, ua = u1.cpu().numpy(), u2.cpu().numpy(), ua.cpu().numpy()
    assert np.array_equal(u1, u2)
    assert i1 == i2
    ref = np.stack([op.recover_interior(f[r], op.solve_condensed(f[r])) for r in range(3)])
    for r in range(3):
        assert i1[r]["status"] == 0
        assert np.abs(u1[r] - ref[r]).max() <= 1e-10 * np.abs(ref[r]).max()
        assert np.abs(u1[r] - ua[r]).max() <= 1e-10 * np.abs(ua[r]).max()


def test_deterministic_persistent_request_runs_stepwise(lib):
    """The persistent kernel scatters with atomics; a deterministic solve that
    asks for it runs one launch per step and still returns the same bits."""
    ctx, op, g, free = both(MESHES["config1"]())
    f = W.random_skeleton_input(op.sizes["N"], k=2, seed=34)
    u1, i1 = ctx.solve(_t(f), tol=1e-12, deterministic=True, persistent=True)
    u2, i2 = ctx.solve(_t(f), tol=1e-12, deterministic=True, persistent=False)
    assert np.array_equal(u1.cpu().numpy(), u2.cpu().numpy()) and i1 == i2


def test_precond_diag_bitwise_between_contexts(lib):
    a = both(MESHES["stretched3_p8"]())[0].precond_diag().cpu().numpy()
    b = both(MESHES["stretched3_p8"]())[0].precond_diag().cpu().numpy()
    assert np.array_equal(a, b)


def test_element_grads_per_rhs_match_oracle(lib):
    """grad[e][m][r] = -a_{e,r}^T A_m u_{e,r} against the oracle's adjoint
    gradients of each right-hand side's own loss, and summed over r against
    the summed entry point."""
    from oracle import grads as OG
    from oracle import mesh as M
    rng = np.random.default_rng(35)
    widths = [w / w.sum() for w in (rng.uniform(0.5, 2, 3), rng.uniform(0.5, 2, 2), rng.uniform(0.5, 2, 2))]
    lam_e = np.exp(rng.uniform(np.log(0.1), np.log(100), 12))
    wmesh = W.mesh(4, (3, 2, 2), widths=widths, lam=None, lam_e=lam_e)
    N = W.num_nodes(4, (3, 2, 2))
    k = 3
    f = rng.standard_normal((k, N))
    t = rng.standard_normal((k, N))
    om = M.make_mesh(**wmesh)
    refs = [OG.loss_and_grads(om, f[r], t[r]) for r in range(k)]
    ctx, op, g, free = both(wmesh)
    u = np.stack([ref["u"][:, 0] for ref in refs])
    a = np.stack([ref["a"][:, 0] for ref in refs])
    G = ctx.element_grads_rhs(_t(u), _t(a)).cpu().numpy()
    assert G.shape == (ctx.n_e, 4, k)
    for r in range(k):
        ref = refs[r]["g_d"]
        np.testing.assert_allclose(G[:, :, r], ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
    S = ctx.element_grads(_t(u), _t(a)).cpu().numpy()
    np.testing.assert_allclose(G.sum(axis=2), S[:, :4], rtol=1e-12, atol=1e-12 * np.abs(S).max())
