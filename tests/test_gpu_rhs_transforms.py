"""Parity of the element passes of Algorithm 4 at the degrees where their
line transforms run on the FP64 matrix cores (p = 9..16): the condensed
right-hand side (first loop), the interior recovery from a given transformed
skeleton solution (second loop) and the FP64 solve around them, against the
oracle (explicit Schur complement, Cholesky interior solves)."""

import numpy as np
import pytest

import workloads as W
from gpu_helpers import MESHES, both, rel_err

pytestmark = pytest.mark.gpu

RHS_MESHES = {
    "p9_lam_e": lambda: W.mesh(9, (2, 2, 1), widths=[[0.3, 0.7], [0.6, 0.4], [1.0]], lam=None,
                               lam_e=[0.5, 3.0, 20.0, 0.2], dirichlet=0b010101),
    "p12_stretched": lambda: W.mesh(12, (2, 1, 2), widths=[[0.05, 0.95], [0.5], [0.8, 0.2]], lam=1.0,
                                    dirichlet=0b100010),
    "p13_partial": lambda: W.mesh(13, (1, 2, 1), lam=0.4, dirichlet=0b001100),
    "p16_cube_limit": MESHES["p16_cube_limit"],
}


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


# right-hand sides per workgroup: timed (None), per-item kernels (-1), batches
BATCHES = [None, -1, 1, 2]


@pytest.mark.parametrize("batch", BATCHES)
@pytest.mark.parametrize("name", list(RHS_MESHES))
def test_condensed_rhs_matrix_cores(lib, name, batch):
    print("case", name, batch, flush=True)
    ctx, op, g, free = both(RHS_MESHES[name]())
    if batch is not None:
        ctx.set_rhs_batch(batch)
    f = W.random_skeleton_input(op.sizes["N"], k=3, seed=61)
    ref = op.condensed_rhs(f.T)
    fhat = ctx.transform(ctx.condense_rhs(_t(f)), lib.DUAL_TO_PHYSICAL).cpu().numpy()
    for r in range(3):
        assert rel_err(fhat[free, r], ref[g[free], r]) <= 1e-12, (name, r)
    assert np.all(fhat[~free] == 0.0)
    ctx.close()


@pytest.mark.parametrize("batch", BATCHES)
@pytest.mark.parametrize("name", list(RHS_MESHES))
def test_recover_interior_matrix_cores(lib, name, batch):
    """Given skeleton values (physical basis, free nodes), the interior the
    library recovers equals u_I = H_II^-1 (F_I - H_IB u_B) of the oracle."""
    print("case", name, batch, flush=True)
    ctx, op, g, free = both(RHS_MESHES[name]())
    if batch is not None:
        ctx.set_rhs_batch(batch)
    f = W.random_skeleton_input(op.sizes["N"], k=2, seed=62)
    us = W.random_skeleton_input(op.sizes["N"], k=2, seed=63)
    phys = us[:, g].T.copy()
    phys[~free] = 0.0
    ut = ctx.transform(_t(phys), lib.COEF_TO_TRANSFORMED)
    u = ctx.recover_interior(_t(f), ut).cpu().numpy()
    for r in range(2):
        unodal = np.zeros(op.sizes["N"])
        unodal[g] = phys[:, r]
        ref = op.recover_interior(f[r], unodal)
        e = np.abs(u[r] - ref).max() / np.abs(ref).max()
        assert e <= 1e-12, (name, r, e)
    ctx.close()


@pytest.mark.parametrize("name", ["p9_lam_e", "p12_stretched"])
def test_solve_fp64_matrix_cores(lib, name):
    print("case", name, flush=True)
    ctx, op, g, free = both(RHS_MESHES[name]())
    f = W.random_skeleton_input(op.sizes["N"], k=2, seed=64)
    u, info = ctx.solve(_t(f), tol=1e-13)
    u = u.cpu().numpy()
    for r in range(2):
        ref = op.recover_interior(f[r], op.solve_condensed(f[r]))
        assert info[r]["status"] == 0
        assert np.abs(u[r] - ref).max() <= 1e-10 * np.abs(ref).max(), (name, r, info[r])
    ctx.close()


@pytest.mark.parametrize("p", [9, 12, 13])
def test_rhs_batches_agree(lib, p):
    """The batched kernels give the same recovery for every R (bitwise) and,
    in deterministic mode, the same condensation (bitwise); the per-item
    kernels agree to rounding.  Seven right-hand sides: batches of 1, 3 (a
    ragged last batch), 7 and 16 (capped at k)."""
    import torch
    from paper_1601_08179_amd import semcond
    print("case p", p, flush=True)
    ctx = semcond.Context(W.mesh(p, (3, 2, 2), widths=[W.geometric_widths(3, 6), [0.4, 0.6], [0.7, 0.3]],
                                 lam=0.8, dirichlet=0b011001))
    k = 7
    rng = np.random.default_rng(70 + p)
    f = _t(rng.standard_normal((k, ctx.N)))
    ut = torch.as_tensor(rng.standard_normal((ctx.N_s, k)), device="cuda", dtype=torch.float64)
    rec, cond = {}, {}
    for R in (-1, 1, 3, 7, 16):
        ctx.set_rhs_batch(R)
        assert ctx.rhs_batch(k) == ((0, 0) if R < 0 else (min(R, k), min(R, k)))
        rec[R] = ctx.recover_interior(f, ut).cpu().numpy()
        ctx.set_deterministic(True)
        cond[R] = ctx.condense_rhs(f).cpu().numpy()
        ctx.set_deterministic(False)
    for R in (3, 7, 16):
        assert np.array_equal(rec[R], rec[1]), R
        assert np.array_equal(cond[R], cond[1]), R
    assert rel_err(rec[1], rec[-1]) <= 1e-13
    assert rel_err(cond[1], cond[-1]) <= 1e-13
    ctx.close()
