"""Two-level preconditioner (solve option coarse): the BT diagonal of Sec. 8
plus a coarse correction on the trilinear functions of the element mesh.
The solutions equal the oracle's direct solve, in FP64 and mixed precision;
the iteration counts fall below the BT ones and stop growing with the
element count."""

import numpy as np
import pytest

import workloads as W
from gpu_helpers import MESHES, both

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


def _direct(op, f):
    return np.stack([op.recover_interior(f[r], op.solve_condensed(f[r])) for r in range(f.shape[0])])


@pytest.mark.parametrize("precision", ["PREC_F64", "PREC_MIXED_IR"])
@pytest.mark.parametrize("name", ["config1", "stretched3_p2", "stretched3_p5", "lam_e_p3", "partial_dirichlet_p4",
                                  "neumann_p6", "stretched3_p8", "p16_cube_limit", "p17_planes"])
def test_coarse_solve_matches_direct(lib, name, precision):
    print("case", name, precision, flush=True)
    ctx, op, g, free = both(MESHES[name]())
    f = W.random_skeleton_input(op.sizes["N"], k=2, seed=121)
    u, info = ctx.solve(_t(f), tol=1e-13 if precision == "PREC_F64" else 1e-12,
                        precision=getattr(lib, precision), coarse=True)
    ref = _direct(op, f)
    u = u.cpu().numpy()
    for r in range(2):
        assert info[r]["status"] == 0, info[r]
        e = np.abs(u[r] - ref[r]).max() / np.abs(ref[r]).max()
        assert e <= 1e-10, (name, precision, r, e, info[r])
    ctx.close()


def test_coarse_iterations_do_not_grow_with_elements(lib):
    """p = 4, n^3 elements for n = 4, 6, 8: BT iterations grow with n, the
    two-level ones stay within 20 % of the n = 4 count and below 60 % of BT."""
    its_bt, its_2l = [], []
    for n in (4, 6, 8):
        wm = W.mesh(4, (n, n, n), lam=1.0)
        ctx = lib.Context(wm)
        f = W.random_skeleton_input(ctx.N, k=1, seed=122)
        _, i1 = ctx.solve(_t(f), tol=1e-10)
        _, i2 = ctx.solve(_t(f), tol=1e-10, coarse=True)
        its_bt.append(i1[0]["iters"])
        its_2l.append(i2[0]["iters"])
        ctx.close()
    print("BT", its_bt, "two-level", its_2l, flush=True)
    assert its_bt[2] > 1.4 * its_bt[0]
    assert max(its_2l) <= 1.2 * its_2l[0]
    assert its_2l[2] <= 0.6 * its_bt[2]


def test_coarse_after_coefficient_update(lib):
    """The coarse matrix follows a change of lambda_e (it is rebuilt)."""
    print("case coefficient update", flush=True)
    wm = MESHES["lam_e_p3"]()
    ctx, op, g, free = both(wm)
    f = W.random_skeleton_input(op.sizes["N"], k=1, seed=123)
    ctx.solve(_t(f), tol=1e-12, coarse=True)
    lam2 = np.exp(np.random.default_rng(9).uniform(np.log(0.1), np.log(100), op.sizes["n_e"]))
    ctx.update_coefficients(lam_e=lam2)
    u, info = ctx.solve(_t(f), tol=1e-13, coarse=True)
    wm2 = dict(wm)
    wm2["lam_e"] = lam2
    ctx2, op2, _, _ = both(wm2)
    ref = _direct(op2, f)
    assert np.abs(u.cpu().numpy()[0] - ref[0]).max() <= 1e-10 * np.abs(ref[0]).max()
    ctx.close()
    ctx2.close()
