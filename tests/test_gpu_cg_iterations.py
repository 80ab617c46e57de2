"""The GPU's BT conjugate gradients against the same iteration run on the
oracle's matrices (Sec. 8): diagonal preconditioning of the transformed
condensed operator T^T H^ T, x0 = 0, stop at ||r~|| <= tol ||F~|| in the
transformed basis.  The oracle side takes the explicit condensed matrix and the
block transform built from scipy's generalized eigensolver; the iteration
counts must agree (one iteration of slack for a residual that lands on the
threshold), and the GPU's reported relative residual must match the oracle's
at that iteration."""

import numpy as np
import pytest

import workloads as W
from gpu_helpers import MESHES, both, oracle_transform

pytestmark = pytest.mark.gpu


def _oracle_bt(At, bt, tol, maxit=5000):
    d = np.diag(At).copy()
    x = np.zeros_like(bt)
    r = bt.copy()
    z = r / d
    p = z.copy()
    rho = r @ z
    bn = np.linalg.norm(bt)
    res = [np.linalg.norm(r) / bn]
    it = 0
    while res[-1] > tol and it < maxit:
        q = At @ p
        alpha = rho / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = r / d
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
        res.append(np.linalg.norm(r) / bn)
        it += 1
    return it, np.array(res)


@pytest.mark.parametrize("tol", [1e-6, 1e-10])
@pytest.mark.parametrize("name", ["stretched3_p5", "stretched3_p8", "lam_e_p3", "partial_dirichlet_p4"])
def test_cg_iterations_match_oracle(lib, name, tol):
    import torch
    print("case", name, tol, flush=True)
    ctx, op, g, free = both(MESHES[name]())
    f = W.random_skeleton_input(op.sizes["N"], k=1, seed=91)[0]
    A, fs, T = oracle_transform(op)
    b = op.condensed_rhs(f)[fs]
    it_o, res_o = _oracle_bt(T.T @ A @ T, T.T @ b, tol)
    _, info = ctx.solve(torch.as_tensor(f, device="cuda"), tol=tol, check_every=1)
    it_g = info[0]["iters"]
    print("iterations gpu", it_g, "oracle", it_o)
    assert abs(it_g - it_o) <= 1, (it_g, it_o)
    if it_g == it_o:
        assert abs(info[0]["rel_res"] - res_o[it_o]) <= 1e-6 * tol + 1e-3 * res_o[it_o]
    ctx.close()


def test_fused_loop_polls_every_iteration_after_another_context(lib):
    """The fused CG loop's pinned convergence flags start as "active" in every
    loop: a context created after another one was closed (whose pinned flag
    buffer the runtime may hand out again) and polled after every iteration
    converges with the same iteration count as the first context."""
    import torch
    from paper_1601_08179_amd import semcond
    wm = MESHES["stretched3_p5"]()
    f = None
    its = []
    for _ in range(3):
        ctx = semcond.Context(wm)
        if f is None:
            f = torch.as_tensor(W.random_skeleton_input(ctx.N, k=1, seed=92)[0], device="cuda")
        _, info = ctx.solve(f, tol=1e-10, check_every=1)
        assert info[0]["status"] == 0 and info[0]["rel_res"] <= 1e-10, info
        its.append(info[0]["iters"])
        ctx.close()
    assert len(set(its)) == 1, its


def _oracle_bt_iterate(At, bt, n):
    """x after n iterations of the same diagonally preconditioned CG (x0 = 0)."""
    d = np.diag(At).copy()
    x = np.zeros_like(bt)
    r = bt.copy()
    z = r / d
    p = z.copy()
    rho = r @ z
    for _ in range(n):
        q = At @ p
        alpha = rho / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = r / d
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x


@pytest.mark.parametrize("det", [True, False])
@pytest.mark.parametrize("n", [1, 2, 5, 6])
def test_stepwise_iterate_after_n_steps(lib, n, det):
    """Both one-launch-per-step loops (deterministic mode takes the one with
    separate reductions; this small mesh otherwise runs the fused loop) update
    x at every other step and add a pending update at the end of the solve:
    after n = 1, 2, 5, 6 iterations (odd and even counts) each of three RHS
    holds the oracle CG's n-th iterate."""
    import torch
    print("case n", n, "deterministic", det, flush=True)
    ctx, op, g, free = both(MESHES["stretched3_p5"]())
    A, fs, T = oracle_transform(op)
    f = W.random_skeleton_input(op.sizes["N"], k=3, seed=93)
    skel = torch.zeros((ctx.N_s, 3), dtype=torch.float64, device="cuda")
    _, info = ctx.solve(torch.as_tensor(f, device="cuda"), tol=1e-14, max_iter=n, skel_out=skel,
                        raise_on_notconv=False, deterministic=det, persistent=False)
    phys = ctx.transform(skel, lib.COEF_TO_PHYSICAL).cpu().numpy()
    pos = {int(v): i for i, v in enumerate(fs)}
    rows = np.array([pos[int(v)] for v in g[free]])
    for r in range(3):
        assert info[r]["iters"] == n, info[r]
        b = op.condensed_rhs(f[r])[fs]
        x = T @ _oracle_bt_iterate(T.T @ A @ T, T.T @ b, n)
        got = phys[free, r]
        assert np.linalg.norm(got - x[rows]) <= 1e-11 * np.linalg.norm(x), (r, n)
    ctx.close()
