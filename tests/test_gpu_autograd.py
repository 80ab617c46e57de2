"""Autograd of the GPU solve (adjoint backward): gradients with respect to the
nodal right-hand side f, the per-element lambda_e and the metric coefficients
d_{e,1..3}, for L = 1/2 sum_k ||u_k - t_k||^2 over free skeleton nodes.

* against the oracle's adjoint gradients (direct solves) on a small stretched
  mesh: <= 1e-9 relative;
* against central finite differences of the GPU forward (h = 1e-6 relative, FP64
  solves to 1e-14) on the full 8^3, p = 8, k = 8 configuration, as directional
  derivatives along seeded random directions.
"""

import numpy as np
import pytest

import workloads as W
from gpu_helpers import both

pytestmark = pytest.mark.gpu


def _setup(wmesh, f, t):
    import torch
    from paper_1601_08179_amd import semcond
    ctx = semcond.Context(wmesh)
    g, free = ctx.skeleton_nodal_index()
    idx = torch.as_tensor(g[free], device="cuda")
    ft = torch.as_tensor(f, device="cuda").clone().requires_grad_(True)
    tt = torch.as_tensor(t, device="cuda")
    return ctx, idx, ft, tt


def _metric(wmesh):
    from oracle import mesh as M
    om = M.make_mesh(**wmesh)
    return M.element_metrics(om), M.element_jacobians(om)


def _loss(u, t, idx):
    d = u[:, idx] - t[:, idx]
    return 0.5 * (d * d).sum()


def test_grads_match_oracle_adjoint(lib):
    import torch
    from oracle import grads as OG
    from oracle import mesh as M
    from paper_1601_08179_amd import autograd
    rng = np.random.default_rng(21)
    widths = [w / w.sum() for w in (rng.uniform(0.5, 2, 3), rng.uniform(0.5, 2, 2), rng.uniform(0.5, 2, 2))]
    lam_e = np.exp(rng.uniform(np.log(0.1), np.log(100), 12))
    wmesh = W.mesh(4, (3, 2, 2), widths=widths, lam=None, lam_e=lam_e)
    N = W.num_nodes(4, (3, 2, 2))
    f = rng.standard_normal((2, N))
    t = rng.standard_normal((2, N))
    d, J = _metric(wmesh)
    ctx, idx, ft, tt = _setup(wmesh, f, t)
    lam_t = torch.tensor(lam_e, device="cuda", requires_grad=True)
    dm_t = torch.tensor(d[:, 1:], device="cuda", requires_grad=True)
    u = autograd.solve(ctx, ft, lam_t, dm_t, tol=1e-14)
    loss = _loss(u, tt, idx)
    loss.backward()
    om = M.make_mesh(**dict(wmesh, dcoef=d))
    ref = OG.loss_and_grads(om, f.T, t.T)
    assert abs(loss.item() - ref["loss"]) <= 1e-10 * abs(ref["loss"])
    gl = lam_t.grad.cpu().numpy()
    gd = dm_t.grad.cpu().numpy()
    gf = ft.grad.cpu().numpy()
    np.testing.assert_allclose(gl, ref["g_lam"], rtol=1e-9, atol=1e-9 * np.abs(ref["g_lam"]).max())
    np.testing.assert_allclose(gd, ref["g_d"][:, 1:], rtol=1e-9, atol=1e-9 * np.abs(ref["g_d"]).max())
    np.testing.assert_allclose(gf, ref["g_f"].T, rtol=1e-9, atol=1e-9 * np.abs(ref["g_f"]).max())


def test_grads_vs_central_fd_config5(lib):
    import torch
    from paper_1601_08179_amd import autograd
    wmesh, f, t = W.config5()
    d, J = _metric(wmesh)
    lam_e = wmesh["lam_e"]
    ctx, idx, ft, tt = _setup(wmesh, f, t)
    lam_t = torch.tensor(lam_e, device="cuda", requires_grad=True)
    dm_t = torch.tensor(d[:, 1:], device="cuda", requires_grad=True)
    tol = 1e-14
    u = autograd.solve(ctx, ft, lam_t, dm_t, tol=tol)
    loss = _loss(u, tt, idx)
    loss.backward()
    L0 = loss.item()

    def L(fv, lv, dv):
        with torch.no_grad():
            uu = autograd.solve(ctx, fv, lv, dv, tol=tol)
            return _loss(uu, tt, idx).item()

    rng = np.random.default_rng(55)
    h = 1e-6
    f0 = ft.detach()
    l0 = lam_t.detach()
    d0 = dm_t.detach()
    checks = []
    # relative steps along random directions for lambda_e and d, absolute for f
    vl = torch.tensor(rng.standard_normal(l0.shape), device="cuda") * l0
    vd = torch.tensor(rng.standard_normal(d0.shape), device="cuda") * d0
    vf = torch.tensor(rng.standard_normal(f0.shape), device="cuda")
    checks.append(((L(f0, l0 + h * vl, d0) - L(f0, l0 - h * vl, d0)) / (2 * h), float((lam_t.grad * vl).sum())))
    checks.append(((L(f0, l0, d0 + h * vd) - L(f0, l0, d0 - h * vd)) / (2 * h), float((dm_t.grad * vd).sum())))
    checks.append(((L(f0 + h * vf, l0, d0) - L(f0 - h * vf, l0, d0)) / (2 * h), float((ft.grad * vf).sum())))
    noise = 100 * (np.finfo(float).eps + tol) * abs(L0) / h
    for fd, ad in checks:
        print("directional FD %.12e autograd %.12e noise %.2e" % (fd, ad, noise))
        assert abs(fd - ad) <= 1e-6 * abs(ad) + noise


def test_host_coefficient_inputs_get_host_gradients(lib):
    """lambda_e and d_{e,1..3} given as host tensors: their gradients come back
    on the host and equal those of device inputs."""
    import torch
    from paper_1601_08179_amd import autograd
    rng = np.random.default_rng(22)
    lam_e = np.exp(rng.uniform(np.log(0.1), np.log(100), 8))
    wmesh = W.mesh(3, (2, 2, 2), lam=None, lam_e=lam_e)
    N = W.num_nodes(3, (2, 2, 2))
    f = rng.standard_normal((1, N))
    t = rng.standard_normal((1, N))
    d, J = _metric(wmesh)
    grads = []
    for dev in ("cpu", "cuda"):
        ctx, idx, ft, tt = _setup(wmesh, f, t)
        lam_t = torch.tensor(lam_e, device=dev, requires_grad=True)
        dm_t = torch.tensor(d[:, 1:], device=dev, requires_grad=True)
        loss = _loss(autograd.solve(ctx, ft, lam_t, dm_t, tol=1e-14), tt, idx)
        loss.backward()
        assert lam_t.grad.device.type == dev and dm_t.grad.device.type == dev
        grads.append((lam_t.grad.cpu().numpy(), dm_t.grad.cpu().numpy(), ft.grad.cpu().numpy()))
        ctx.close()
    for a, b in zip(*grads):   # the scatter's atomic order may differ between runs
        np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-10 * np.abs(b).max())


def test_backward_after_second_forward_uses_first_operator(lib):
    """Two forwards with different lambda_e on one context, then the backward
    of the first: its gradients are those of the first operator (oracle)."""
    import torch
    from oracle import grads as OG
    from oracle import mesh as M
    from paper_1601_08179_amd import autograd
    rng = np.random.default_rng(23)
    lam_a = np.exp(rng.uniform(np.log(0.1), np.log(100), 8))
    lam_b = np.exp(rng.uniform(np.log(0.1), np.log(100), 8))
    wmesh = W.mesh(3, (2, 2, 2), lam=None, lam_e=lam_a)
    N = W.num_nodes(3, (2, 2, 2))
    f = rng.standard_normal((1, N))
    t = rng.standard_normal((1, N))
    d, J = _metric(wmesh)
    ctx, idx, ft, tt = _setup(wmesh, f, t)
    la = torch.tensor(lam_a, device="cuda", requires_grad=True)
    lb = torch.tensor(lam_b, device="cuda", requires_grad=True)
    da = torch.tensor(d[:, 1:], device="cuda", requires_grad=True)
    db = torch.tensor(d[:, 1:], device="cuda", requires_grad=True)
    loss_a = _loss(autograd.solve(ctx, ft, la, da, tol=1e-14), tt, idx)
    loss_b = _loss(autograd.solve(ctx, ft.detach(), lb, db, tol=1e-14), tt, idx)
    loss_a.backward()
    om = M.make_mesh(**dict(wmesh, lam_e=lam_a, dcoef=d))
    ref = OG.loss_and_grads(om, f.T, t.T)
    assert abs(loss_a.item() - ref["loss"]) <= 1e-10 * abs(ref["loss"])
    np.testing.assert_allclose(la.grad.cpu().numpy(), ref["g_lam"], rtol=1e-9,
                               atol=1e-9 * np.abs(ref["g_lam"]).max())
    np.testing.assert_allclose(da.grad.cpu().numpy(), ref["g_d"][:, 1:], rtol=1e-9,
                               atol=1e-9 * np.abs(ref["g_d"]).max())
    np.testing.assert_allclose(ft.grad.cpu().numpy(), ref["g_f"].T, rtol=1e-9,
                               atol=1e-9 * np.abs(ref["g_f"]).max())
    # the second forward's backward still sees its own operator
    loss_b.backward()
    d_b, _ = _metric(W.mesh(3, (2, 2, 2), lam=None, lam_e=lam_b))
    omb = M.make_mesh(**dict(wmesh, lam_e=lam_b, dcoef=d_b))
    refb = OG.loss_and_grads(omb, f.T, t.T)
    np.testing.assert_allclose(lb.grad.cpu().numpy(), refb["g_lam"], rtol=1e-9,
                               atol=1e-9 * np.abs(refb["g_lam"]).max())
