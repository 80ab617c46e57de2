"""Pin of the gradient oracle: central finite differences of direct solves."""

import numpy as np

import workloads as W
from oracle import grads, mesh as M


def _setup():
    g = np.random.default_rng(42)
    widths = [g.uniform(0.5, 2.0, 2) for _ in range(3)]
    widths = [w / w.sum() for w in widths]
    lam_e = np.exp(g.uniform(np.log(0.1), np.log(100.0), 8))
    wm = W.mesh(3, (2, 2, 2), widths=widths, lam=None, lam_e=lam_e)
    mesh = M.make_mesh(**wm)
    N = M.sizes(mesh)["N"]
    f = g.standard_normal((N, 2))
    t = g.standard_normal((N, 2))
    return mesh, f, t


def test_grads_vs_central_fd():
    mesh, f, t = _setup()
    out = grads.loss_and_grads(mesh, f, t)
    h = 1e-6
    # central differences of an FP64 loss carry rounding noise ~ eps |L| / h
    noise = 50 * np.finfo(float).eps * abs(out["loss"]) / h
    # lambda_e
    lam_e = mesh["lam_e"]
    for e in (0, 3, 7):
        lp, lm = lam_e.copy(), lam_e.copy()
        lp[e] *= 1 + h
        lm[e] *= 1 - h
        Lp = grads.loss_only(dict(mesh, lam_e=lp), f, t)
        Lm = grads.loss_only(dict(mesh, lam_e=lm), f, t)
        fd = (Lp - Lm) / (2 * h * lam_e[e])
        assert abs(fd - out["g_lam"][e]) <= 1e-6 * abs(fd) + noise / lam_e[e]
    # metric coefficients as independent parameters
    d0 = M.element_metrics(mesh)
    for e, m in ((1, 1), (2, 2), (5, 3), (6, 0)):
        dp, dm = d0.copy(), d0.copy()
        dp[e, m] *= 1 + h
        dm[e, m] *= 1 - h
        Lp = grads.loss_only(dict(mesh, dcoef=dp), f, t)
        Lm = grads.loss_only(dict(mesh, dcoef=dm), f, t)
        fd = (Lp - Lm) / (2 * h * d0[e, m])
        assert abs(fd - out["g_d"][e, m]) <= 1e-6 * abs(fd) + noise / d0[e, m]
    # nodal right-hand side (absolute step)
    fsk = np.nonzero(~M.constrained_mask(mesh))[0]
    for node in fsk[[0, 17, 101]]:
        for r in range(2):
            fp, fm = f.copy(), f.copy()
            fp[node, r] += h
            fm[node, r] -= h
            fd = (grads.loss_only(mesh, fp, t) - grads.loss_only(mesh, fm, t)) / (2 * h)
            assert abs(fd - out["g_f"][node, r]) <= 1e-6 * abs(fd) + noise
    # lambda gradient is J_e times the d_0 gradient
    np.testing.assert_allclose(out["g_lam"], M.element_jacobians(mesh) * out["g_d"][:, 0])
