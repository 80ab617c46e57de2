"""Differentiable solve: torch.autograd.Function around the library's BT solve.

forward:  u = H_G^-1 M_G f for nodal right-hand sides f [k, N], with the element
          operators H_e = sum_m d_{e,m} A_m (Sec. 3), d_{e,0} = J_e lambda_e and
          the metric terms d_{e,1..3} taken as independent per-element inputs.
backward: one adjoint solve with the same operator (H_G is symmetric), a =
          H_G^-1 dL/du (the library's solve with an assembled right-hand side,
          interior recovered), then dL/df = M_G a, dL/dlambda_e and dL/dd_{e,1..3}
          from the library's per-element kernel (-a_e^T A_m u_e).
All arithmetic runs in the HIP library; this module only moves tensors.

The forward sets the context's coefficients to (lambda_e, d) and leaves them
there; the backward puts them back when anything changed them in between.
"""

import torch

from . import semcond


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(fctx, f, lam_e, dmetric, ctx, tol, precision):
        dcoef = torch.zeros((ctx.n_e, 4), dtype=torch.float64)
        dcoef[:, 1:] = dmetric.detach().to("cpu", torch.float64)
        lam_h = lam_e.detach().to("cpu", torch.float64).numpy().copy()
        dcoef_h = dcoef.numpy().copy()
        ctx.update_coefficients(lam_e=lam_h, dcoef=dcoef_h)
        u, info = ctx.solve(f.detach().contiguous(), tol=tol, precision=precision)
        fctx.ctx = ctx
        fctx.tol = tol
        fctx.precision = precision
        fctx.info = info
        fctx.devices = (lam_e.device, dmetric.device)
        # the operator this solution belongs to: host copies of its coefficients
        # and the context's coefficient version right after they were set
        fctx.coef = (lam_h, dcoef_h)
        fctx.coef_version = ctx.coef_version
        fctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(fctx, grad_u):
        (u,) = fctx.saved_tensors
        ctx = fctx.ctx
        if ctx.coef_version != fctx.coef_version:
            # another forward or a coefficient update came in between: the
            # adjoint must use the operator of this forward
            ctx.update_coefficients(lam_e=fctx.coef[0], dcoef=fctx.coef[1])
            fctx.coef_version = ctx.coef_version
        a, _ = ctx.solve(grad_u.contiguous(), tol=fctx.tol, precision=fctx.precision, rhs_dual=True)
        g = ctx.element_grads(u, a)
        grad_f = ctx.mass_apply(a)
        dev_lam, dev_d = fctx.devices
        return grad_f, g[:, 4].to(dev_lam), g[:, 1:4].to(dev_d), None, None, None


def solve(ctx, f, lam_e, dmetric, tol=1e-12, precision=semcond.PREC_F64):
    """Differentiable u(f, lambda_e, d_{e,1..3}) on the mesh of `ctx` (a semcond.Context).

    f: [k, N] or [N] float64 CUDA tensor; lam_e: [n_e]; dmetric: [n_e, 3]
    (the metric coefficients d_{e,1}, d_{e,2}, d_{e,3}), on the host or the
    device (their gradients come back on the same device).  Returns nodal u like f.
    """
    return _Solve.apply(f, lam_e, dmetric, ctx, tol, precision)
