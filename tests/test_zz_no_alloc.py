"""semcond_apply_noalloc (the apply for callers that cannot allocate device
memory) against semcond_apply, called through the C ABI: the same results to
the apply's parity bar on two calls in a row, the second with a smaller input,
and size / mode limits rejected on the host before any launch."""

import ctypes

import numpy as np
import pytest

import workloads as W
from gpu_helpers import MESHES, both, rel_err

pytestmark = pytest.mark.gpu

# 32 MiB fixed workspace: 2 N_s k values of the call's scalar type
WS_BYTES = 32 << 20


def _t(a, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype or torch.float64)


def _call(lib, fn, ctx, u, v, k, dtype, basis):
    import torch
    stream = torch.cuda.current_stream().cuda_stream
    return fn(ctx._h, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(v.data_ptr()), k, dtype, basis,
              ctypes.c_void_p(stream))


def _both_applies(lib, ctx, u, k, dtype, basis):
    """(semcond_apply result, semcond_apply_noalloc result) on the same input."""
    import torch
    ref = torch.full_like(u, float("nan"))
    out = torch.full_like(u, float("nan"))
    lib._check(_call(lib, lib._lib.semcond_apply, ctx, u, ref, k, dtype, basis), ctx._h)
    lib._check(_call(lib, lib._lib.semcond_apply_noalloc, ctx, u, out, k, dtype, basis), ctx._h)
    torch.cuda.synchronize()
    return ref.double().cpu().numpy(), out.double().cpu().numpy()


@pytest.mark.parametrize("name", ["stretched3_p8", "p17_planes", "lam_e_p3"])
def test_noalloc_matches_apply_two_calls(lib, name):
    import torch
    print("case", name, flush=True)
    ctx, op, g, free = both(MESHES[name]())
    # first call: physical basis, k = 3 (basis change + RHS-major copies in the workspace)
    u = W.random_skeleton_input(op.sizes["N"], k=3, seed=71)
    assert 2 * 8 * ctx.N_s * 3 <= WS_BYTES
    ref, out = _both_applies(lib, ctx, _t(u[:, g].T), 3, lib.F64, lib.PHYSICAL)
    oref = op.apply(u.T)[g]
    for r in range(3):
        assert rel_err(out[free, r], ref[free, r]) <= 1e-14
        assert rel_err(out[free, r], oref[free, r]) <= 1e-12
        assert np.all(out[~free, r] == 0.0)
    # second call, smaller input: physical basis, k = 1
    u1 = W.random_skeleton_input(op.sizes["N"], k=1, seed=72)[0]
    ref, out = _both_applies(lib, ctx, _t(u1[g]), 1, lib.F64, lib.PHYSICAL)
    oref = op.apply(u1)[g]
    assert rel_err(out[free], ref[free]) <= 1e-14
    assert rel_err(out[free], oref[free]) <= 1e-12
    assert np.all(out[~free] == 0.0)
    # transformed basis FP32, k = 2: same kernels, FP32 rounding
    x = torch.randn((ctx.N_s, 2), dtype=torch.float32, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    ref, out = _both_applies(lib, ctx, x, 2, lib.F32, lib.TRANSFORMED)
    for r in range(2):
        assert rel_err(out[:, r], ref[:, r]) <= 1e-6
    # transformed basis FP64, k = 1 (no workspace)
    x = torch.randn(ctx.N_s, dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(6))
    ref, out = _both_applies(lib, ctx, x, 1, lib.F64, lib.TRANSFORMED)
    assert rel_err(out, ref) <= 1e-14
    ctx.close()


def test_noalloc_limits(lib):
    import torch
    # 6^3 elements at p = 8: N_s = 43561, so the workspace holds k <= 48 (FP64)
    ctx = lib.Context(W.mesh(8, (6, 6, 6), lam=1.0))
    # the largest k whose FP64 workspace fits, and one more
    kmax = WS_BYTES // (2 * 8 * ctx.N_s)
    assert 1 <= kmax < 255
    u = torch.zeros((ctx.N_s, kmax + 1), dtype=torch.float64, device="cuda")
    v = torch.empty_like(u)
    rc = _call(lib, lib._lib.semcond_apply_noalloc, ctx, u, v, kmax + 1, lib.F64, lib.PHYSICAL)
    assert rc == lib.EINVAL
    assert b"32 MiB" in lib._lib.semcond_last_error(ctx._h)
    # deterministic mode needs the slot workspace: rejected
    ctx.set_deterministic(True)
    u1 = torch.zeros(ctx.N_s, dtype=torch.float64, device="cuda")
    v1 = torch.empty_like(u1)
    assert _call(lib, lib._lib.semcond_apply_noalloc, ctx, u1, v1, 1, lib.F64, lib.PHYSICAL) == lib.EINVAL
    ctx.set_deterministic(False)
    # a call at the limit itself runs (zero input -> zero output)
    uk = torch.zeros((ctx.N_s, kmax), dtype=torch.float64, device="cuda")
    vk = torch.full_like(uk, 1.0)
    lib._check(_call(lib, lib._lib.semcond_apply_noalloc, ctx, uk, vk, kmax, lib.F64, lib.PHYSICAL), ctx._h)
    torch.cuda.synchronize()
    assert float(vk.abs().max()) == 0.0
    ctx.close()
