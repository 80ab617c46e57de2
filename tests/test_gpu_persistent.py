"""The persistent cooperative CG launch (k right-hand sides in one launch)
against the one-launch-per-step path and the oracle, and the autotuner."""

import os

import numpy as np
import pytest

import workloads as W
from gpu_helpers import MESHES, both, rel_err

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


@pytest.mark.parametrize("name", ["config1", "stretched3_p2", "stretched3_p5", "stretched3_p8", "lam_e_p3",
                                  "partial_dirichlet_p4", "neumann_p6", "p16_cube_limit"])
@pytest.mark.parametrize("k", [1, 4])
def test_persistent_matches_stepwise_and_oracle(lib, name, k):
    print("case", name, k, flush=True)
    ctx, op, g, free = both(MESHES[name]())
    f = W.random_skeleton_input(op.sizes["N"], k=k, seed=31)
    up, ip = ctx.solve(_t(f), tol=1e-12, persistent=True)
    us, is_ = ctx.solve(_t(f), tol=1e-12, persistent=False)
    up, us = up.cpu().numpy(), us.cpu().numpy()
    for r in range(k):
        assert ip[r]["status"] == 0 and ip[r]["rel_res"] <= 1e-12
        assert abs(ip[r]["iters"] - is_[r]["iters"]) <= 2, (ip[r], is_[r])
        assert rel_err(up[r], us[r]) <= 1e-10
    ref = op.recover_interior(f[0], op.solve_condensed(f[0]))
    assert np.abs(up[0] - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("k", [2, 8, 16])
def test_persistent_mixed_ir(lib, k):
    ctx, op, g, free = both(MESHES["stretched3_p5"]())
    f = W.random_skeleton_input(op.sizes["N"], k=k, seed=32)
    u, info = ctx.solve(_t(f), tol=1e-12, precision=lib.PREC_MIXED_IR, inner_tol=1e-4, persistent=True)
    u = u.cpu().numpy()
    for r in (0, k - 1):
        ref = op.recover_interior(f[r], op.solve_condensed(f[r]))
        assert info[r]["status"] == 0
        assert np.abs(u[r] - ref).max() <= 1e-10 * np.abs(ref).max()


def test_persistent_max_iter_and_freeze(lib):
    """max_iter stops inside the launch (ENOTCONV); a zero RHS beside others
    stays at zero iterations."""
    ctx, op, g, free = both(MESHES["stretched3_p5"]())
    f = W.random_skeleton_input(op.sizes["N"], k=2, seed=33)
    _, info = ctx.solve(_t(f), tol=1e-12, max_iter=7, persistent=True, raise_on_notconv=False)
    assert [i["iters"] for i in info] == [7, 7]
    assert all(i["status"] == lib.ENOTCONV for i in info)
    f[1] = 0.0
    u, info = ctx.solve(_t(f), tol=1e-12, persistent=True)
    assert info[1]["iters"] == 0 and np.all(u.cpu().numpy()[1] == 0.0)


def test_autotune_and_cache(lib, tmp_path):
    import torch
    ctx, op, g, free = both(MESHES["stretched3_p8"]())
    path = str(tmp_path / "tune.txt")
    S, G = ctx.autotune(k=4, dtype=torch.float64, cache_path=path)
    assert (S, G) == (0, 0) or (S >= 1 and G >= 1)       # (0, 0): one launch per step is fastest
    line = open(path).read().split()
    assert [int(v) for v in line[-2:]] == [S, G]
    S2, G2 = ctx.autotune(k=4, dtype=torch.float64, cache_path=path)   # read back from the cache
    assert (S2, G2) == (S, G)
    f = W.random_skeleton_input(op.sizes["N"], k=4, seed=34)
    u, info = ctx.solve(_t(f), tol=1e-12)                # the tuned launch
    ref = op.recover_interior(f[2], op.solve_condensed(f[2]))
    assert np.abs(u.cpu().numpy()[2] - ref).max() <= 1e-10 * np.abs(ref).max()
    with pytest.raises(lib.SemcondError):
        ctx.autotune(k=3)


def test_autotune_cache_entries_both_kinds(lib, tmp_path):
    """A cache line naming one launch per step (0 0) or a persistent grid is
    taken as it is; a grid beyond what the device holds is rejected at solve."""
    import torch
    ctx, op, g, free = both(MESHES["stretched3_p5"]())
    f = W.random_skeleton_input(op.sizes["N"], k=2, seed=35)
    ref = op.recover_interior(f[1], op.solve_condensed(f[1]))
    key = "%d %d %d %d 2 %d" % (ctx.p, *ctx.n, lib.F64)
    for S, G in [(0, 0), (1, 16)]:
        path = str(tmp_path / ("c%d.txt" % S))
        open(path, "w").write("%s %d %d\n" % (key, S, G))
        assert ctx.autotune(k=2, dtype=torch.float64, cache_path=path) == (S, G)
        u, info = ctx.solve(_t(f), tol=1e-12)
        assert all(i["status"] == 0 for i in info)
        assert np.abs(u.cpu().numpy()[1] - ref).max() <= 1e-10 * np.abs(ref).max()
    path = str(tmp_path / "big.txt")
    open(path, "w").write("%s 1 100000000\n" % key)
    ctx.autotune(k=2, dtype=torch.float64, cache_path=path)
    with pytest.raises(lib.SemcondError):
        ctx.solve(_t(f), tol=1e-12)
