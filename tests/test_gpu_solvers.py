"""GPU solver modes against the oracle: FP32 inner CG with FP64 iterative
refinement (refined solution within 1e-10 of the oracle's direct solve), the
unrefined FP32 solve (reported), k right-hand sides at once equal to k single
solves, initial guess / resume, and error reporting."""

import numpy as np
import pytest

import workloads as W
from gpu_helpers import MESHES, both, rel_err

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


def _direct(op, f):
    return np.stack([op.recover_interior(f[r], op.solve_condensed(f[r])) for r in range(f.shape[0])])


@pytest.mark.parametrize("restart", [False, True])
@pytest.mark.parametrize("name", ["config1", "stretched3_p5", "lam_e_p3", "neumann_p6", "stretched3_p8", "p17_planes"])
def test_mixed_ir_matches_direct(lib, name, restart):
    """Refinement with the inner direction continued across steps (default)
    and with every inner CG restarted."""
    print("case", name, "restart", restart, flush=True)
    ctx, op, g, free = both(MESHES[name]())
    f = W.random_skeleton_input(op.sizes["N"], k=3, seed=11)
    u, info = ctx.solve(_t(f), tol=1e-12, precision=lib.PREC_MIXED_IR, inner_tol=1e-4, ir_restart=restart)
    ref = _direct(op, f)
    u = u.cpu().numpy()
    for r in range(3):
        assert info[r]["status"] == 0 and info[r]["rel_res"] <= 1e-12, info[r]
        assert info[r]["outer"] >= 2
        assert np.abs(u[r] - ref[r]).max() <= 1e-10 * np.abs(ref[r]).max(), (name, r, info[r])


@pytest.mark.parametrize("name", ["config1", "stretched3_p5"])
def test_fp32_unrefined_reported(lib, name):
    ctx, op, g, free = both(MESHES[name]())
    f = W.random_skeleton_input(op.sizes["N"], k=2, seed=12)
    u32, info = ctx.solve(_t(f), tol=1e-6, precision=lib.PREC_F32, raise_on_notconv=False)
    u64, _ = ctx.solve(_t(f), tol=1e-12)
    d = u32.cpu().numpy() - u64.cpu().numpy()
    err = np.abs(d).max() / np.abs(u64.cpu().numpy()).max()
    print("unrefined FP32 vs FP64 max rel err", name, err, info)
    assert err < 1e-3


@pytest.mark.parametrize("precision", ["PREC_F64", "PREC_MIXED_IR"])
def test_batched_equals_single(lib, precision):
    ctx, op, g, free = both(MESHES["stretched3_p5"]())
    f = W.random_skeleton_input(op.sizes["N"], k=5, seed=13)
    prec = getattr(lib, precision)
    ub, infob = ctx.solve(_t(f), tol=1e-12, precision=prec)
    ub = ub.cpu().numpy()
    for r in range(5):
        us, infos = ctx.solve(_t(f[r]), tol=1e-12, precision=prec)
        assert rel_err(ub[r], us.cpu().numpy()) <= 1e-11
        if precision == "PREC_F64":
            assert infob[r]["iters"] == infos[0]["iters"]


def test_zero_and_mixed_rhs(lib):
    """A zero right-hand side converges in zero iterations beside nonzero ones."""
    ctx, op, g, free = both(MESHES["config1"]())
    f = W.random_skeleton_input(op.sizes["N"], k=3, seed=14)
    f[1] = 0.0
    u, info = ctx.solve(_t(f), tol=1e-12)
    assert info[1]["iters"] == 0 and np.all(u.cpu().numpy()[1] == 0.0)
    assert info[0]["iters"] > 0 and info[2]["iters"] > 0


def test_resume_from_initial_guess(lib):
    """Stop early (ENOTCONV, best iterate returned), resume with x0 = the
    transformed skeleton iterate, reach the tolerance."""
    import torch
    ctx, op, g, free = both(MESHES["stretched3_p5"]())
    f = W.random_skeleton_input(op.sizes["N"], k=1, seed=15)
    skel = torch.zeros((ctx.N_s, 1), dtype=torch.float64, device="cuda")
    _, info = ctx.solve(_t(f), tol=1e-12, max_iter=5, skel_out=skel, raise_on_notconv=False)
    assert info[0]["status"] == lib.ENOTCONV and info[0]["iters"] == 5
    u, info2 = ctx.solve(_t(f), tol=1e-12, x0=skel)
    assert info2[0]["status"] == 0
    ref = _direct(op, f)
    assert np.abs(u.cpu().numpy()[0] - ref[0]).max() <= 1e-10 * np.abs(ref).max()
    with pytest.raises(lib.SemcondError) as ei:
        ctx.solve(_t(f), tol=1e-12, max_iter=3)
    assert ei.value.code == lib.ENOTCONV


def test_invalid_arguments(lib):
    import torch
    ctx, op, g, free = both(MESHES["config1"]())
    f = _t(W.random_skeleton_input(op.sizes["N"], k=1, seed=16))
    with pytest.raises(lib.SemcondError) as ei:
        ctx.solve(f, tol=-1.0)
    assert ei.value.code == lib.EINVAL
    with pytest.raises(lib.SemcondError):
        ctx.solve(f, precision=7)
    with pytest.raises(lib.SemcondError):
        ctx.solve(f, precision=lib.PREC_MIXED_IR, inner_tol=2.0)
    with pytest.raises(ValueError):
        ctx.apply(torch.zeros(ctx.N_s + 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        ctx.apply(torch.zeros(ctx.N_s, dtype=torch.int32, device="cuda"))


def test_nonfinite_rhs_reported(lib):
    ctx, op, g, free = both(MESHES["config1"]())
    f = W.random_skeleton_input(op.sizes["N"], k=2, seed=17)
    f[1, 434] = np.nan   # node (2, 3, 5): interior of element (0, 0, 1)
    with pytest.raises(lib.SemcondError) as ei:
        ctx.solve(_t(f), tol=1e-10)
    assert ei.value.code == lib.ENONFINITE


@pytest.mark.parametrize("precision", ["PREC_F64", "PREC_MIXED_IR"])
def test_separate_reduction_loop_matches_direct(lib, precision):
    """n_e k = 216 * 76 > 16384 at p = 4: the CG loop with separate reduction
    launches, whose applies assemble edge and vertex rows (FP32: all rows)
    through per-side slots; partial Dirichlet faces leave boundary sides
    unwritten.  References: the oracle's condensed direct solve (its sparse LU
    factored once) and interior recovery."""
    import scipy.sparse.linalg as spla
    print("case separate-reduction loop", precision, flush=True)
    wm = W.mesh(4, (6, 6, 6), widths=[W.geometric_widths(6, 8)] * 3, lam=0.5, dirichlet=0b011001)
    ctx, op, g, free = both(wm)
    k = 76
    assert ctx.n_e * k > 16384
    f = W.random_skeleton_input(op.sizes["N"], k=k, seed=23)
    u, info = ctx.solve(_t(f), tol=1e-12, precision=getattr(lib, precision))
    u = u.cpu().numpy()
    A, fs = op.assembled_condensed()
    lu = spla.splu(A.tocsc())
    for r in range(0, k, 25):
        skel = np.zeros(op.sizes["N"])
        skel[fs] = lu.solve(op.condensed_rhs(f[r])[fs])
        ref = op.recover_interior(f[r], skel)
        assert info[r]["status"] == 0 and info[r]["rel_res"] <= 1e-12, info[r]
        assert np.abs(u[r] - ref).max() <= 1e-10 * np.abs(ref).max(), (r, info[r])


_P10 = {}


def _p10_case():
    """5^3 stretched elements at p = 10 with 132 RHS (n_e k = 16500 > 16384):
    built once for both precisions."""
    if not _P10:
        wm = W.mesh(10, (5, 5, 5), widths=[W.geometric_widths(5, 8)] * 3, lam=0.5, dirichlet=0b011001)
        ctx, op, g, free = both(wm)
        _P10.update(wm=wm, ctx=ctx, op=op, f=W.random_skeleton_input(op.sizes["N"], k=132, seed=29))
    return _P10


@pytest.mark.parametrize("precision", ["PREC_F64", "PREC_MIXED_IR"])
def test_separate_reduction_loop_residual_p10(lib, precision):
    """The separate-reduction loop at n_I = 9 (FP64 rows added into q, FP32
    rows through slots): the skeleton solution's residual in the oracle's own
    explicit condensed operator, F^ - H^_G u_B on free skeleton nodes, is
    within 1e-9 of F^ (the solve stops at a 1e-12 residual in the transformed
    basis)."""
    print("case separate-reduction loop p=10", precision, flush=True)
    c = _p10_case()
    ctx, op, f = c["ctx"], c["op"], c["f"]
    k = f.shape[0]
    assert ctx.n_e * k > 16384
    u, info = ctx.solve(_t(f), tol=1e-12, precision=getattr(lib, precision), recover_interior=False)
    u = u.cpu().numpy()
    for r in range(0, k, 43):
        assert info[r]["status"] == 0 and info[r]["rel_res"] <= 1e-12, info[r]
        fh = op.condensed_rhs(f[r])
        res = fh - op.apply(u[r])
        fs = op.free_skel
        assert np.linalg.norm(res[fs]) <= 1e-9 * np.linalg.norm(fh[fs]), (r, info[r])


@pytest.mark.parametrize("prescribed", [False, True])
def test_recover_interior_entry_point(lib, prescribed):
    """semcond_recover_interior on a solve's transformed skeleton output
    reproduces the solve's nodal solution (the same kernels: bitwise), which
    matches the oracle's direct solve with interior recovery; with prescribed
    Dirichlet values the skeleton output carries them."""
    import torch
    print("case recover_interior prescribed", prescribed, flush=True)
    ctx, op, g, free = both(MESHES["stretched3_p5"]())
    f = W.random_skeleton_input(op.sizes["N"], k=3, seed=31)
    skel = torch.empty((ctx.N_s, 3), dtype=torch.float64, device="cuda")
    kw = {}
    if prescribed:
        kw["g"] = _t(W.random_skeleton_input(op.sizes["N"], k=3, seed=32))
    u, info = ctx.solve(_t(f), tol=1e-13, skel_out=skel, **kw)
    v = ctx.recover_interior(_t(f), skel)
    assert torch.equal(u, v)
    if not prescribed:
        ref = _direct(op, f)
        v = v.cpu().numpy()
        for r in range(3):
            assert np.abs(v[r] - ref[r]).max() <= 1e-10 * np.abs(ref[r]).max(), (r, info[r])


def test_reserve_then_solve(lib):
    """After semcond_reserve(k_max = 4, FP32) solves and applies with k <= 4
    give what they give on a context without the reservation; invalid
    arguments are rejected."""
    import torch
    print("case reserve", flush=True)
    wm = MESHES["stretched3_p5"]()
    from paper_1601_08179_amd import semcond
    a, b = semcond.Context(wm), semcond.Context(wm)
    a.reserve(4, torch.float32)
    f = _t(W.random_skeleton_input(a.N, k=4, seed=33))
    for kw in (dict(), dict(precision=lib.PREC_MIXED_IR), dict(persistent=True)):
        ua, ia = a.solve(f, tol=1e-12, **kw)
        ub, ib = b.solve(f, tol=1e-12, **kw)
        # the right-hand side condensation adds edge and vertex rows with atomics:
        # rounding may differ between the two contexts' runs
        assert all(abs(x["iters"] - y["iters"]) <= 1 for x, y in zip(ia, ib)), kw
        d = (ua - ub).abs().max().item() / ub.abs().max().item()
        assert d <= 1e-10, (kw, d)
    x = torch.randn((a.N_s, 4), dtype=torch.float64, device="cuda")
    va, vb = a.apply(x), b.apply(x)
    assert (va - vb).abs().max().item() <= 1e-13 * vb.abs().max().item()
    with pytest.raises(lib.SemcondError):
        a.reserve(0)
    with pytest.raises(lib.SemcondError):
        lib._check(lib._lib.semcond_reserve(a._h, 4, 7), a._h)
    a.close()
    b.close()


@pytest.mark.parametrize("name", ["stretched3_p8", "p16_cube_limit"])
def test_mixed_ir_unreachable_inner_tol(lib, name):
    """An inner tolerance far below what the FP32 operator can reach (1e-9):
    the inner tolerance is raised to the FP32 rounding level and an inner
    solve that stops halving its residual ends its step, so the refinement
    converges to 1e-10 in a bounded number of steps and inner iterations."""
    print("case", name, flush=True)
    ctx, op, g, free = both(MESHES[name]())
    f = W.random_skeleton_input(op.sizes["N"], k=2, seed=18)
    _, ref_info = ctx.solve(_t(f), tol=1e-10)
    u, info = ctx.solve(_t(f), tol=1e-10, precision=lib.PREC_MIXED_IR, inner_tol=1e-9)
    ref = _direct(op, f)
    u = u.cpu().numpy()
    for r in range(2):
        print("FP64 iterations", ref_info[r]["iters"], "mixed", info[r], flush=True)
        assert info[r]["status"] == 0 and info[r]["rel_res"] <= 1e-10, info[r]
        assert info[r]["outer"] <= 12
        assert info[r]["iters"] <= 6 * ref_info[r]["iters"] + 200
        assert np.abs(u[r] - ref[r]).max() <= 1e-8 * np.abs(ref[r]).max()
