"""The operator variants of Sec. 7 against the oracle, in the physical basis:
TPC (Algorithm 3 with the Table 1 suboperators) and MMC (Algorithm 2 with the
primary part, one dense element matrix per metric class and a DGEMM), each
<= 1e-12 relative (2-norm and largest entry) on the small-mesh cases and at
p = 18..32, and equal to the TPT apply to 1e-13."""

import numpy as np
import pytest

import workloads as W
from gpu_helpers import LARGE_P, MESHES, both, rel_err

pytestmark = pytest.mark.gpu

CASES = dict(MESHES)
CASES.update(LARGE_P)


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


def _check(out, ref, free, tag):
    for r in range(out.shape[1]):
        e = rel_err(out[free, r], ref[free, r])
        emax = np.abs(out[free, r] - ref[free, r]).max() / np.abs(ref[free, r]).max()
        assert e <= 1e-12 and emax <= 1e-12, (tag, r, e, emax)
    assert np.all(out[~free] == 0.0)


@pytest.mark.parametrize("name", list(CASES))
def test_tpc_matches_oracle(lib, name):
    print("case", name, flush=True)
    ctx, op, g, free = both(CASES[name]())
    u = W.random_skeleton_input(op.sizes["N"], k=2, seed=101)
    ref = op.apply(u.T)[g]
    ut = _t(u.T[g])
    ctx.variant_setup(lib.VARIANT_TPC)
    out = ctx.apply_variant(ut, lib.VARIANT_TPC).cpu().numpy()
    _check(out, ref, free, ("tpc", name))
    tpt = ctx.apply(ut, basis=lib.PHYSICAL).cpu().numpy()
    assert rel_err(out, tpt) <= 1e-13
    ctx.close()


@pytest.mark.parametrize("name", ["config1", "stretched3_p2", "stretched3_p5", "lam_e_p3", "partial_dirichlet_p4",
                                  "neumann_p6", "stretched3_p8", "p16_cube_limit", "p17_planes", "p20_stretched",
                                  "p32_lam_e"])
def test_mmc_matches_oracle(lib, name):
    print("case", name, flush=True)
    ctx, op, g, free = both(CASES[name]())
    u = W.random_skeleton_input(op.sizes["N"], k=3, seed=102)
    ref = op.apply(u.T)[g]
    ut = _t(u.T[g])
    ctx.variant_setup(lib.VARIANT_MMC)
    out = ctx.apply_variant(ut, lib.VARIANT_MMC).cpu().numpy()
    _check(out, ref, free, ("mmc", name))
    # one RHS, after the three-RHS call (the workspace is reused)
    one = ctx.apply_variant(ut[:, 1].contiguous(), lib.VARIANT_MMC).cpu().numpy()
    assert rel_err(one, out[:, 1]) <= 1e-14
    ctx.close()


def test_variant_errors(lib):
    import torch
    ctx, op, g, free = both(MESHES["config1"]())
    x = torch.zeros(ctx.N_s, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.SemcondError):
        ctx.apply_variant(x, lib.VARIANT_MMC)  # no setup yet
    with pytest.raises(lib.SemcondError):
        ctx.apply_variant(x, 7)
    ctx.close()
