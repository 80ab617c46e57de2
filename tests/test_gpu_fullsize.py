"""Apply parity at the full sizes of the stretched-mesh sweep and of the
16-right-hand-side configuration, on sampled outputs the oracle evaluates one
at a time.

At N = 257^3 nodes the oracle's assembled operator is out of reach, so for each
sampled skeleton node the oracle forms, from its definitions, every incident
element's condensed operator (explicit element matrix, Schur complement by
Cholesky, Sec. 4), applies it to that element's boundary values and sums the
rows of the node (the assembly R of Sec. 3).  Samples are the face, edge and
vertex nodes of the elements with the most extreme aspect ratios (the corners
of the geometric grading) and of seeded random elements; the GPU runs the apply
in the physical basis on the whole mesh in the launch configuration the solver
uses.  Bar: relative 2-norm error over the samples <= 1e-12 per RHS; sampled
nodes on Dirichlet faces must come back exactly 0.
"""

import numpy as np
import pytest

import workloads as W
from sampled_oracle import SampledOracle

pytestmark = pytest.mark.gpu


def _samples(wmesh, rng):
    """Global (I1, I2, I3) of face / edge / vertex nodes of anchor elements
    (fewer anchors at p >= 16, where each element's Schur complement costs
    seconds on the host)."""
    p, n = wmesh["p"], wmesh["n"]
    last = [a - 1 for a in n]
    anchors = [(0, 0, 0), (0, last[1], last[2])]
    if p < 16:
        anchors += [tuple(last), (last[0], 0, last[2]), (last[0], last[1], 0)]
    anchors += [tuple(int(rng.integers(0, a)) for a in n) for _ in range(1 if p >= 16 else 2)]
    mid = p // 2
    local = [(0, mid, mid), (p, mid, 1), (mid, 0, mid), (1, p, mid), (mid, mid, 0), (mid, 1, p),   # faces
             (mid, 0, 0), (p, mid, 0), (0, p, mid), (p, p, mid),                                     # edges
             (0, 0, 0), (p, p, p), (p, 0, p)]                                                        # vertices
    out = []
    for (e1, e2, e3) in anchors:
        for (i, j, k) in local:
            out.append((e1 * p + i, e2 * p + j, e3 * p + k))
    return sorted(set(out))


CASES = {
    "config3_p2_ar128": (lambda: W.config3(2, 128, k=1)[0], 1),
    "config3_p4_ar32": (lambda: W.config3(4, 32, k=1)[0], 1),
    "config3_p8_ar128": (lambda: W.config3(8, 128, k=1)[0], 1),
    "config3_p16_ar8": (lambda: W.config3(16, 8, k=1)[0], 1),
    "config3_p32_ar128": (lambda: W.config3(32, 128, k=1)[0], 1),
    "config4_p12_k16": (lambda: W.config4(k=1)[0], 16),
}


@pytest.mark.parametrize("name", list(CASES))
def test_apply_full_size_sampled(lib, name):
    import torch
    print("case", name, flush=True)
    make, k = CASES[name]
    wmesh = make()
    ctx = lib.Context(wmesh)
    g, free = ctx.skeleton_nodal_index()
    N1, N2 = ctx.n[0] * ctx.p + 1, ctx.n[1] * ctx.p + 1
    slot_of = {}
    rng = np.random.default_rng(160108179 + 41)
    samples = _samples(wmesh, rng)
    u = rng.standard_normal((ctx.N_s, k))
    v = ctx.apply(torch.as_tensor(u if k > 1 else u[:, 0], device="cuda"), basis=lib.PHYSICAL).cpu().numpy()
    v = v.reshape(ctx.N_s, k)
    # nodal number -> slot, for the nodes the oracle reads (sorted search, no dense table)
    order = np.argsort(g)
    gs = g[order]

    def slot(I1, I2, I3):
        G = I1 + N1 * (I2 + N2 * I3)
        key = (I1, I2, I3)
        if key not in slot_of:
            i = np.searchsorted(gs, G)
            assert gs[i] == G
            slot_of[key] = order[i]
        return slot_of[key]

    so = SampledOracle(wmesh)
    for r in sorted({0, k - 1}):
        memo = {}
        ref, got = [], []
        for I in samples:
            s = slot(*I)
            if not free[s]:
                assert v[s, r] == 0.0
                continue
            ref.append(so.row(I, lambda a, b, c: u[slot(a, b, c), r], memo))
            got.append(v[s, r])
        ref, got = np.array(ref), np.array(got)
        assert len(ref) >= 20
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(name, "rhs", r, "samples", len(ref), "rel err", err, flush=True)
        assert err <= 1e-12
    ctx.close()


# ---------------------------------------------------------------------------
# Whole-mesh oracle checks at full size
# ---------------------------------------------------------------------------

def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


@pytest.mark.parametrize("cfg", ["config2", "config5"])
def test_apply_full_size_whole_mesh(lib, cfg):
    """The 16^3 p = 8 benchmark mesh (k = 2) and the 8^3 p = 8 differentiation
    mesh with per-element lambda and graded widths (k = 8): the physical-basis
    apply at every free skeleton node against the oracle's assembled operator
    (one explicit Schur complement per element class)."""
    from gpu_helpers import both, rel_err
    print("case", cfg, flush=True)
    wmesh, k = (W.config2()[0], 2) if cfg == "config2" else (W.config5()[0], 8)
    ctx, op, g, free = both(wmesh)
    u = W.random_skeleton_input(op.sizes["N"], k=k, seed=91)
    ref = op.apply(u.T)[g]
    out = ctx.apply(_t(u.T[g]), basis=lib.PHYSICAL).cpu().numpy()
    for r in range(k):
        e = rel_err(out[free, r], ref[free, r])
        emax = np.abs(out[free, r] - ref[free, r]).max() / np.abs(ref[free, r]).max()
        assert e <= 1e-12 and emax <= 1e-12, (cfg, r, e, emax)
    print(cfg, "k", k, "max rel err", e, flush=True)
    assert np.all(out[~free] == 0.0)
    ctx.close()


@pytest.mark.parametrize("precision", ["PREC_F64", "PREC_MIXED_IR"])
def test_config4_solution_oracle_residual(lib, precision):
    """24^3 elements, p = 12, 16 N(0,1) right-hand sides solved together to
    1e-10 (FP64 CG, or FP32 inner CG with FP64 refinement): for the first and
    last right-hand side the oracle's residual ||F^ - H^ u_B|| / ||F^|| of the
    returned skeleton values (free nodes, physical basis) is <= 1e-9."""
    print("case config4", precision, flush=True)
    from oracle import mesh as M
    from oracle.operators import CondensedOperator
    wmesh, f = W.config4(k=16)
    ctx = lib.Context(wmesh)
    u, info = ctx.solve(_t(f), tol=1e-10, precision=getattr(lib, precision))
    pick = [0, 15]
    u = u[pick].cpu().numpy()
    ctx.close()
    op = CondensedOperator(M.make_mesh(**wmesh))
    fs = op.free_skel
    Fh = op.condensed_rhs(f[pick].T)
    V = op.apply(u.T)
    for j, r in enumerate(pick):
        assert info[r]["status"] == 0 and info[r]["rel_res"] <= 1e-10, info[r]
        rr = np.linalg.norm(Fh[fs, j] - V[fs, j]) / np.linalg.norm(Fh[fs, j])
        print("config4", precision, "rhs", r, "iters", info[r]["iters"], "outer", info[r]["outer"],
              "oracle residual", rr, flush=True)
        assert rr <= 1e-9, (precision, r, rr)
