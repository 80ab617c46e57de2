"""The single-node oracle rows used by the full-size GPU parity test agree with
the oracle's assembled condensed operator on small meshes."""

import numpy as np

import workloads as W
from oracle import mesh as M
from oracle.operators import CondensedOperator
from sampled_oracle import SampledOracle


def test_sampled_rows_match_assembled_operator():
    wm = W.mesh(3, (3, 2, 2), widths=[W.geometric_widths(3, 8), W.geometric_widths(2, 4), [0.3, 0.7]],
                lam=0.9, dirichlet=0b011001)
    om = M.make_mesh(**wm)
    op = CondensedOperator(om)
    rng = np.random.default_rng(5)
    N1, N2, N3 = (a * 3 + 1 for a in wm["n"])
    u = rng.standard_normal(N1 * N2 * N3)
    ref = op.apply(u)
    so = SampledOracle(wm)
    G = M.global_ijk(om)
    free = M.free_skeleton(om)
    memo = {}
    idx = lambda a, b, c: a + N1 * (b + N2 * c)
    for g in rng.choice(free, 40, replace=False):
        I = tuple(int(x) for x in G[g])
        val = so.row(I, lambda a, b, c: u[idx(a, b, c)], memo)
        assert abs(val - ref[g]) <= 1e-13 * np.abs(ref).max()


def test_sampled_rows_match_assembled_operator_large_p():
    """Same at p = 18 (separable route) with per-element lambda."""
    lam_e = np.array([0.3, 7.0])
    wm = W.mesh(18, (2, 1, 1), widths=[[0.15, 0.85], [0.6], [1.0]], lam=None, lam_e=lam_e, dirichlet=0b000001)
    om = M.make_mesh(**wm)
    op = CondensedOperator(om)
    rng = np.random.default_rng(6)
    N1, N2, N3 = (a * 18 + 1 for a in wm["n"])
    u = rng.standard_normal(N1 * N2 * N3)
    ref = op.apply(u)
    so = SampledOracle(wm)
    G = M.global_ijk(om)
    free = M.free_skeleton(om)
    memo = {}
    idx = lambda a, b, c: a + N1 * (b + N2 * c)
    for g in rng.choice(free, 30, replace=False):
        I = tuple(int(x) for x in G[g])
        val = so.row(I, lambda a, b, c: u[idx(a, b, c)], memo)
        assert abs(val - ref[g]) <= 1e-13 * np.abs(ref).max()
