"""Shared helpers of the GPU parity tests: build the same mesh for the oracle and
the library, and map between the oracle's nodal numbering and the library's
skeleton slots (through the slot coordinates the library reports)."""

import numpy as np

import workloads as W
from oracle import mesh as M
from oracle.operators import CondensedOperator


def both(wmesh):
    """(library Context, oracle CondensedOperator, slot->nodal index g, free mask)."""
    from paper_1601_08179_amd import semcond
    ctx = semcond.Context(wmesh)
    om = M.make_mesh(**wmesh)
    op = CondensedOperator(om, max_classes=100000)
    g, free = ctx.skeleton_nodal_index()
    return ctx, op, g, free


def check_layout(op, g, free):
    """The slots are a bijection onto the oracle's skeleton with the same free set."""
    assert len(np.unique(g)) == len(g)
    sk = np.nonzero(op.skel)[0]
    assert np.array_equal(np.sort(g), sk)
    assert np.array_equal(free, op.free_skel[g])


def rel_err(a, b):
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


MESHES = {
    "config1": lambda: W.config1()[0],
    "stretched3_p2": lambda: W.mesh(2, (3, 3, 3), widths=[W.geometric_widths(3, 8)] * 3, lam=1.0),
    "stretched3_p5": lambda: W.mesh(5, (3, 3, 3), widths=[W.geometric_widths(3, 8), W.geometric_widths(3, 32),
                                                          W.geometric_widths(3, 2)], lam=0.7),
    "stretched3_p8": lambda: W.mesh(8, (3, 3, 3), widths=[W.geometric_widths(3, 128)] * 3, lam=1.0),
    "lam_e_p3": lambda: W.mesh(3, (2, 3, 2), lam=None,
                               lam_e=np.exp(np.random.default_rng(3).uniform(np.log(0.1), np.log(100), 12))),
    "partial_dirichlet_p4": lambda: W.mesh(4, (3, 2, 2), lam=0.3, dirichlet=0b100110),
    "neumann_p6": lambda: W.mesh(6, (2, 2, 1), widths=[[0.3, 0.7], [0.5, 0.5], [0.25]], lam=2.0, dirichlet=0),
    # 75 metric classes: more than the apply's D^-1 tables take, so the cube
    # path recomputes D^-1 point by point (the meshes above with 6 <= n_I <= 15
    # use the per-class tables)
    "lam_e_p8_classes": lambda: W.mesh(
        8, (5, 5, 3), widths=[W.geometric_widths(5, 4), W.geometric_widths(5, 4), W.geometric_widths(3, 4)],
        lam=None, lam_e=np.exp(np.random.default_rng(8).uniform(np.log(0.1), np.log(100), 75)), dirichlet=0b011011),
    "p16_cube_limit": lambda: W.mesh(16, (2, 1, 1), lam=1.0, dirichlet=0b000001),
    "p17_planes": lambda: W.mesh(17, (2, 1, 1), widths=[[0.4, 0.6], [1.0], [0.5]], lam=1.5, dirichlet=0b000010),
}


# Degrees above the oracle's dense route (separable interior inverse, Sec. 5):
# the k-plane element path at n_I = 17..31, including the lane-group splits of
# n_I = 30, 31, with lambda > 0 or per-element lambda, graded widths (aspect
# ratios up to 100) and partial Dirichlet masks that leave vertices free.
LARGE_P = {
    "p18_lam_e": lambda: W.mesh(18, (2, 2, 1), widths=[[0.1, 0.9], [0.35, 0.65], [0.5]], lam=None,
                                lam_e=[0.2, 5.0, 60.0, 1.0], dirichlet=0b010101),
    "p20_stretched": lambda: W.mesh(20, (2, 1, 2), widths=[[0.8, 0.2], [0.3], [0.04, 0.96]], lam=1.0,
                                    dirichlet=0b100010),
    "p24_lam": lambda: W.mesh(24, (1, 2, 2), widths=[[1.0], [0.03, 0.97], [0.4, 0.6]], lam=2.5,
                              dirichlet=0b001001),
    "p28_lam_e": lambda: W.mesh(28, (2, 1, 1), widths=[[0.45, 0.55], [0.2], [0.7]], lam=None,
                                lam_e=[0.1, 100.0], dirichlet=0b000100),
    "p31_planes": lambda: W.mesh(31, (2, 1, 1), widths=[[0.7, 0.3], [0.25], [0.9]], lam=1.0, dirichlet=0b001000),
    "p32_lam_e": lambda: W.mesh(32, (2, 1, 2), widths=[[0.01, 0.99], [1.0], [0.5, 0.5]], lam=None,
                                lam_e=[0.1, 100.0, 3.0, 0.7], dirichlet=0b000100),
}


def oracle_transform(op):
    """Dense (A, fs, T) over free skeleton nodes fs: A the oracle's assembled
    condensed matrix, T the block transform with S along every interior axis of
    each entity, S from scipy's generalized eigensolver (the oracle side's own)."""
    import scipy.linalg as sla
    from oracle import gll
    p = op.p
    A, fs = op.assembled_condensed()
    A = A.toarray()
    t = gll.tables(p)
    _, S = sla.eigh(t["K"][1:p, 1:p], t["M"][1:p, 1:p])
    G = M.global_ijk(op.mesh)[fs]
    _, ids = op.entity_ids()
    T = np.zeros_like(A)
    for ent in range(ids.max() + 1):
        loc = np.nonzero(ids == ent)[0]
        gl = G[loc]
        axes = [a for a in range(3) if np.any(gl[:, a] % p != 0)]
        Tl = np.ones((1, 1))
        for a in axes[::-1]:
            Tl = np.kron(Tl, S)
        order = np.lexsort([gl[:, a] for a in range(3)])
        T[np.ix_(loc[order], loc[order])] = Tl
    return A, fs, T
