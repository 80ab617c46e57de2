"""Mesh bookkeeping of the oracle: global numbering, gather/scatter, skeleton.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3 writes the discrete system as R H_L R^T u_G = R F_L, where R^T copies
global values to the element-local vectors and R sums element contributions
back.  The oracle makes R explicit through an (n_e, (p+1)^3) table of global
node numbers.

A mesh here is a plain dict (built by ``make_mesh``):
  p         polynomial degree
  n         (n1, n2, n3) elements per axis
  widths    three arrays of element widths per axis (Cartesian mesh)
  lam       scalar Helmholtz parameter, or None when ``lam_e`` is given
  lam_e     optional per-element lambda (n_e,), element order e1 fastest
  dcoef     optional (n_e, 4) override of the metric coefficients
  dirichlet 6-bit mask of Dirichlet domain faces: bit 0 x1-low, 1 x1-high,
            2 x2-low, 3 x2-high, 4 x3-low, 5 x3-high
  origin    lower corner of the domain
"""

import numpy as np

from . import gll
from .element import metric


def make_mesh(p, n, widths, lam=1.0, lam_e=None, dcoef=None, dirichlet=0x3F,
              origin=(0.0, 0.0, 0.0)):
    n = tuple(int(v) for v in n)
    widths = [np.asarray(w, dtype=np.float64).copy() for w in widths]
    for a in range(3):
        if widths[a].shape != (n[a],):
            raise ValueError("widths[%d] must have n[%d] entries" % (a, a))
    return {"p": int(p), "n": n, "widths": widths, "lam": lam,
            "lam_e": None if lam_e is None else np.asarray(lam_e, dtype=np.float64),
            "dcoef": None if dcoef is None else np.asarray(dcoef, dtype=np.float64),
            "dirichlet": int(dirichlet), "origin": tuple(float(v) for v in origin)}


def sizes(mesh):
    p, (n1, n2, n3) = mesh["p"], mesh["n"]
    N1, N2, N3 = n1 * p + 1, n2 * p + 1, n3 * p + 1
    return {"N": N1 * N2 * N3, "Nax": (N1, N2, N3), "n_e": n1 * n2 * n3}


def element_ijk(mesh):
    """(n_e, 3) array of element indices (e1, e2, e3), e1 fastest."""
    n1, n2, n3 = mesh["n"]
    e3, e2, e1 = np.meshgrid(np.arange(n3), np.arange(n2), np.arange(n1), indexing="ij")
    return np.stack([e1.ravel(), e2.ravel(), e3.ravel()], axis=1)


def element_metrics(mesh):
    """(n_e, 4) metric coefficients d_e (Sec. 3, eq. metriccoeffelement)."""
    if mesh["dcoef"] is not None:
        return mesh["dcoef"].copy()
    E = element_ijk(mesh)
    out = np.empty((len(E), 4))
    for e, (e1, e2, e3) in enumerate(E):
        lam = mesh["lam"] if mesh["lam_e"] is None else mesh["lam_e"][e]
        out[e] = metric((mesh["widths"][0][e1], mesh["widths"][1][e2],
                         mesh["widths"][2][e3]), lam)
    return out


def element_jacobians(mesh):
    """(n_e,) J_e = h1 h2 h3 / 8, the factor of the element mass matrix."""
    E = element_ijk(mesh)
    w = mesh["widths"]
    return np.array([w[0][a] * w[1][b] * w[2][c] / 8.0 for a, b, c in E])


def gather_map(mesh):
    """(n_e, (p+1)^3) global node numbers of each element's nodes (the R^T table).

    Element node (k, j, i) of element (e1, e2, e3) is the global node
    (e1 p + i, e2 p + j, e3 p + k), numbered lexicographically with I1 fastest.
    """
    p = mesh["p"]
    N1, N2, _ = sizes(mesh)["Nax"]
    E = element_ijk(mesh)
    loc = np.arange(p + 1)
    kk, jj, ii = np.meshgrid(loc, loc, loc, indexing="ij")
    kk, jj, ii = kk.ravel(), jj.ravel(), ii.ravel()
    I1 = E[:, 0:1] * p + ii[None, :]
    I2 = E[:, 1:2] * p + jj[None, :]
    I3 = E[:, 2:3] * p + kk[None, :]
    return I1 + N1 * (I2 + N2 * I3)


def global_ijk(mesh):
    """(N, 3) array of global node indices (I1, I2, I3) in global order."""
    N1, N2, N3 = sizes(mesh)["Nax"]
    I3, I2, I1 = np.meshgrid(np.arange(N3), np.arange(N2), np.arange(N1), indexing="ij")
    return np.stack([I1.ravel(), I2.ravel(), I3.ravel()], axis=1)


def skeleton_mask(mesh):
    """Boolean (N,) mask of skeleton nodes: some global index a multiple of p."""
    p = mesh["p"]
    G = global_ijk(mesh)
    return np.any(G % p == 0, axis=1)


def constrained_mask(mesh):
    """Boolean (N,) mask of nodes on Dirichlet domain faces."""
    Nax = sizes(mesh)["Nax"]
    G = global_ijk(mesh)
    m = np.zeros(len(G), dtype=bool)
    bits = mesh["dirichlet"]
    for a in range(3):
        if bits & (1 << (2 * a)):
            m |= G[:, a] == 0
        if bits & (1 << (2 * a + 1)):
            m |= G[:, a] == Nax[a] - 1
    return m


def free_skeleton(mesh):
    """Sorted global numbers of the free (unconstrained) skeleton nodes."""
    return np.nonzero(skeleton_mask(mesh) & ~constrained_mask(mesh))[0]


def free_nodes(mesh):
    """Sorted global numbers of all unconstrained nodes."""
    return np.nonzero(~constrained_mask(mesh))[0]


def node_coordinates(mesh):
    """(N, 3) physical coordinates of the global GLL nodes."""
    p = mesh["p"]
    xi = gll.tables(p)["x"]
    axes = []
    for a in range(3):
        w = mesh["widths"][a]
        left = mesh["origin"][a] + np.concatenate(([0.0], np.cumsum(w)[:-1]))
        pts = [left[e] + (xi[:-1] + 1.0) * 0.5 * w[e] for e in range(len(w))]
        pts.append(np.array([mesh["origin"][a] + np.sum(w)]))
        axes.append(np.concatenate(pts))
    G = global_ijk(mesh)
    return np.stack([axes[0][G[:, 0]], axes[1][G[:, 1]], axes[2][G[:, 2]]], axis=1)
