"""Seeded synthetic workloads: meshes and right-hand sides.

This module only draws inputs.  It holds none of the solver's arithmetic: no
GLL tables, no operators, no condensation.  Both the library's tests/benchmark
and the CPU oracle receive the arrays produced here.

A workload mesh is a dict of plain values:
  p, n=(n1,n2,n3), widths=[w1 (n1,), w2 (n2,), w3 (n3,)], lam (float or None),
  lam_e (None or (n_e,) with e1 fastest), dirichlet (6-bit mask, default all).
Right-hand sides are nodal arrays f[k][N] over the global GLL nodes in
lexicographic order (I1 fastest), N = prod(n_a p + 1).

Configurations (all on the unit cube unless stated):
  1  2^3 elements, p=4, lambda=1, f ~ U[-1,1]
  2  16^3 elements, p=8, lambda=1e-3, f ~ N(0,1)
  3  n = 256/p per axis, p in {2,4,8,16,32}, geometric widths with maximum
     aspect ratio AR in {1,8,32,128} on every axis, lambda=1, f ~ U[-1,1]
  4  24^3 elements, p=12, lambda=1, k=16 right-hand sides f ~ N(0,1)
  5  8^3 elements, p=8, widths ~ U[0.5,2] per axis normalised to 1,
     lambda_e log-uniform on [0.1, 100], k=8, f ~ N(0,1), targets t ~ N(0,1)
Random streams: numpy.random.default_rng(160108179 + config).
"""

import numpy as np

SEED_BASE = 160108179


def rng_for(config, salt=0):
    return np.random.default_rng(SEED_BASE + int(config) + 1000 * int(salt))


def uniform_widths(n, length=1.0):
    return np.full(int(n), float(length) / int(n))


def geometric_widths(n, aspect, length=1.0):
    """Widths h_i proportional to r^i, i = 0..n-1, r = aspect^(1/(n-1)), sum = length.

    The largest-to-smallest width ratio along the axis is ``aspect``.
    """
    n = int(n)
    if n == 1 or aspect == 1:
        return uniform_widths(n, length)
    r = float(aspect) ** (1.0 / (n - 1))
    h = r ** np.arange(n)
    return h * (float(length) / h.sum())


def expansion_widths(n, alpha, length=1.0):
    """Widths growing by the constant expansion factor alpha from the domain
    middle towards both ends (symmetric two-sided stretching)."""
    n = int(n)
    half = n // 2
    g = float(alpha) ** np.arange(half)
    h = np.concatenate((g[::-1], g)) if n % 2 == 0 else np.concatenate((g[::-1], [1.0], g))
    return h * (float(length) / h.sum())


def num_nodes(p, n):
    return int(np.prod([int(a) * int(p) + 1 for a in n]))


def mesh(p, n, widths=None, lam=1.0, lam_e=None, dirichlet=0x3F):
    n = tuple(int(a) for a in n)
    if widths is None:
        widths = [uniform_widths(a) for a in n]
    return {"p": int(p), "n": n, "widths": [np.asarray(w, dtype=np.float64) for w in widths],
            "lam": None if lam is None else float(lam),
            "lam_e": None if lam_e is None else np.asarray(lam_e, dtype=np.float64),
            "dirichlet": int(dirichlet)}


# ---------------------------------------------------------------------------
# The five configurations
# ---------------------------------------------------------------------------

def config1(k=1):
    m = mesh(4, (2, 2, 2), lam=1.0)
    f = rng_for(1).uniform(-1.0, 1.0, size=(k, num_nodes(4, m["n"])))
    return m, f


def config2(k=1, n=16, p=8):
    m = mesh(p, (n, n, n), lam=1e-3)
    f = rng_for(2).standard_normal(size=(k, num_nodes(p, m["n"])))
    return m, f


def config3(p, aspect, k=1, n=None):
    n = 256 // p if n is None else int(n)
    w = geometric_widths(n, aspect)
    m = mesh(p, (n, n, n), widths=[w, w, w], lam=1.0)
    f = rng_for(3, salt=p * 1000 + int(aspect)).uniform(-1.0, 1.0, size=(k, num_nodes(p, m["n"])))
    return m, f


def config4(k=16, n=24, p=12):
    m = mesh(p, (n, n, n), lam=1.0)
    f = rng_for(4).standard_normal(size=(k, num_nodes(p, m["n"])))
    return m, f


def config5(k=8, n=8, p=8):
    g = rng_for(5)
    widths = []
    for _ in range(3):
        w = g.uniform(0.5, 2.0, size=n)
        widths.append(w / w.sum())
    lam_e = np.exp(g.uniform(np.log(0.1), np.log(100.0), size=n ** 3))
    m = mesh(p, (n, n, n), widths=widths, lam=None, lam_e=lam_e)
    N = num_nodes(p, m["n"])
    f = g.standard_normal(size=(k, N))
    t = g.standard_normal(size=(k, N))
    return m, f, t


def random_skeleton_input(N, k=1, seed=0):
    """Dense random nodal vectors (k, N); the operator reads the skeleton part."""
    return np.random.default_rng(SEED_BASE + 7 + int(seed)).standard_normal(size=(k, N))


# ---------------------------------------------------------------------------
# Manufactured solution with inhomogeneous Dirichlet values (solver experiment
# on (0, 2 pi)^3, Sec. 8): u = cos(k(x1 - 3 x2 + 2 x3)) sin(k(1 + x1))
# sin(k(1 - x2)) sin(k(2 x1 + x2)) sin(k(3 x1 - 2 x2 + 2 x3)), f = lam u - Lap u.
# Each factor is a sinusoid of a linear form; the Laplacian of the product is
# sum_j f_j'' |w_j|^2 prod_{l != j} f_l + 2 sum_{j<l} f_j' f_l' (w_j . w_l) prod_{m != j,l} f_m.
# ---------------------------------------------------------------------------
_MS_FORMS = [  # (is_cos, direction w, offset c): factor trig(k (w . x + c))
    (True, (1.0, -3.0, 2.0), 0.0),
    (False, (1.0, 0.0, 0.0), 1.0),
    (False, (0.0, -1.0, 0.0), 1.0),
    (False, (2.0, 1.0, 0.0), 0.0),
    (False, (3.0, -2.0, 2.0), 0.0),
]


def _ms_factors(X, k):
    """Values, first and second derivatives (w.r.t. the linear form) of the factors."""
    out = []
    for is_cos, w, c in _MS_FORMS:
        t = k * (X @ np.asarray(w) + c)
        if is_cos:
            out.append((np.cos(t), -k * np.sin(t), -k * k * np.cos(t), np.asarray(w)))
        else:
            out.append((np.sin(t), k * np.cos(t), -k * k * np.sin(t), np.asarray(w)))
    return out


def manufactured_u(X, k=5.0):
    """u_ex at points X (n, 3)."""
    u = np.ones(len(X))
    for v, _, _, _ in _ms_factors(X, k):
        u = u * v
    return u


def manufactured_laplacian(X, k=5.0):
    """Lap u_ex at points X (n, 3), from the product rule above."""
    F = _ms_factors(X, k)
    n = len(F)
    lap = np.zeros(len(X))
    for j in range(n):
        term = F[j][2] * float(F[j][3] @ F[j][3])
        for l in range(n):
            if l != j:
                term = term * F[l][0]
        lap += term
        for l in range(j + 1, n):
            term = 2.0 * F[j][1] * F[l][1] * float(F[j][3] @ F[l][3])
            for m in range(n):
                if m != j and m != l:
                    term = term * F[m][0]
            lap += term
    return lap


def one_sided_widths(n, alpha, length=1.0):
    """Widths with the constant expansion factor alpha, h_i proportional to alpha^i."""
    h = float(alpha) ** np.arange(int(n))
    return h * (float(length) / h.sum())


def solver_experiment_mesh(p, alpha, n=8):
    """n^3 elements on (0, 2 pi)^3, expansion factor alpha on every axis, lambda = 0,
    Dirichlet on all faces."""
    w = one_sided_widths(n, alpha, 2.0 * np.pi)
    return mesh(p, (n, n, n), widths=[w, w, w], lam=0.0)


def nodal_coordinates(p, n, widths, x_gll):
    """(N, 3) coordinates of the global nodes (I1 fastest) from per-axis widths and
    the p+1 reference GLL nodes x_gll on [-1, 1] (origin 0)."""
    axes = []
    for a in range(3):
        h = np.asarray(widths[a], dtype=np.float64)
        left = np.concatenate(([0.0], np.cumsum(h)[:-1]))
        pts = [0.0]
        for e in range(int(n[a])):
            pts.extend(left[e] + 0.5 * h[e] * (1.0 + np.asarray(x_gll[1:])))
        axes.append(np.array(pts))
    X3, X2, X1 = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([X1.ravel(), X2.ravel(), X3.ravel()], axis=1)
