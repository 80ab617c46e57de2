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
