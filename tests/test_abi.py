"""CPU tests of the C ABI: the library loads, exports every symbol the header
declares, computes the host 1D tables like the oracle, and validates mesh
arguments before touching a device."""

import ctypes
import os
import re

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import gll

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "semcond.h")
LIB = os.path.join(ROOT, "paper_1601_08179_amd", "libsemcond.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(semcond_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def raw():
    if not os.path.exists(LIB):
        pytest.fail("libsemcond.so is not built; run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(raw):
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(raw, n), n


def test_binding_signatures_cover_header():
    from paper_1601_08179_amd import semcond
    assert set(_declared()) == set(semcond._SIGS)


@pytest.mark.parametrize("p", [2, 3, 5, 8, 12, 16, 24, 32])
def test_host_tables_match_oracle(p):
    from paper_1601_08179_amd import semcond
    t = semcond.host_tables(p)
    o = gll.tables(p)
    np.testing.assert_allclose(t["x"], o["x"], atol=2e-16)
    np.testing.assert_allclose(t["w"], o["w"], rtol=4e-16)
    assert np.abs(t["K"] - o["K"]).max() <= 2.5e-16 * np.abs(o["K"]).max()
    lam = sla.eigh(o["K"][1:p, 1:p], o["M"][1:p, 1:p], eigvals_only=True)
    np.testing.assert_allclose(t["lam"], lam, rtol=1e-13)
    S = t["S"]
    MII = np.diag(o["w"][1:p])
    np.testing.assert_allclose(S.T @ MII @ S, np.eye(p - 1), atol=1e-13)
    np.testing.assert_allclose(S.T @ o["K"][1:p, 1:p] @ S, np.diag(t["lam"]), atol=1e-12 * t["lam"].max())


def test_host_tables_reject_bad_p():
    from paper_1601_08179_amd import semcond
    for p in (0, 1, 33):
        with pytest.raises(semcond.SemcondError) as ei:
            semcond.host_tables(p)
        assert ei.value.code == semcond.EINVAL


def _mesh_struct(semcond, p=4, n=(2, 2, 2), widths=None, lam=1.0, mask=63):
    m = semcond.Mesh()
    m.p = p
    keep = []
    for a in range(3):
        m.n[a] = n[a]
        w = np.full(n[a], 1.0 / max(n[a], 1)) if widths is None else np.asarray(widths[a], dtype=np.float64)
        keep.append(w)
        m.widths[a] = w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    m.lam = lam
    m.lambda_e = None
    m.dcoef_e = None
    m.dirichlet_mask = mask
    return m, keep


@pytest.mark.parametrize("kw", [
    {"p": 1}, {"p": 33}, {"n": (0, 2, 2)}, {"lam": -1.0}, {"lam": float("nan")},
    {"widths": [[0.5, -0.5], [0.5, 0.5], [0.5, 0.5]]},
    {"widths": [[0.5, float("inf")], [0.5, 0.5], [0.5, 0.5]]},
    {"lam": 0.0, "mask": 0}, {"mask": 64},
])
def test_create_validates_before_device(kw):
    from paper_1601_08179_amd import semcond
    m, keep = _mesh_struct(semcond, **kw)
    h = ctypes.c_void_p()
    rc = semcond._lib.semcond_create(ctypes.byref(m), None, ctypes.byref(h))
    assert rc == semcond.EINVAL
    assert not h.value
    assert semcond._lib.semcond_last_error(None)
