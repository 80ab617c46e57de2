"""Python binding of libsemcond (ctypes): argument marshalling only.

Every computation runs in the HIP library; this module checks shapes, dtypes
and devices of torch tensors, passes raw device pointers and the current HIP
stream, and turns status codes into exceptions.  There is no fallback: if the
library is missing or fails to load, importing this module raises.
"""

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SEMCOND_LIBRARY") or os.path.join(HERE, "libsemcond.so")

OK, ENOTCONV, EINVAL, ENOMEM, EDEVICE, EBREAKDOWN, ENONFINITE = 0, 1, -1, -2, -3, -4, -5
F64, F32 = 0, 1
PHYSICAL, TRANSFORMED = 0, 1
COEF_TO_TRANSFORMED, COEF_TO_PHYSICAL, DUAL_TO_TRANSFORMED, DUAL_TO_PHYSICAL = 0, 1, 2, 3
PREC_F64, PREC_F32, PREC_MIXED_IR = 0, 1, 2
KERNEL_APPLY, KERNEL_PCG, KERNEL_APPLY_F32 = 0, 1, 2
VARIANT_TPC, VARIANT_MMC = 1, 2
CG_STEPWISE, CG_PERSISTENT, CG_AUTO = 0, 1, -1

_c_double_p = ctypes.POINTER(ctypes.c_double)


class Mesh(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("n", ctypes.c_int * 3), ("widths", _c_double_p * 3),
                ("lam", ctypes.c_double), ("lambda_e", _c_double_p), ("dcoef_e", _c_double_p),
                ("dirichlet_mask", ctypes.c_uint)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("precision", ctypes.c_int),
                ("check_every", ctypes.c_int), ("recover_interior", ctypes.c_int),
                ("x0", ctypes.c_void_p), ("skel_out", ctypes.c_void_p),
                ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int), ("rhs_dual", ctypes.c_int),
                ("persistent", ctypes.c_int), ("g_dirichlet", ctypes.c_void_p), ("ir_restart", ctypes.c_int),
                ("deterministic", ctypes.c_int), ("coarse", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("status", ctypes.c_int)]


# Exported symbols with their ctypes signatures (kept in step with include/semcond.h).
_SIGS = {
    "semcond_version": (ctypes.c_char_p, []),
    "semcond_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "semcond_host_tables": (ctypes.c_int, [ctypes.c_int] + [_c_double_p] * 5),
    "semcond_create": (ctypes.c_int, [ctypes.POINTER(Mesh), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "semcond_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "semcond_set_deterministic": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "semcond_sizes": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int64)] * 4),
    "semcond_skeleton_coords": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                               ctypes.POINTER(ctypes.c_uint8)]),
    "semcond_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "semcond_apply_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "semcond_variant_setup": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "semcond_apply_variant": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_void_p]),
    "semcond_transform": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "semcond_precond_diag": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "semcond_condense_rhs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                            ctypes.c_int, ctypes.c_void_p]),
    "semcond_skeleton_to_nodal": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_int, ctypes.c_void_p]),
    "semcond_nodal_to_skeleton": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_int, ctypes.c_void_p]),
    "semcond_solve_opts_default": (None, [ctypes.POINTER(SolveOpts)]),
    "semcond_recover_interior": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "semcond_reserve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "semcond_update_coefficients": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double, _c_double_p, _c_double_p,
                                                   ctypes.c_void_p]),
    "semcond_nodal_mass": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "semcond_mass_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_void_p]),
    "semcond_element_grads": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int, ctypes.c_void_p]),
    "semcond_element_grads_rhs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "semcond_set_rhs_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "semcond_get_rhs_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                             ctypes.POINTER(ctypes.c_int)]),
    "semcond_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_char_p,
                                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "semcond_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "semcond_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "semcond_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), ctypes.c_void_p]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsemcond.so is not built (run paper_1601_08179_amd.build.build())")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


class SemcondError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("semcond error %d: %s" % (code, msg))
        self.code = code


def _check(code, ctx=None, allow=(OK,)):
    if code not in allow:
        msg = _lib.semcond_last_error(ctx)
        raise SemcondError(code, msg.decode() if msg else "")
    return code


def version():
    return _lib.semcond_version().decode()


def host_tables(p):
    """1D tables computed by the library's host code (no GPU needed)."""
    if not 2 <= int(p) <= 32:
        _check(_lib.semcond_host_tables(int(p), None, None, None, None, None))
    n, ni = p + 1, p - 1
    x, w = np.zeros(n), np.zeros(n)
    K, S, lam = np.zeros(n * n), np.zeros(ni * ni), np.zeros(ni)
    ptr = lambda a: a.ctypes.data_as(_c_double_p)
    _check(_lib.semcond_host_tables(p, ptr(x), ptr(w), ptr(K), ptr(S), ptr(lam)))
    return {"x": x, "w": w, "K": K.reshape(n, n), "S": S.reshape(ni, ni), "lam": lam}


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("tensor dtype must be float64 or float32")


def _dev(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


# Contexts still open.  They are destroyed by an exit hook that runs while the
# HIP runtime is still intact (Python's exit hooks run before the C runtime's
# exit handlers tear HIP down); a context reached only by the garbage collector
# during interpreter shutdown is left to the process exit instead of calling
# into a runtime that may already be gone.
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    for c in list(_live):
        try:
            c.close()
        except Exception:
            pass


class Context:
    """A mesh + degree + lambda on the current device (semcond_create).

    mesh: dict with p, n, widths (3 arrays), lam (or None), lam_e (or None),
    optional dcoef (n_e x 4), dirichlet (6-bit mask, default 63).
    """

    def __init__(self, mesh, stream=None):
        p = int(mesh["p"])
        n = [int(v) for v in mesh["n"]]
        self._widths = [np.ascontiguousarray(w, dtype=np.float64) for w in mesh["widths"]]
        lam_e = mesh.get("lam_e")
        dcoef = mesh.get("dcoef")
        self._lam_e = None if lam_e is None else np.ascontiguousarray(lam_e, dtype=np.float64)
        self._dcoef = None if dcoef is None else np.ascontiguousarray(dcoef, dtype=np.float64).reshape(-1)
        m = Mesh()
        m.p = p
        for a in range(3):
            m.n[a] = n[a]
            m.widths[a] = self._widths[a].ctypes.data_as(_c_double_p)
        lam = mesh.get("lam")
        m.lam = 0.0 if lam is None else float(lam)
        m.lambda_e = self._lam_e.ctypes.data_as(_c_double_p) if self._lam_e is not None else None
        m.dcoef_e = self._dcoef.ctypes.data_as(_c_double_p) if self._dcoef is not None else None
        m.dirichlet_mask = int(mesh.get("dirichlet", 0x3F))
        h = ctypes.c_void_p()
        _check(_lib.semcond_create(ctypes.byref(m), _stream(stream), ctypes.byref(h)))
        self._h = h
        self.coef_version = 0  # bumped by update_coefficients
        _live.add(self)
        self.p = p
        self.n = tuple(n)
        vals = [ctypes.c_int64() for _ in range(4)]
        _check(_lib.semcond_sizes(self._h, *[ctypes.byref(v) for v in vals]), self._h)
        self.N, self.N_s, self.N_free, self.n_e = (v.value for v in vals)

    def close(self):
        if getattr(self, "_h", None):
            _lib.semcond_destroy(self._h)
            self._h = None
        _live.discard(self)

    def __del__(self, _finalizing=sys.is_finalizing):
        # (bound as a default: module globals may already be cleared when a
        # context is collected during interpreter shutdown)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_deterministic(self, on=True):
        """Fixed-order assembly (per-side slots, no atomics) for later applies,
        condensations and solves on this context."""
        _check(_lib.semcond_set_deterministic(self._h, 1 if on else 0), self._h)

    # -- introspection ---------------------------------------------------------
    def skeleton_coords(self):
        ijk = np.zeros((self.N_s, 3), dtype=np.int32)
        free = np.zeros(self.N_s, dtype=np.uint8)
        _check(_lib.semcond_skeleton_coords(self._h, ijk.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            free.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))), self._h)
        return ijk, free.astype(bool)

    def skeleton_nodal_index(self):
        """Nodal number of every skeleton slot (host numpy), and the free mask."""
        ijk, free = self.skeleton_coords()
        N1 = self.n[0] * self.p + 1
        N2 = self.n[1] * self.p + 1
        g = ijk[:, 0].astype(np.int64) + N1 * (ijk[:, 1].astype(np.int64) + N2 * ijk[:, 2].astype(np.int64))
        return g, free

    # -- tracing -------------------------------------------------------------------
    def profile_enable(self, enable=True):
        _check(_lib.semcond_profile_enable(self._h, 1 if enable else 0), self._h)

    def profile_read(self, kernel=KERNEL_APPLY):
        """(summed kernel milliseconds, launches, CG iterations) since the last enable."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        it = ctypes.c_int64()
        _check(_lib.semcond_profile_read(self._h, int(kernel), ctypes.byref(ms), ctypes.byref(n),
                                         ctypes.byref(it)), self._h)
        return ms.value, n.value, it.value

    # -- operations --------------------------------------------------------------
    def _k_skel(self, t, name):
        if t.dim() == 1:
            k = 1
        elif t.dim() == 2:
            k = t.shape[1]
        else:
            raise ValueError("%s must be (N_s,) or (N_s, k)" % name)
        if t.shape[0] != self.N_s:
            raise ValueError("%s has %d rows, expected N_s = %d" % (name, t.shape[0], self.N_s))
        return k

    def _k_nodal(self, t, name):
        if t.dim() == 1:
            k = 1
            n = t.shape[0]
        elif t.dim() == 2:
            k, n = t.shape
        else:
            raise ValueError("%s must be (N,) or (k, N)" % name)
        if n != self.N:
            raise ValueError("%s has %d nodes, expected N = %d" % (name, n, self.N))
        return k

    def apply(self, u, out=None, basis=TRANSFORMED, stream=None):
        import torch
        k = self._k_skel(u, "u")
        if out is None:
            out = torch.empty_like(u)
        if out.shape != u.shape or out.dtype != u.dtype:
            raise ValueError("out must match u")
        _check(_lib.semcond_apply(self._h, _dev(u, "u"), _dev(out, "out"), k, _dtype_code(u), basis,
                                  _stream(stream)), self._h)
        return out

    def variant_setup(self, variant, stream=None):
        """Precomputation of an operator variant of Sec. 7 (MMC: element matrices)."""
        _check(_lib.semcond_variant_setup(self._h, int(variant), _stream(stream)), self._h)

    def apply_variant(self, u, variant, out=None, stream=None):
        """TPC or MMC evaluation of the condensed operator, physical basis, FP64 [N_s] or [N_s][k]."""
        import torch
        k = self._k_skel(u, "u")
        if u.dtype != torch.float64:
            raise TypeError("u must be float64")
        if out is None:
            out = torch.empty_like(u)
        if out.shape != u.shape or out.dtype != u.dtype:
            raise ValueError("out must match u")
        _check(_lib.semcond_apply_variant(self._h, _dev(u, "u"), _dev(out, "out"), k, int(variant),
                                          _stream(stream)), self._h)
        return out

    def transform(self, x, direction, out=None, stream=None):
        import torch
        k = self._k_skel(x, "x")
        if out is None:
            out = torch.empty_like(x)
        _check(_lib.semcond_transform(self._h, _dev(x, "x"), _dev(out, "out"), k, _dtype_code(x), direction,
                                      _stream(stream)), self._h)
        return out

    def precond_diag(self, dtype=None, stream=None):
        import torch
        dtype = dtype or torch.float64
        out = torch.empty(self.N_s, dtype=dtype, device="cuda")
        _check(_lib.semcond_precond_diag(self._h, _dev(out, "out"), _dtype_code(out), _stream(stream)), self._h)
        return out

    def condense_rhs(self, f, dtype=None, stream=None):
        import torch
        k = self._k_nodal(f, "f")
        if f.dtype != torch.float64:
            raise TypeError("f must be float64")
        dtype = dtype or torch.float64
        out = torch.empty((self.N_s, k) if f.dim() == 2 else (self.N_s,), dtype=dtype, device=f.device)
        _check(_lib.semcond_condense_rhs(self._h, _dev(f, "f"), _dev(out, "out"), k, _dtype_code(out),
                                         _stream(stream)), self._h)
        return out

    def recover_interior(self, f, u_skel, out=None, stream=None):
        """Nodal solution from nodal right-hand sides f ((k, N) or (N,)) and the
        TRANSFORMED skeleton solution u_skel ((N_s, k) or (N_s,)), e.g. a solve's
        skel_out: skeleton nodes u = T u~, interior nodes recovered per element."""
        import torch
        k = self._k_nodal(f, "f")
        if self._k_skel(u_skel, "u_skel") != k:
            raise ValueError("u_skel must hold as many right-hand sides as f")
        if f.dtype != torch.float64 or u_skel.dtype != torch.float64:
            raise TypeError("f and u_skel must be float64")
        if out is None:
            out = torch.empty_like(f)
        _check(_lib.semcond_recover_interior(self._h, _dev(f, "f"), _dev(u_skel, "u_skel"), _dev(out, "out"), k, F64,
                                             _stream(stream)), self._h)
        return out

    def reserve(self, k_max, dtype=None):
        """Pre-size the workspace for calls with up to k_max right-hand sides
        (dtype torch.float32: FP32 and mixed-precision solves too)."""
        import torch
        code = F32 if dtype == torch.float32 else F64
        _check(_lib.semcond_reserve(self._h, int(k_max), code), self._h)

    def skeleton_to_nodal(self, skel, nodal=None, stream=None):
        import torch
        k = self._k_skel(skel, "skel")
        if nodal is None:
            nodal = torch.zeros((k, self.N) if skel.dim() == 2 else (self.N,), dtype=torch.float64,
                                device=skel.device)
        _check(_lib.semcond_skeleton_to_nodal(self._h, _dev(skel, "skel"), _dev(nodal, "nodal"), k,
                                              _stream(stream)), self._h)
        return nodal

    def nodal_to_skeleton(self, nodal, stream=None):
        import torch
        k = self._k_nodal(nodal, "nodal")
        out = torch.empty((self.N_s, k) if nodal.dim() == 2 else (self.N_s,), dtype=torch.float64,
                          device=nodal.device)
        _check(_lib.semcond_nodal_to_skeleton(self._h, _dev(nodal, "nodal"), _dev(out, "out"), k,
                                              _stream(stream)), self._h)
        return out

    def update_coefficients(self, lam=None, lam_e=None, dcoef=None, stream=None):
        """Replace lambda / lambda_e / metric table and rebuild the preconditioner."""
        self._lam_e = None if lam_e is None else np.ascontiguousarray(lam_e, dtype=np.float64).reshape(-1)
        self._dcoef = None if dcoef is None else np.ascontiguousarray(dcoef, dtype=np.float64).reshape(-1)
        le = self._lam_e.ctypes.data_as(_c_double_p) if self._lam_e is not None else None
        dc = self._dcoef.ctypes.data_as(_c_double_p) if self._dcoef is not None else None
        _check(_lib.semcond_update_coefficients(self._h, 0.0 if lam is None else float(lam), le, dc,
                                                _stream(stream)), self._h)
        self.coef_version += 1

    def set_rhs_batch(self, R):
        """Right-hand sides per workgroup of the batched condensation / recovery
        (R > 0 fixed, -1: per-item kernels, 0: timed per k on first use)."""
        _check(_lib.semcond_set_rhs_batch(self._h, int(R)), self._h)

    def rhs_batch(self, k):
        """(R_condense, R_recover) in use for k right-hand sides (0: per-item
        kernels, -1: not yet timed)."""
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(_lib.semcond_get_rhs_batch(self._h, int(k), ctypes.byref(a), ctypes.byref(b)), self._h)
        return a.value, b.value

    def autotune(self, k=1, dtype=None, cache_path=None):
        """Pick the CG launch by timing; returns (S, G): the persistent grid, or (0, 0) for one
        launch per step.  Later solves with persistent=None use the choice."""
        import torch
        code = F32 if dtype == torch.float32 else F64
        S = ctypes.c_int()
        G = ctypes.c_int()
        _check(_lib.semcond_autotune(self._h, int(k), code, None if cache_path is None else cache_path.encode(),
                                     ctypes.byref(S), ctypes.byref(G)), self._h)
        return S.value, G.value

    def nodal_mass(self, stream=None):
        import torch
        out = torch.empty(self.N, dtype=torch.float64, device="cuda")
        _check(_lib.semcond_nodal_mass(self._h, _dev(out, "out"), _stream(stream)), self._h)
        return out

    def mass_apply(self, x, inverse=False, out=None, stream=None):
        import torch
        k = self._k_nodal(x, "x")
        if x.dtype != torch.float64:
            raise TypeError("x must be float64")
        if out is None:
            out = torch.empty_like(x)
        _check(_lib.semcond_mass_apply(self._h, _dev(x, "x"), _dev(out, "out"), k, 1 if inverse else 0,
                                       _stream(stream)), self._h)
        return out

    def element_grads(self, u, a, stream=None):
        """[n_e, 5]: dL/dd_{e,0..3} and dL/dlambda_e for adjoint a of nodal solutions u."""
        import torch
        k = self._k_nodal(u, "u")
        if a.shape != u.shape:
            raise ValueError("a must match u")
        out = torch.empty((self.n_e, 5), dtype=torch.float64, device=u.device)
        _check(_lib.semcond_element_grads(self._h, _dev(u, "u"), _dev(a, "a"), _dev(out, "out"), k,
                                          _stream(stream)), self._h)
        return out

    def element_grads_rhs(self, u, a, stream=None):
        """[n_e, 4, k]: -a_{e,r}^T A_m u_{e,r} per right-hand side r."""
        import torch
        k = self._k_nodal(u, "u")
        if a.shape != u.shape:
            raise ValueError("a must match u")
        out = torch.empty((self.n_e, 4, k), dtype=torch.float64, device=u.device)
        _check(_lib.semcond_element_grads_rhs(self._h, _dev(u, "u"), _dev(a, "a"), _dev(out, "out"), k,
                                              _stream(stream)), self._h)
        return out

    def solve(self, f, out=None, tol=1e-10, max_iter=20000, precision=PREC_F64, check_every=8,
              recover_interior=True, x0=None, skel_out=None, inner_tol=3e-3, max_outer=30,
              rhs_dual=False, persistent=None, stream=None, raise_on_notconv=True, g=None, ir_restart=False,
              deterministic=False, coarse=False):
        """Solve for nodal right-hand sides f (k, N) or (N,), FP64.  Returns (u, info).
        ir_restart (MIXED_IR): restart every FP32 inner CG from p = 0 instead of
        continuing its direction across refinement steps.
        coarse: two-level preconditioner (BT diagonal plus the trilinear coarse correction).
        persistent: True (one persistent CG launch), False (one launch per step) or None
        (the autotuned choice, else one launch per step).  g: optional nodal array like f
        with the prescribed values on the Dirichlet faces (inhomogeneous conditions)."""
        import torch
        k = self._k_nodal(f, "f")
        if f.dtype != torch.float64:
            raise TypeError("f must be float64")
        if out is None:
            out = torch.zeros_like(f)
        o = SolveOpts()
        _lib.semcond_solve_opts_default(ctypes.byref(o))
        o.tol = tol
        o.max_iter = max_iter
        o.precision = precision
        o.check_every = check_every
        o.recover_interior = 1 if recover_interior else 0
        o.x0 = None if x0 is None else _dev(x0, "x0").value
        o.skel_out = None if skel_out is None else _dev(skel_out, "skel_out").value
        o.inner_tol = inner_tol
        o.max_outer = max_outer
        o.rhs_dual = 1 if rhs_dual else 0
        o.persistent = CG_AUTO if persistent is None else (CG_PERSISTENT if persistent else CG_STEPWISE)
        o.ir_restart = 1 if ir_restart else 0
        o.deterministic = 1 if deterministic else 0
        o.coarse = 1 if coarse else 0
        if g is not None:
            if g.shape != f.shape or g.dtype != torch.float64:
                raise ValueError("g must match f (shape, float64)")
            o.g_dirichlet = _dev(g, "g").value
        info = (SolveInfo * k)()
        allow = (OK, ENOTCONV) if not raise_on_notconv else (OK,)
        _check(_lib.semcond_solve(self._h, _dev(f, "f"), _dev(out, "out"), k, ctypes.byref(o), info,
                                  _stream(stream)), self._h, allow=allow)
        return out, [{"iters": i.iters, "outer": i.outer, "rel_res": i.rel_res, "status": i.status}
                     for i in info]
