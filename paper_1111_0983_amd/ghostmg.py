"""ctypes binding of the C ABI declared in include/ghostmg.h (argument marshalling only).

Device buffers are torch tensors on the GPU; every step of the solve runs in the HIP
library.  Importing this module loads libghostmg.so and raises if it is missing: there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libghostmg.so")

MG_OK, MG_EINVAL, MG_ENOMEM, MG_EHIP, MG_EGEOM, MG_ENOCONV, MG_EDIVERGED = 0, -1, -2, -3, -4, -5, -6
MG_FP64, MG_FP32_DC = 0, 1
KERNELS = {"relax": 0, "defect": 1, "restrict": 2, "prolong": 3, "residual": 4,
           "relax_prolong": 5, "relax_restrict": 6, "coarse": 7}


class mg_grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("lo", ctypes.c_double),
                ("hi", ctypes.c_double), ("n_coarse", ctypes.c_int), ("nu1", ctypes.c_int),
                ("nu2", ctypes.c_int), ("gamma", ctypes.c_int), ("lambda_", ctypes.c_int),
                ("delta_h", ctypes.c_double), ("cD", ctypes.c_double), ("cN", ctypes.c_double),
                ("split", ctypes.c_int), ("precision", ctypes.c_int),
                ("inner_cycles", ctypes.c_int), ("max_cycles", ctypes.c_int),
                ("batch", ctypes.c_int), ("smoother", ctypes.c_int)]


class mg_bc_rule(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double * 3), ("c", ctypes.c_double), ("strict", ctypes.c_int)]


class mg_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("cycles", ctypes.c_int), ("outer", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_len", ctypes.c_int)]


# partition of the boundary: (problem, B[3], ctx) -> nonzero on Gamma_D
MG_BC_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                            ctypes.c_void_p)


class GhostMGError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    # torch (and its HIP runtime) is loaded first, so that the library binds to the runtime
    # that owns the tensors it is given; with the library loaded before torch, its HIP calls
    # reported that no device was present
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    lib.mg_grid_default.argtypes = [ctypes.POINTER(mg_grid), ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.mg_setup.argtypes = [vp, ctypes.POINTER(mg_bc_rule), ctypes.POINTER(mg_grid),
                             ctypes.POINTER(vp)]
    lib.mg_setup_partition.argtypes = [vp, MG_BC_FN, vp, ctypes.POINTER(mg_grid),
                                       ctypes.POINTER(vp)]
    lib.mg_set_stream.argtypes = [vp, vp]
    lib.mg_query_level.argtypes = [vp, ctypes.c_int, vp]
    lib.mg_query_ghosts.argtypes = [vp, ctypes.c_int, ctypes.c_int, i64p, vp, vp, vp, vp, vp]
    lib.mg_query_classes.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp]
    lib.mg_solve.argtypes = [vp, vp, vp, vp, ctypes.c_double, ctypes.POINTER(mg_stats)]
    lib.mg_cycles.argtypes = [vp, vp, vp, vp, ctypes.c_int]
    lib.mg_residual.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.mg_rho.argtypes = [vp, vp, ctypes.c_int, ctypes.c_double, vp, vp, vp]
    lib.mg_warm_start.argtypes = [vp, vp, vp]
    lib.mg_reinit.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                              ctypes.c_double, vp, ctypes.c_int, vp, vp, vp]
    lib.mg_time_kernel.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.mg_free.argtypes = [vp]
    lib.mg_free.restype = None
    lib.mg_strerror.argtypes = [ctypes.c_int]
    lib.mg_strerror.restype = ctypes.c_char_p
    return lib


_lib = _load()
lib = _lib


def strerror(code: int) -> str:
    return _lib.mg_strerror(int(code)).decode()


def _check(code, what):
    if code != MG_OK:
        raise GhostMGError(code, what)


def mg_grid_default(dim: int, n: int, n_coarse: int, **kw) -> mg_grid:
    g = mg_grid()
    _check(_lib.mg_grid_default(ctypes.byref(g), dim, n, n_coarse), "mg_grid_default")
    for k, v in kw.items():
        setattr(g, "lambda_" if k in ("lam", "lambda") else k, v)
    return g


def _rules(rules):
    if isinstance(rules, dict):
        rules = [rules]
    arr = (mg_bc_rule * len(rules))()
    for i, r in enumerate(rules):
        a = list(r.get("a", (0.0, 0.0, 0.0))) + [0.0] * 3
        arr[i].a = (ctypes.c_double * 3)(*a[:3])
        arr[i].c = float(r.get("c", 0.0))
        arr[i].strict = int(r.get("strict", 1))
    return arr


def _ptr(t):
    """Device (or host) address of a contiguous float64 tensor / array."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        assert t.dtype == np.float64 and t.flags.c_contiguous
        return ctypes.c_void_p(t.ctypes.data)
    assert t.dtype.is_floating_point and t.is_contiguous()
    return ctypes.c_void_p(t.data_ptr())


def reinit(phi0, dim: int, n: int, iters: int, batch: int = 1, lo: float = -1.0,
           hi: float = 1.0, stream=None):
    """Signed distance function from the level-set function phi0 (device tensor of
    batch * (n+1)^dim FP64 values) by `iters` steps of Eq. (sdf) (mg_reinit)."""
    import torch

    assert phi0.dtype == torch.float64 and phi0.is_contiguous() and phi0.is_cuda
    phi = torch.empty_like(phi0)
    tmp = torch.empty_like(phi0)
    _check(_lib.mg_reinit(dim, n, batch, lo, hi, _ptr(phi0), int(iters), _ptr(phi), _ptr(tmp),
                          ctypes.c_void_p(stream)), "mg_reinit")
    return phi


class Solver:
    """One mg_setup handle.  phi: torch tensor (device or host) or numpy array of
    batch * (n+1)^dim FP64 values; rules: one dict per problem (see mg_bc_rule), or
    partition: a function (problem, B) -> bool (True on Gamma_D) called during setup."""

    def __init__(self, phi, rules, grid: mg_grid, partition=None):
        import torch

        if isinstance(phi, torch.Tensor):
            assert phi.dtype == torch.float64
            phi = phi.contiguous()
        self._phi_keep = phi
        self.grid = grid
        self.dim, self.n, self.batch = grid.dim, grid.n, grid.batch
        h = ctypes.c_void_p()
        if partition is not None:
            cb = MG_BC_FN(lambda p, B, ctx: int(bool(partition(p, (B[0], B[1], B[2])))))
            _check(_lib.mg_setup_partition(_ptr(phi), cb, None, ctypes.byref(grid),
                                           ctypes.byref(h)), "mg_setup_partition")
        else:
            _check(_lib.mg_setup(_ptr(phi), _rules(rules), ctypes.byref(grid), ctypes.byref(h)),
                   "mg_setup")
        self._h = h
        self.nlev = int(self.level(0)["levels"])
        self._phi_keep = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.mg_free(h)
            self._h = None

    def close(self):
        self.__del__()

    def set_stream(self, stream_ptr: int | None):
        _check(_lib.mg_set_stream(self._h, ctypes.c_void_p(stream_ptr or 0)), "mg_set_stream")

    def level(self, l: int) -> dict:
        info = np.zeros(8, np.int64)
        _check(_lib.mg_query_level(self._h, l, ctypes.c_void_p(info.ctypes.data)), "mg_query_level")
        keys = ("n", "nint", "nghost", "nband", "next", "ntiles", "ncoarse", "levels")
        return dict(zip(keys, info.tolist()))

    def ghosts(self, problem: int = 0, level: int = 0) -> dict:
        cnt = ctypes.c_int64(0)
        _check(_lib.mg_query_ghosts(self._h, problem, level, ctypes.byref(cnt), None, None, None,
                                    None, None), "mg_query_ghosts")
        n = cnt.value
        o = dict(node=np.zeros(n, np.int64), B=np.zeros((n, 3)), nB=np.zeros((n, 3)),
                 type=np.zeros(n, np.int8), rung=np.zeros(n, np.int8))
        _check(_lib.mg_query_ghosts(self._h, problem, level, ctypes.byref(cnt),
                                    *[ctypes.c_void_p(o[k].ctypes.data)
                                      for k in ("node", "B", "nB", "type", "rung")]),
               "mg_query_ghosts")
        return o

    def classes(self, problem: int = 0, level: int = 0) -> np.ndarray:
        n = self.level(level)["n"]
        c = np.zeros((n + 1) ** self.dim, np.int8)
        _check(_lib.mg_query_classes(self._h, problem, level, ctypes.c_void_p(c.ctypes.data)),
               "mg_query_classes")
        return c

    def solve(self, f, g, u, tol: float = 1e-10, check: bool = True) -> dict:
        st = mg_stats()
        rc = _lib.mg_solve(self._h, _ptr(f), _ptr(g), _ptr(u), float(tol), ctypes.byref(st))
        if check and rc not in (MG_OK,):
            raise GhostMGError(rc, "mg_solve")
        hist = [st.history[i] for i in range(st.history_len)] if st.history_len else []
        return dict(status=rc, cycles=st.cycles, outer=st.outer, rel=st.rel_residual,
                    ms=st.solve_ms, history=hist)

    def cycles(self, f, g, u, ncycles: int):
        _check(_lib.mg_cycles(self._h, _ptr(f), _ptr(g), _ptr(u), int(ncycles)), "mg_cycles")

    def warm_start(self, prev: "Solver", u):
        """Map the solution u of handle prev onto this handle's unknowns, in place
        (mg_warm_start)."""
        _check(_lib.mg_warm_start(self._h, prev._h, _ptr(u)), "mg_warm_start")

    def rho(self, u0, max_cycles: int = 100, rtol: float = 1e-3):
        """Convergence factor of the cycle on the homogeneous problem from u0 (mg_rho):
        (last factor, the factors of every cycle)."""
        hist = np.zeros(max_cycles)
        r = ctypes.c_double(0.0)
        m = ctypes.c_int(0)
        _check(_lib.mg_rho(self._h, _ptr(u0), int(max_cycles), float(rtol), ctypes.byref(r),
                           ctypes.c_void_p(hist.ctypes.data), ctypes.byref(m)), "mg_rho")
        return r.value, hist[:m.value]

    def residual(self, f, g, u, r=None):
        norms = np.zeros(2 * self.batch)
        _check(_lib.mg_residual(self._h, _ptr(f), _ptr(g), _ptr(u), _ptr(r),
                                ctypes.c_void_p(norms.ctypes.data)), "mg_residual")
        return norms.reshape(self.batch, 2)

    def time_kernel(self, kernel: str, level: int = 0, reps: int = 20):
        ms = ctypes.c_double(0)
        by = ctypes.c_double(0)
        _check(_lib.mg_time_kernel(self._h, KERNELS[kernel], level, reps, ctypes.byref(ms),
                                   ctypes.byref(by)), "mg_time_kernel")
        return ms.value, by.value
