"""FP64 CPU oracle for the ghost-cell multigrid method (arXiv 1111.0983).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product library never
does.  It shares no code with the GPU library (``paper_1111_0983_amd``).

The arithmetic lives in ``ghostmg_oracle.c`` (plain C, FP64; its red-black passes may run on
several threads with results identical to one thread's); this module is
argument marshalling plus the two "plain definition" solvers of the discrete system
Eq. (discr): a dense LAPACK solve and a sparse direct solve of the assembled rows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ghostmg_oracle.c")
_LIB = os.path.join(_HERE, "libghostmg_oracle.so")

OUT, IN, GHOST = 0, 1, 2
OK, EINVAL, ENOMEM, EGEOM, ENOCONV, EDIVERGED = 0, -1, -2, -4, -5, -6


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, so its geometry decisions are
    reproducible bit for bit)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
               "-fPIC", "-shared", "-Wall", "-Wno-unused-function", _SRC, "-o", _LIB, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


_LIB_NATIVE = os.path.join(_HERE, "libghostmg_oracle_native.so")


def use_native() -> str:
    """Compile the oracle for the host it runs on (gcc -O3 -march=native, OpenMP, still no
    FMA contraction, so results are those of the portable build) and load that library for
    every later call.  Only the CPU-baseline timing uses it; call before the first Oracle."""
    global _LIB, _lib
    cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-std=c99", "-fPIC", "-shared", "-Wall", "-Wno-unused-function", _SRC, "-o",
           _LIB_NATIVE, "-lm"]
    subprocess.run(cmd, check=True)
    _LIB, _lib = _LIB_NATIVE, None
    _load()
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int), ("lo", ctypes.c_double),
                ("hi", ctypes.c_double), ("n_coarse", ctypes.c_int), ("nu1", ctypes.c_int),
                ("nu2", ctypes.c_int), ("gamma", ctypes.c_int), ("lam", ctypes.c_int),
                ("delta_h", ctypes.c_double), ("cD", ctypes.c_double), ("cN", ctypes.c_double),
                ("ordering", ctypes.c_int), ("split", ctypes.c_int), ("smoother", ctypes.c_int)]


class _Rule(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double * 3), ("c", ctypes.c_double), ("strict", ctypes.c_int)]


# partition of the boundary: nonzero when the boundary point B (3 doubles) is on Gamma_D
_BC_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        vp, i64p, dp, i8p = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p
        _lib.orc_setup.restype = vp
        _lib.orc_setup.argtypes = [dp, ctypes.POINTER(_Rule), ctypes.POINTER(_Grid),
                                   ctypes.POINTER(ctypes.c_int)]
        _lib.orc_setup_fn.restype = vp
        _lib.orc_setup_fn.argtypes = [dp, _BC_FN, vp, ctypes.POINTER(_Grid),
                                      ctypes.POINTER(ctypes.c_int)]
        _lib.orc_free.argtypes = [vp]
        _lib.orc_free.restype = None
        _lib.orc_threads.argtypes = [ctypes.c_int]
        for name in ("orc_num_levels",):
            getattr(_lib, name).argtypes = [vp]
        _lib.orc_level_info.argtypes = [vp, ctypes.c_int, i64p]
        _lib.orc_get_cls.argtypes = [vp, ctypes.c_int, i8p, i8p]
        _lib.orc_get_ghosts.argtypes = [vp, ctypes.c_int] + [vp] * 11
        _lib.orc_get_labels.argtypes = [vp, ctypes.c_int, i8p]
        _lib.orc_get_extension.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        _lib.orc_get_boxes.argtypes = [vp, ctypes.c_int, vp, vp]
        _lib.orc_defect.argtypes = [vp, ctypes.c_int, dp, dp, dp, dp]
        _lib.orc_relax.argtypes = [vp, ctypes.c_int, dp, dp, ctypes.c_int]
        _lib.orc_extend.argtypes = [vp, ctypes.c_int, dp]
        _lib.orc_boundary_step.argtypes = [vp, ctypes.c_int, ctypes.c_int64, dp, dp, ctypes.c_int]
        _lib.orc_smoothing.argtypes = [vp, dp, ctypes.c_int, dp]
        _lib.orc_restrict.argtypes = [vp, ctypes.c_int, dp, dp]
        _lib.orc_prolong.argtypes = [vp, ctypes.c_int, dp, dp]
        _lib.orc_coarse_solve.argtypes = [vp, dp, dp]
        _lib.orc_cycle.argtypes = [vp, dp, dp]
        _lib.orc_solve.argtypes = [vp, dp, dp, ctypes.c_double, ctypes.c_int, dp,
                                   ctypes.POINTER(ctypes.c_int)]
        _lib.orc_rho.argtypes = [vp, dp, ctypes.c_int, ctypes.c_double,
                                 ctypes.POINTER(ctypes.c_double), dp,
                                 ctypes.POINTER(ctypes.c_int)]
        _lib.orc_assemble.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64), vp, vp, vp, vp]
    return _lib


def threads(n: int = 0) -> int:
    """Threads of the oracle's red-black passes (n <= 0: query).  Results do not depend on
    it."""
    return int(_load().orc_threads(int(n)))


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def default_grid(dim: int, n: int, n_coarse: int, **kw) -> dict:
    """Paper constants: lambda = 5 and delta = 3h (Sec. 3.2); mu_D dt = 0.9 and
    mu_N dt = 0.9 * 2h / (3 sqrt(d)) (Sec. 2.3, Sec. 1.1 for d = 1)."""
    g = dict(dim=dim, n=n, lo=-1.0, hi=1.0, n_coarse=n_coarse, nu1=2, nu2=1, gamma=1,
             lam=5, delta_h=3.0, cD=0.9, cN=0.9 * 2.0 / (3.0 * np.sqrt(dim)), ordering=1,
             split=1, smoother=0)
    g.update(kw)
    return g


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


class Oracle:
    """Ghost-cell multigrid hierarchy built from nodal phi on the finest grid."""

    def __init__(self, phi: np.ndarray, grid: dict, rule: dict | None = None,
                 partition=None):
        """rule: half-space Dirichlet rule {a, c, strict}; partition: instead of a rule, a
        Python function of the boundary point B (3 floats) returning True on Gamma_D."""
        lib = _load()
        self.grid = dict(grid)
        self.dim = int(grid["dim"])
        self.n = int(grid["n"])
        self.phi = np.ascontiguousarray(phi, dtype=np.float64).ravel()
        if self.phi.size != (self.n + 1) ** self.dim:
            raise ValueError("phi has the wrong size")
        g = _Grid(**{k: grid[k] for k in _Grid._fields_names})
        err = ctypes.c_int(0)
        if partition is not None:
            cb = _BC_FN(lambda B, ctx: int(bool(partition((B[0], B[1], B[2])))))
            self._h = lib.orc_setup_fn(_p(self.phi), cb, None, ctypes.byref(g),
                                       ctypes.byref(err))
        else:
            a = list(rule.get("a", (0.0, 0.0, 0.0))) + [0.0] * 3
            r = _Rule((ctypes.c_double * 3)(*a[:3]), float(rule.get("c", 0.0)),
                      int(rule.get("strict", 1)))
            self._h = lib.orc_setup(_p(self.phi), ctypes.byref(r), ctypes.byref(g),
                                    ctypes.byref(err))
        if not self._h:
            raise OracleError(err.value, "orc_setup")
        self.nlev = lib.orc_num_levels(self._h)
        self.K = 3 ** self.dim

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_free(h)
            self._h = None

    # -- structure queries ------------------------------------------------------------
    def info(self, l: int) -> dict:
        out = np.zeros(8, np.int64)
        _lib.orc_level_info(self._h, l, _p(out))
        return dict(n=int(out[0]), nn=int(out[1]), nint=int(out[2]), ng=int(out[3]),
                    nband=int(out[4]), ne=int(out[5]), nu=int(out[6]))

    def cls(self, l: int):
        nn = self.info(l)["nn"]
        c = np.zeros(nn, np.int8)
        b = np.zeros(nn, np.int8)
        _lib.orc_get_cls(self._h, l, _p(c), _p(b))
        return c, b

    def labels(self, l: int) -> np.ndarray:
        """BC type (1 D, 0 N) of the closest boundary point of every ghost and extension
        node of level l, -1 elsewhere."""
        lab = np.zeros(self.info(l)["nn"], np.int8)
        _lib.orc_get_labels(self._h, l, _p(lab))
        return lab

    def ghosts(self, l: int) -> dict:
        ng = self.info(l)["ng"]
        K = self.K
        o = dict(node=np.zeros(ng, np.int64), type=np.zeros(ng, np.int8),
                 rung=np.zeros(ng, np.int8), sgn=np.zeros((ng, 3), np.int8),
                 B=np.zeros((ng, 3)), nG=np.zeros((ng, 3)), nB=np.zeros((ng, 3)),
                 xi=np.zeros((ng, 3)), c=np.zeros(ng), wn=np.zeros((ng, K), np.int64),
                 w=np.zeros((ng, K)))
        _lib.orc_get_ghosts(self._h, l, *[_p(o[k]) for k in
                                          ("node", "type", "rung", "sgn", "B", "nG", "nB",
                                           "xi", "c", "wn", "w")])
        return o

    def extension(self, l: int) -> dict:
        ne = self.info(l)["ne"]
        o = dict(node=np.zeros(ne, np.int64), src=np.zeros((ne, 3), np.int64),
                 wt=np.zeros((ne, 3)))
        _lib.orc_get_extension(self._h, l, _p(o["node"]), _p(o["src"]), _p(o["wt"]))
        return o

    def boxes(self, l: int):
        nnc = self.info(l + 1)["nn"]
        lo = np.zeros((nnc, 3), np.int8)
        hi = np.zeros((nnc, 3), np.int8)
        _lib.orc_get_boxes(self._h, l, _p(lo), _p(hi))
        return lo, hi

    # -- operators (arrays are full-grid node arrays of the level) ---------------------
    def _arr(self, x, l):
        a = np.ascontiguousarray(x, dtype=np.float64).ravel()
        if a.size != self.info(l)["nn"]:
            raise ValueError("array has the wrong size for this level")
        return a

    def defect(self, l, u, rhs):
        u, rhs = self._arr(u, l), self._arr(rhs, l)
        r = np.zeros_like(u)
        nrm = np.zeros(2)
        _lib.orc_defect(self._h, l, _p(u), _p(rhs), _p(r), _p(nrm))
        return r, (float(nrm[0]), float(nrm[1]))

    def relax(self, l, u, rhs, band_only=-1):
        """In place.  band_only = -1: one relaxation + lambda band sweeps; 0: one pass over
        all unknowns; 1: one pass over the band."""
        assert u.dtype == np.float64 and u.flags.c_contiguous
        _lib.orc_relax(self._h, l, _p(u), _p(self._arr(rhs, l)), band_only)

    def boundary_step(self, l, P, u, rhs, kind):
        """In place: one Kaczmarz step (kind 1) or one block relaxation (kind 2) at node P of
        level l (Sec. 3.3); returns the oracle status (EGEOM: singular block)."""
        assert u.dtype == np.float64 and u.flags.c_contiguous
        return _lib.orc_boundary_step(self._h, l, int(P), _p(u), _p(self._arr(rhs, l)), kind)

    def smoothing(self, u0, iters):
        """Smoothing factors mu^(m) of the relaxation alone on the homogeneous problem."""
        u = np.ascontiguousarray(u0, dtype=np.float64).ravel().copy()
        hist = np.zeros(iters)
        _lib.orc_smoothing(self._h, _p(u), int(iters), _p(hist))
        return hist

    def extend(self, l, r):
        assert r.dtype == np.float64 and r.flags.c_contiguous
        _lib.orc_extend(self._h, l, _p(r))

    def restrict(self, l, r):
        rc = np.zeros(self.info(l + 1)["nn"])
        _lib.orc_restrict(self._h, l, _p(self._arr(r, l)), _p(rc))
        return rc

    def prolong(self, l, ec, u):
        assert u.dtype == np.float64 and u.flags.c_contiguous
        _lib.orc_prolong(self._h, l, _p(self._arr(ec, l + 1)), _p(u))

    def coarse_solve(self, rhs):
        l = self.nlev - 1
        u = np.zeros(self.info(l)["nn"])
        _lib.orc_coarse_solve(self._h, _p(u), _p(self._arr(rhs, l)))
        return u

    def cycle(self, u, rhs):
        assert u.dtype == np.float64 and u.flags.c_contiguous
        _lib.orc_cycle(self._h, _p(u), _p(self._arr(rhs, 0)))

    def solve(self, rhs, u0=None, tol=1e-10, max_cycles=100):
        u = np.zeros((self.n + 1) ** self.dim) if u0 is None else \
            np.ascontiguousarray(u0, dtype=np.float64).ravel().copy()
        hist = np.zeros(max_cycles + 2)
        nc = ctypes.c_int(0)
        st = _lib.orc_solve(self._h, _p(u), _p(self._arr(rhs, 0)), tol, max_cycles, _p(hist),
                            ctypes.byref(nc))
        return st, u, hist[: nc.value + 1]

    def rho(self, u0, max_cycles=100, rtol=1e-3):
        u = np.ascontiguousarray(u0, dtype=np.float64).ravel().copy()
        hist = np.zeros(max_cycles + 1)
        rho = ctypes.c_double(0)
        nc = ctypes.c_int(0)
        _lib.orc_rho(self._h, _p(u), max_cycles, rtol, ctypes.byref(rho), _p(hist),
                     ctypes.byref(nc))
        return float(rho.value), hist[: nc.value]

    # -- the discrete system Eq. (discr) ---------------------------------------------
    def assemble(self, l: int = 0):
        import scipy.sparse as sp
        nr = ctypes.c_int64(0)
        nz = ctypes.c_int64(0)
        _lib.orc_assemble(self._h, l, ctypes.byref(nr), ctypes.byref(nz), None, None, None,
                          None)
        rowmap = np.zeros(nr.value, np.int64)
        indptr = np.zeros(nr.value + 1, np.int64)
        ind = np.zeros(nz.value, np.int64)
        dat = np.zeros(nz.value)
        _lib.orc_assemble(self._h, l, ctypes.byref(nr), ctypes.byref(nz), _p(rowmap),
                          _p(indptr), _p(ind), _p(dat))
        A = sp.csr_matrix((dat, ind, indptr), shape=(nr.value, nr.value))
        return A, rowmap

    def direct_solve(self, rhs, l: int = 0, dense: bool = False, refine: int = 2):
        """The unique solution of Eq. (discr): a library direct solve of the assembled
        rows (LAPACK for dense, SuperLU for sparse), followed by `refine` steps of iterative
        refinement with the same factorisation (the Neumann rows make the system's
        condition number ~1e6, so a plain FP64 factor solve is accurate to ~1e-10 only)."""
        A, rowmap = self.assemble(l)
        b = self._arr(rhs, l)[rowmap]
        if dense:
            import scipy.linalg as sla
            fac = sla.lu_factor(A.toarray())
            solve = lambda v: sla.lu_solve(fac, v)
        else:
            import scipy.sparse.linalg as spla
            fac = spla.splu(A.tocsc())
            solve = fac.solve
        x = solve(b)
        for _ in range(refine):
            x = x + solve(b - A @ x)
        u = np.zeros(self.info(l)["nn"])
        u[rowmap] = x
        return u


_Grid._fields_names = ["dim", "n", "lo", "hi", "n_coarse", "nu1", "nu2", "gamma", "lam",
                       "delta_h", "cD", "cN", "ordering", "split", "smoother"]
