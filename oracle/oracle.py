"""ctypes wrapper of the C oracle (oracle.c).  Test infrastructure only.

Every function mirrors one of the oracle's C entry points; the arithmetic lives in C.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB names another build of oracle.c to load instead (the sanitizer test's build)
_OVERRIDE = os.environ.get("ORACLE_LIB")
lib_path = _OVERRIDE or os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build_oracle(force: bool = False) -> str:
    """Compile oracle.c with gcc (no FMA contraction, x86-64 baseline ISA, OpenMP)."""
    if force or not os.path.exists(lib_path) or os.path.getmtime(lib_path) < os.path.getmtime(_SRC):
        tmp = lib_path + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, lib_path)
    return lib_path


def build_oracle_sanitized(out: str, src: str = _SRC) -> str:
    """Compile oracle.c (or another C file, `src`) with AddressSanitizer and
    UndefinedBehaviorSanitizer (gcc, -O1, every UB report fatal) into `out`; load it with
    ORACLE_LIB=out in a process that has gcc's libasan preloaded."""
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", out, src, "-lm"])
    return out


class OracleOpts(C.Structure):
    _fields_ = [("rel_tol", C.c_double), ("max_cycles", C.c_int), ("nu1", C.c_int), ("nu2", C.c_int),
                ("coarsest_sweeps", C.c_int), ("use_initial_guess", C.c_int), ("fixed_cycles", C.c_int),
                ("method", C.c_int), ("srj_m", C.c_int), ("srj_omega", C.POINTER(C.c_double)),
                ("breakdown_tol", C.c_double)]

    @staticmethod
    def make(rel_tol=1e-10, max_cycles=200, nu1=2, nu2=2, coarsest_sweeps=16, use_initial_guess=0,
             fixed_cycles=0, method="mg", srj_omega=None, breakdown_tol=1e-12):
        """method "bicgstab_srj" needs srj_omega (the relaxation factors of one preconditioner
        application, kept alive by the caller for the duration of the call)."""
        m = ({"mg": 0, "vcycle": 0, "bicgstab": 1, "bicgstab_srj": 2}[method] if isinstance(method, str)
             else int(method))
        o = OracleOpts(rel_tol, max_cycles, nu1, nu2, coarsest_sweeps, use_initial_guess, fixed_cycles, m)
        o.breakdown_tol = breakdown_tol
        if srj_omega is not None:
            o.srj_m = len(srj_omega)
            o.srj_omega = srj_omega.ctypes.data_as(C.POINTER(C.c_double))
        return o


class _Stats(C.Structure):
    _fields_ = [("cycles", C.c_int), ("status", C.c_int), ("rel_residual", C.c_double),
                ("ghost_residual_max", C.c_double), ("lambda_", C.c_double), ("ref_norm", C.c_double),
                ("first_norm", C.c_double), ("restarts", C.c_int)]


@dataclass
class OracleStats:
    status: int
    cycles: int
    rel_residual: float
    ghost_residual_max: float
    lam: float
    ref_norm: float
    history: np.ndarray
    restarts: int = 0


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not _OVERRIDE:
            build_oracle()
        lib = C.CDLL(lib_path)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        lib.orc_create.restype = P
        lib.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp]
        lib.orc_destroy.argtypes = [P]
        lib.orc_set_mesh.argtypes = [P, dp, C.c_int64, C.c_void_p, C.c_int64]
        lib.orc_classify.argtypes = [P, C.c_void_p]
        lib.orc_stream_triad.restype = C.c_double
        lib.orc_stream_triad.argtypes = [C.c_int64, C.c_int]
        lib.orc_threads.restype = C.c_int
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_odd_columns.restype = C.c_int64
        lib.orc_odd_columns.argtypes = [P]
        lib.orc_num_ghosts.restype = C.c_int64
        lib.orc_num_ghosts.argtypes = [P]
        lib.orc_get_types.argtypes = [P, C.c_void_p]
        lib.orc_get_ghost_cells.argtypes = [P, C.c_void_p]
        lib.orc_closest_point.restype = C.c_int64
        lib.orc_closest_point.argtypes = [P, dp, dp]
        lib.orc_build_stencils.argtypes = [P, C.c_void_p]
        lib.orc_set_neumann.argtypes = [P, C.c_void_p]
        lib.orc_get_ghosts.argtypes = [P] + [C.c_void_p] * 9
        lib.orc_apply_S.argtypes = [P, dp, dp]
        lib.orc_sweep.argtypes = [P, dp, dp, C.c_double, C.c_int, C.c_uint64, C.c_int]
        lib.orc_ghost_refresh.argtypes = [P, dp]
        lib.orc_num_levels.argtypes = [P]
        lib.orc_level_info.argtypes = [P, C.c_int, C.c_void_p, C.c_void_p, dp]
        lib.orc_level_map.argtypes = [P, C.c_int, C.c_int, C.c_void_p]
        lib.orc_level_arrays.argtypes = [P, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.orc_solve.argtypes = [P, dp, dp, C.POINTER(OracleOpts), C.POINTER(_Stats), C.c_void_p, C.c_int]
        lib.orc_rhs.argtypes = [P, dp, dp, dp, C.c_double, dp]
        lib.orc_correct.argtypes = [P, dp, dp, dp, dp, C.c_double]
        lib.orc_div_max.restype = C.c_double
        lib.orc_div_max.argtypes = [P, dp, dp, dp]
        lib.orc_get_metrics.argtypes = [P] + [dp] * 9
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _vp(a: np.ndarray | None):
    return None if a is None else C.c_void_p(a.ctypes.data)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed with status %d" % (what, code))
        self.code = code


class OracleProblem:
    """One grid (+ optional body).  Arrays are numpy, shape (nz, ny, nx) for cell fields."""

    def __init__(self, xf, yf, zf):
        self.xf = np.ascontiguousarray(xf, dtype=np.float64)
        self.yf = np.ascontiguousarray(yf, dtype=np.float64)
        self.zf = np.ascontiguousarray(zf, dtype=np.float64)
        self.nx, self.ny, self.nz = len(self.xf) - 1, len(self.yf) - 1, len(self.zf) - 1
        self._h = _L().orc_create(self.nx, self.ny, self.nz, _dp(self.xf), _dp(self.yf), _dp(self.zf))
        if not self._h:
            raise OracleError(-1, "orc_create")

    @classmethod
    def from_workload(cls, wl, classify=True, stencils=True):
        P = cls(wl.xf, wl.yf, wl.zf)
        P.set_mesh(wl.verts, wl.tris)
        if classify:
            P.classify()
            if stencils:
                P.build_stencils()
        return P

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_destroy(self._h)
            self._h = None

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def set_mesh(self, verts, tris):
        self.verts = np.ascontiguousarray(verts, dtype=np.float64)
        self.tris = np.ascontiguousarray(tris, dtype=np.int32)
        s = _L().orc_set_mesh(self._h, _dp(self.verts), len(self.verts), _vp(self.tris), len(self.tris))
        if s != 0:
            raise OracleError(s, "orc_set_mesh")

    def classify(self):
        c = np.zeros(3, dtype=np.int64)
        s = _L().orc_classify(self._h, _vp(c))
        if s != 0:
            raise OracleError(s, "orc_classify")
        return c

    def odd_columns(self):
        return int(_L().orc_odd_columns(self._h))

    def types(self):
        t = np.empty(self.shape, dtype=np.uint8)
        _L().orc_get_types(self._h, _vp(t))
        return t

    def ghost_cells(self):
        g = np.empty(_L().orc_num_ghosts(self._h), dtype=np.int32)
        _L().orc_get_ghost_cells(self._h, _vp(g))
        return g

    def closest_point(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        bi = np.empty(3)
        t = _L().orc_closest_point(self._h, _dp(x), _dp(bi))
        return bi, int(t)

    def build_stencils(self):
        n = np.zeros(1, dtype=np.int64)
        s = _L().orc_build_stencils(self._h, _vp(n))
        if s != 0:
            raise OracleError(s, "orc_build_stencils")
        return int(n[0])

    def set_neumann(self, g):
        g = np.ascontiguousarray(g, dtype=np.float64)
        s = _L().orc_set_neumann(self._h, _vp(g))
        if s != 0:
            raise OracleError(s, "orc_set_neumann")

    def ghosts(self):
        ng = int(_L().orc_num_ghosts(self._h))
        d = dict(cell=self.ghost_cells(), bi=np.empty((ng, 3)), n=np.empty((ng, 3)), ip=np.empty((ng, 3)),
                 stencil=np.empty((ng, 8), dtype=np.int32), beta=np.empty((ng, 8)), beta_g=np.empty(ng),
                 dl=np.empty(ng), h=np.empty(ng), flags=np.empty(ng, dtype=np.int32))
        _L().orc_get_ghosts(self._h, *[_vp(d[k]) for k in ("bi", "n", "ip", "stencil", "beta", "beta_g", "dl", "h", "flags")])
        return d

    def metrics(self):
        out = [np.empty(self.nx), np.empty(self.ny), np.empty(self.nz), np.empty(self.nx), np.empty(self.nx),
               np.empty(self.ny), np.empty(self.ny), np.empty(self.nz), np.empty(self.nz)]
        _L().orc_get_metrics(self._h, *[_dp(a) for a in out])
        return dict(zip(("xc", "yc", "zc", "axm", "axp", "aym", "ayp", "azm", "azp"), out))

    def apply_S(self, p):
        p = np.ascontiguousarray(p, dtype=np.float64)
        out = np.empty_like(p)
        _L().orc_apply_S(self._h, _dp(p), _dp(out))
        return out

    def sweep(self, p, f, lam=0.0, nsweeps=1, perm_seed=0, refresh=True):
        p = np.array(p, dtype=np.float64, order="C", copy=True)
        f = np.ascontiguousarray(f, dtype=np.float64)
        s = _L().orc_sweep(self._h, _dp(p), _dp(f), float(lam), int(nsweeps), int(perm_seed), int(refresh))
        if s != 0:
            raise OracleError(s, "orc_sweep")
        return p

    def ghost_refresh(self, p):
        p = np.array(p, dtype=np.float64, order="C", copy=True)
        s = _L().orc_ghost_refresh(self._h, _dp(p))
        if s != 0:
            raise OracleError(s, "orc_ghost_refresh")
        return p

    def levels(self):
        nl = _L().orc_num_levels(self._h)
        out = []
        for l in range(nl):
            dims = np.zeros(3, dtype=np.int32)
            hv = np.zeros(3, dtype=np.int32)
            va = C.c_double()
            _L().orc_level_info(self._h, l, _vp(dims), _vp(hv), C.byref(va))
            out.append(dict(dims=tuple(int(x) for x in dims), halved=tuple(int(x) for x in hv), vol_active=va.value))
        return out

    def level_map(self, l):
        """Children starts of level l >= 1 per axis: coarse index I holds the cells
        cs[I] .. cs[I+1]-1 of level l-1."""
        dims = self.levels()[l]["dims"]
        out = []
        for d in range(3):
            cs = np.zeros(dims[d] + 1, dtype=np.int32)
            _L().orc_level_map(self._h, l, d, _vp(cs))
            out.append(cs)
        return out

    def level_arrays(self, l):
        info = self.levels()[l]
        nx, ny, nz = info["dims"]
        act = np.empty((nz, ny, nx), dtype=np.uint8)
        T = [np.zeros((nz, ny, nx)) for _ in range(3)]
        _L().orc_level_arrays(self._h, l, _vp(act), *[_vp(t) for t in T])
        return act, T

    def solve(self, f, p0=None, hist_len=256, **kw):
        om = kw.get("srj_omega")
        if om is not None:
            kw["srj_omega"] = om = np.ascontiguousarray(om, dtype=np.float64)
        o = OracleOpts.make(**kw)
        f = np.ascontiguousarray(f, dtype=np.float64)
        p = np.zeros(self.shape) if p0 is None else np.array(p0, dtype=np.float64, order="C", copy=True)
        if p0 is not None:
            o.use_initial_guess = 1
        st = _Stats()
        hist = np.full(hist_len, np.nan)
        s = _L().orc_solve(self._h, _dp(f), _dp(p), C.byref(o), C.byref(st), _vp(hist), hist_len)
        if s < 0:
            raise OracleError(s, "orc_solve")
        return p, OracleStats(st.status, st.cycles, st.rel_residual, st.ghost_residual_max, st.lambda_,
                              st.ref_norm, hist[:st.cycles].copy(), st.restarts)

    def rhs(self, u, v, w, dt=1.0):
        f = np.empty(self.shape)
        _L().orc_rhs(self._h, _dp(np.ascontiguousarray(u)), _dp(np.ascontiguousarray(v)),
                     _dp(np.ascontiguousarray(w)), float(dt), _dp(f))
        return f

    def correct(self, u, v, w, p, dt=1.0):
        u, v, w = (np.array(a, dtype=np.float64, order="C", copy=True) for a in (u, v, w))
        _L().orc_correct(self._h, _dp(u), _dp(v), _dp(w), _dp(np.ascontiguousarray(p)), float(dt))
        return u, v, w

    def div_max(self, u, v, w):
        return float(_L().orc_div_max(self._h, _dp(np.ascontiguousarray(u)), _dp(np.ascontiguousarray(v)),
                                      _dp(np.ascontiguousarray(w))))

    def project(self, u, v, w, dt=1.0, **kw):
        f = self.rhs(u, v, w, dt)
        p, st = self.solve(f, **kw)
        u2, v2, w2 = self.correct(u, v, w, p, dt)
        return u2, v2, w2, p, st, f


def stream_triad_gbs(n: int = 1 << 27, reps: int = 5) -> float:
    """Host memory bandwidth (STREAM triad, GB/s) with the oracle's OpenMP threads."""
    return float(_L().orc_stream_triad(int(n), int(reps)))


def threads() -> int:
    """OpenMP threads the oracle uses."""
    return int(_L().orc_threads())


def set_threads(n: int) -> None:
    """Set the oracle's OpenMP thread count (process-wide)."""
    _L().orc_set_threads(int(n))
