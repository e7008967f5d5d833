"""Thin ctypes binding of the HIP library (include/ibm.h).  Argument marshalling only.

PyTorch provides the device memory (one workspace tensor per grid) and the streams; every
step of the method runs in the library's kernels.  Importing this module raises if the
built library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# IBM_LIB names another build of the library to load instead (the sanitized host build)
LIB_PATH = os.environ.get("IBM_LIB") or os.path.join(_HERE, "libibm.so")

IBM_OK, IBM_NOT_CONVERGED = 0, 1
IBM_E_ARG, IBM_E_STATE, IBM_E_GEOMETRY, IBM_E_NOMEM, IBM_E_DEVICE, IBM_E_NUMERIC = -1, -2, -3, -4, -5, -6
IBM_FP64, IBM_MIXED = 0, 1
_STATUS = {0: "IBM_OK", 1: "IBM_NOT_CONVERGED", -1: "IBM_E_ARG", -2: "IBM_E_STATE", -3: "IBM_E_GEOMETRY",
           -4: "IBM_E_NOMEM", -5: "IBM_E_DEVICE", -6: "IBM_E_NUMERIC"}


class SolveOpts(C.Structure):
    _fields_ = [("rel_tol", C.c_double), ("max_cycles", C.c_int), ("nu1", C.c_int), ("nu2", C.c_int),
                ("coarsest_sweeps", C.c_int), ("precision", C.c_int), ("use_initial_guess", C.c_int),
                ("fixed_cycles", C.c_int), ("method", C.c_int), ("srj_sweeps", C.c_int),
                ("breakdown_tol", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("cycles", C.c_int), ("rel_residual", C.c_double), ("ghost_residual_max", C.c_double),
                ("lambda_", C.c_double), ("div_max", C.c_double), ("t_setup", C.c_double),
                ("t_solve", C.c_double), ("t_correct", C.c_double), ("vcycles", C.c_int), ("restarts", C.c_int)]


IBM_VCYCLE, IBM_BICGSTAB, IBM_BICGSTAB_SRJ = 0, 1, 2
_METHODS = {"vcycle": IBM_VCYCLE, "bicgstab": IBM_BICGSTAB, "bicgstab_srj": IBM_BICGSTAB_SRJ}
IBM_SRJ_MAX = 256


class MomentumOpts(C.Structure):
    _fields_ = [("nu", C.c_double), ("dt", C.c_double), ("first_step", C.c_int), ("srj_factors", C.c_int),
                ("omega", C.POINTER(C.c_double)), ("rel_tol", C.c_double), ("max_cycles", C.c_int),
                ("fixed_cycles", C.c_int)]


class MomentumStats(C.Structure):
    _fields_ = [("cycles", C.c_int), ("sweeps", C.c_int), ("rel_residual", C.c_double), ("rho", C.c_double),
                ("t_step", C.c_double)]


@dataclass
class Stats:
    status: int
    cycles: int
    rel_residual: float
    lam: float
    div_max: float
    t_solve: float
    t_correct: float
    vcycles: int = 0
    ghost_residual_max: float = 0.0
    t_setup: float = 0.0
    restarts: int = 0


def _stats(code, st):
    return Stats(code, st.cycles, st.rel_residual, st.lambda_, st.div_max, st.t_solve, st.t_correct, st.vcycles,
                 st.ghost_residual_max, st.t_setup, st.restarts)


class IBMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_STATUS.get(code, str(code)), msg))
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libibm.so is not built (run `python -m paper_2505_17287_amd.build`)")
        L = C.CDLL(LIB_PATH)
        vp, i64, dp = C.c_void_p, C.c_int64, C.POINTER(C.c_double)
        L.ibm_default_opts.argtypes = [C.POINTER(SolveOpts)]
        L.ibm_create_grid.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp, C.POINTER(vp)]
        L.ibm_workspace_bytes.restype = C.c_size_t
        L.ibm_workspace_bytes.argtypes = [C.c_int, C.c_int, C.c_int, i64, i64, i64, C.c_int]
        L.ibm_grid_workspace_bytes.restype = C.c_size_t
        L.ibm_grid_workspace_bytes.argtypes = [vp, i64, i64, i64, C.c_int]
        L.ibm_bind_workspace.argtypes = [vp, vp, C.c_size_t, i64, i64, i64, C.c_int, vp]
        L.ibm_set_geometry.argtypes = [vp, dp, i64, vp, i64, vp]
        L.ibm_classify.argtypes = [vp, vp, vp]
        L.ibm_classify_noalloc.argtypes = [C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, i64, vp, i64, vp, vp, vp]
        L.ibm_build_ghost_stencils.argtypes = [vp, vp, vp]
        L.ibm_get_ghosts.argtypes = [vp, vp] + [vp] * 7
        L.ibm_set_neumann_data.argtypes = [vp, vp, vp]
        L.ibm_get_cell_types.argtypes = [vp, vp, vp]
        L.ibm_poisson_solve.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveStats), vp]
        L.ibm_project.argtypes = [vp, vp, vp, vp, C.c_double, vp, C.POINTER(SolveOpts), C.POINTER(SolveStats), vp]
        L.ibm_solve_begin.argtypes = [vp, vp, vp, C.POINTER(SolveOpts), vp]
        L.ibm_solve_step.argtypes = [vp, C.c_int]
        L.ibm_solve_poll.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(SolveStats)]
        L.ibm_get_levels.argtypes = [vp, C.POINTER(C.c_int), vp]
        L.ibm_debug_sweep.argtypes = [vp, vp, vp, C.c_double, C.c_int, C.c_int, vp]
        L.ibm_debug_apply.argtypes = [vp, vp, vp, vp]
        L.ibm_debug_poison.argtypes = [vp, C.c_int]
        L.ibm_debug_vector.argtypes = [vp, C.c_int, vp, vp]
        L.ibm_set_profiling.argtypes = [vp, C.c_int]
        L.ibm_get_profile.argtypes = [vp, vp, vp, vp, vp]
        L.ibm_set_profiling.restype = C.c_int
        L.ibm_get_profile.restype = C.c_int
        L.ibm_default_momentum_opts.argtypes = [C.POINTER(MomentumOpts)]
        L.ibm_srj_schedule.argtypes = [C.c_double, C.c_int, vp]
        L.ibm_set_dirichlet_data.argtypes = [vp, vp, vp]
        L.ibm_get_dirichlet_weights.argtypes = [vp, vp, vp, vp]
        L.ibm_momentum_step.argtypes = [vp] + [vp] * 6 + [C.POINTER(MomentumOpts), C.POINTER(MomentumStats), vp]
        L.ibm_move_geometry.argtypes = [vp, dp, i64, vp, i64, vp, vp, vp]
        L.ibm_fill_fresh.argtypes = [vp, vp, vp, vp, vp, vp]
        L.ibm_cell_to_faces.argtypes = [vp] * 8
        L.ibm_get_level_map.argtypes = [vp, C.c_int, C.c_int, vp]
        L.ibm_correct_cells.argtypes = [vp, vp, vp, vp, vp, C.c_double, vp]
        L.ibm_get_fresh.argtypes = [vp, vp] + [vp] * 7
        L.ibm_destroy_grid.argtypes = [vp]
        L.ibm_last_error.restype = C.c_char_p
        L.ibm_last_error.argtypes = [vp]
        for name in ("ibm_create_grid", "ibm_bind_workspace", "ibm_set_geometry", "ibm_classify",
                     "ibm_build_ghost_stencils", "ibm_get_ghosts", "ibm_set_neumann_data", "ibm_get_cell_types",
                     "ibm_poisson_solve", "ibm_project", "ibm_solve_begin", "ibm_solve_step", "ibm_solve_poll",
                     "ibm_get_levels", "ibm_debug_sweep", "ibm_debug_apply", "ibm_srj_schedule",
                     "ibm_set_dirichlet_data", "ibm_get_dirichlet_weights", "ibm_momentum_step", "ibm_debug_poison", "ibm_debug_vector",
                     "ibm_classify_noalloc",
                     "ibm_move_geometry", "ibm_fill_fresh", "ibm_get_fresh"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def declared_symbols(header=None):
    """Names of the functions declared in include/ibm.h."""
    import re
    header = header or os.path.join(os.path.dirname(_HERE), "include", "ibm.h")
    txt = open(header).read()
    return sorted(set(re.findall(r"\b(ibm_[a-z_0-9]+)\s*\(", txt)))


def make_opts(rel_tol=1e-10, max_cycles=200, nu1=2, nu2=2, coarsest_sweeps=16, precision="fp64",
              use_initial_guess=False, fixed_cycles=0, method="bicgstab", srj_sweeps=16, breakdown_tol=None):
    o = SolveOpts()
    lib().ibm_default_opts(C.byref(o))
    o.rel_tol = rel_tol
    o.max_cycles = max_cycles
    o.nu1, o.nu2, o.coarsest_sweeps = nu1, nu2, coarsest_sweeps
    o.precision = IBM_MIXED if precision in ("mixed", IBM_MIXED) else IBM_FP64
    o.use_initial_guess = int(bool(use_initial_guess))
    o.fixed_cycles = fixed_cycles
    o.method = _METHODS[method] if isinstance(method, str) else int(method)
    o.srj_sweeps = int(srj_sweeps)
    if breakdown_tol is not None:
        o.breakdown_tol = float(breakdown_tol)
    return o


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def srj_schedule(rho, m):
    """The library's relaxation factors for [1 - rho, 1 + rho] (host call, no device)."""
    out = np.zeros(m, dtype=np.float64)
    code = lib().ibm_srj_schedule(float(rho), int(m), C.c_void_p(out.ctypes.data))
    if code < 0:
        raise IBMError(code, lib().ibm_last_error(None).decode())
    return out


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _tptr(t):
    return C.c_void_p(t.data_ptr())


def estimate_max_ghosts(xf, yf, zf, verts, tris):
    """Capacity for the ghost list: four cells per finest-cell face of surface, plus slack."""
    v = np.asarray(verts, dtype=np.float64)
    t = np.asarray(tris)
    area = 0.5 * np.linalg.norm(np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]]), axis=1).sum()
    h = [np.min(np.diff(f)) for f in (xf, yf, zf)]
    if len(zf) == 2:  # one cell thick: count per unit of the z extent inside the cell
        hmin = min(h[0], h[1])
        est = 4.0 * area * (h[2] / 2.0) / (hmin * hmin)
    else:
        hmin = min(h)
        est = 4.0 * area / (hmin * hmin)
    n = (len(xf) - 1) * (len(yf) - 1) * (len(zf) - 1)
    return int(min(n, est + 4096))


class Grid:
    """One problem: grid + body + workspace (a torch uint8 tensor on the device)."""

    def __init__(self, xf, yf, zf, precision="fp64", device="cuda:0", stream=None, poison=False):
        """poison: every floating-point sub-buffer of each workspace bound to this grid starts
        as NaN (ibm_debug_poison), a read-before-write check."""
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.xf = np.ascontiguousarray(xf, dtype=np.float64)
        self.yf = np.ascontiguousarray(yf, dtype=np.float64)
        self.zf = np.ascontiguousarray(zf, dtype=np.float64)
        self.nx, self.ny, self.nz = len(self.xf) - 1, len(self.yf) - 1, len(self.zf) - 1
        self.prec = IBM_MIXED if precision in ("mixed", IBM_MIXED) else IBM_FP64
        self.stream = stream
        h = C.c_void_p()
        self._check(lib().ibm_create_grid(self.nx, self.ny, self.nz, _dp(self.xf), _dp(self.yf), _dp(self.zf),
                                          C.byref(h)), None)
        self._h = h
        if poison:
            self._check(lib().ibm_debug_poison(h, 1))
        self.ws = None
        self.ng = 0
        self.nfresh = 0

    # -- helpers -------------------------------------------------------------------------
    def _check(self, code, h=True):
        if code < 0:
            msg = lib().ibm_last_error(self._h if h else None)
            raise IBMError(code, msg.decode() if msg else "")
        return code

    def _s(self):
        return _stream_ptr(self.stream)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def close(self):
        if getattr(self, "_h", None):
            lib().ibm_destroy_grid(self._h)
            self._h = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup ---------------------------------------------------------------------------
    def workspace_bytes(self, nv_max, nt_max, max_ghosts):
        return int(lib().ibm_grid_workspace_bytes(self._h, nv_max, nt_max, max_ghosts, self.prec))

    def bind(self, nv_max, nt_max, max_ghosts):
        torch = self.torch
        nbytes = self.workspace_bytes(nv_max, nt_max, max_ghosts)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        self.ws = ws
        self._ws_ptr = ws.data_ptr() + off
        self._caps = (nv_max, nt_max, max_ghosts)
        with torch.cuda.device(self.device):
            self._check(lib().ibm_bind_workspace(self._h, C.c_void_p(self._ws_ptr), nbytes, nv_max, nt_max, max_ghosts,
                                                 self.prec, self._s()))
        return nbytes

    def set_geometry(self, verts, tris, max_ghosts=None):
        self.verts = np.ascontiguousarray(verts, dtype=np.float64)
        self.tris = np.ascontiguousarray(tris, dtype=np.int32)
        nv, nt = len(self.verts), len(self.tris)
        if max_ghosts is None:
            max_ghosts = estimate_max_ghosts(self.xf, self.yf, self.zf, self.verts, self.tris)
        if self.ws is None or self._caps[0] < nv or self._caps[1] < nt or self._caps[2] < max_ghosts:
            self.bind(nv, nt, max_ghosts)
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_set_geometry(self._h, _dp(self.verts), nv, C.c_void_p(self.tris.ctypes.data), nt,
                                               self._s()))

    def classify(self):
        counts = np.zeros(3, dtype=np.int64)
        with self.torch.cuda.device(self.device):
            code = lib().ibm_classify(self._h, self._s(), C.c_void_p(counts.ctypes.data))
            if code == IBM_E_NOMEM and counts[1] > self._caps[2]:
                # more ghost cells than estimated: rebind with the exact count and redo
                self.bind(self._caps[0], self._caps[1], int(counts[1]) + 1024)
                self._check(lib().ibm_set_geometry(self._h, _dp(self.verts), len(self.verts),
                                                   C.c_void_p(self.tris.ctypes.data), len(self.tris), self._s()))
                code = lib().ibm_classify(self._h, self._s(), C.c_void_p(counts.ctypes.data))
            self._check(code)
        return counts

    def build_ghost_stencils(self):
        n = np.zeros(1, dtype=np.int64)
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_build_ghost_stencils(self._h, self._s(), C.c_void_p(n.ctypes.data)))
        self.ng = int(n[0])
        return self.ng

    def setup(self, verts, tris):
        self.set_geometry(verts, tris)
        counts = self.classify()
        self.build_ghost_stencils()
        return counts

    def ghosts(self):
        ng = self.ng
        d = dict(cell=np.empty(ng, np.int32), bi=np.empty((ng, 3)), n=np.empty((ng, 3)), ip=np.empty((ng, 3)),
                 stencil=np.empty((ng, 8), np.int32), beta=np.empty((ng, 8)), flags=np.empty(ng, np.int32))
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_get_ghosts(self._h, self._s(), *[C.c_void_p(d[k].ctypes.data) for k in
                                                                    ("cell", "bi", "n", "ip", "stencil", "beta", "flags")]))
        return d

    def set_neumann_data(self, dpdn=None):
        arr = None if dpdn is None else np.ascontiguousarray(dpdn, dtype=np.float64)
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_set_neumann_data(self._h, None if arr is None else C.c_void_p(arr.ctypes.data),
                                                   self._s()))

    def cell_types(self):
        t = self.torch.empty(self.shape, dtype=self.torch.uint8, device=self.device)
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_get_cell_types(self._h, _tptr(t), self._s()))
        return t

    def levels(self):
        n = C.c_int()
        dims = np.zeros(3 * 32, dtype=np.int32)
        self._check(lib().ibm_get_levels(self._h, C.byref(n), C.c_void_p(dims.ctypes.data)))
        return [tuple(int(x) for x in dims[3 * l:3 * l + 3]) for l in range(n.value)]

    # -- solve ---------------------------------------------------------------------------
    def _field(self, a, name):
        torch = self.torch
        if not (isinstance(a, torch.Tensor) and a.dtype == torch.float64 and a.is_contiguous()
                and a.device == self.device):
            raise TypeError("%s must be a contiguous float64 tensor on %s" % (name, self.device))
        return a

    def poisson_solve(self, rhs, p=None, **kw):
        torch = self.torch
        self._field(rhs, "rhs")
        if tuple(rhs.shape) != self.shape:
            raise ValueError("rhs shape %s != %s" % (tuple(rhs.shape), self.shape))
        if p is None:
            p = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._field(p, "p")
        o = make_opts(**kw)
        st = SolveStats()
        with torch.cuda.device(self.device):
            code = self._check(lib().ibm_poisson_solve(self._h, _tptr(rhs), _tptr(p), C.byref(o), C.byref(st),
                                                       self._s()))
        return p, _stats(code, st)

    def project(self, u, v, w, dt=1.0, p=None, **kw):
        torch = self.torch
        for a, nm, shp in ((u, "u", (self.nz, self.ny, self.nx + 1)), (v, "v", (self.nz, self.ny + 1, self.nx)),
                           (w, "w", (self.nz + 1, self.ny, self.nx))):
            self._field(a, nm)
            if tuple(a.shape) != shp:
                raise ValueError("%s shape %s != %s" % (nm, tuple(a.shape), shp))
        if p is None:
            p = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._field(p, "p")
        o = make_opts(**kw)
        st = SolveStats()
        with torch.cuda.device(self.device):
            code = self._check(lib().ibm_project(self._h, _tptr(u), _tptr(v), _tptr(w), float(dt), _tptr(p), C.byref(o),
                                                 C.byref(st), self._s()))
        return p, _stats(code, st)

    # non-blocking step API (serving)
    def solve_begin(self, rhs, p, **kw):
        self._field(rhs, "rhs")
        self._field(p, "p")
        self._opts = make_opts(**kw)
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_solve_begin(self._h, _tptr(rhs), _tptr(p), C.byref(self._opts), self._s()))

    def solve_step(self, n=1):
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_solve_step(self._h, n))

    def solve_poll(self):
        done = C.c_int()
        st = SolveStats()
        code = self._check(lib().ibm_solve_poll(self._h, C.byref(done), C.byref(st)))
        return done.value, _stats(code, st)

    # advection-diffusion half-step
    def set_dirichlet_data(self, ubi=None):
        arr = None if ubi is None else np.ascontiguousarray(ubi, dtype=np.float64).reshape(-1)
        if arr is not None and arr.size != 3 * self.ng:
            raise ValueError("need 3 values per ghost")
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_set_dirichlet_data(self._h, None if arr is None else C.c_void_p(arr.ctypes.data),
                                                     self._s()))

    def dirichlet_weights(self):
        beta = np.empty((self.ng, 8))
        beta_g = np.empty(self.ng)
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_get_dirichlet_weights(self._h, self._s(), C.c_void_p(beta.ctypes.data),
                                                        C.c_void_p(beta_g.ctypes.data)))
        return beta, beta_g

    def momentum_step(self, U, H, nu, dt, first_step=False, m=8, omega=None, rel_tol=1e-10, max_cycles=200,
                      fixed_cycles=0):
        """U: (3, nz, ny, nx) float64 device tensor, in u^n, out u*; H: same shape, in H^{n-1},
        out H^n.  Returns (status, MomentumStats)."""
        for a, nm in ((U, "U"), (H, "H")):
            self._field(a, nm)
            if tuple(a.shape) != (3,) + self.shape:
                raise ValueError("%s shape %s != %s" % (nm, tuple(a.shape), (3,) + self.shape))
        o = MomentumOpts()
        lib().ibm_default_momentum_opts(C.byref(o))
        o.nu, o.dt, o.first_step, o.srj_factors = float(nu), float(dt), int(bool(first_step)), int(m)
        om = None
        if omega is not None:
            om = np.ascontiguousarray(omega, dtype=np.float64)
            if om.size != m:
                raise ValueError("omega must hold m factors")
            o.omega = _dp(om)
        o.rel_tol, o.max_cycles, o.fixed_cycles = float(rel_tol), int(max_cycles), int(fixed_cycles)
        st = MomentumStats()
        with self.torch.cuda.device(self.device):
            code = self._check(lib().ibm_momentum_step(self._h, _tptr(U[0]), _tptr(U[1]), _tptr(U[2]), _tptr(H[0]),
                                                       _tptr(H[1]), _tptr(H[2]), C.byref(o), C.byref(st), self._s()))
        return code, st

    # fractional step: momentum half-step, then projection
    def face_shapes(self):
        nz, ny, nx = self.shape
        return (nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)

    def cell_to_faces(self, U, faces=None):
        """Face-normal velocities (uf, vf, wf) from the cell-centred U (3, nz, ny, nx)."""
        self._field(U, "U")
        if faces is None:
            faces = tuple(self.torch.empty(sh, dtype=self.torch.float64, device=self.device) for sh in self.face_shapes())
        for a, nm in zip(faces, ("uf", "vf", "wf")):
            self._field(a, nm)
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_cell_to_faces(self._h, _tptr(U[0]), _tptr(U[1]), _tptr(U[2]), *(_tptr(a) for a in faces),
                                                self._s()))
        return faces

    def correct_cells(self, U, p, dt):
        """u_c -= mean of its two face corrections, on fluid cells (in place)."""
        self._field(U, "U")
        self._field(p, "p")
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_correct_cells(self._h, _tptr(U[0]), _tptr(U[1]), _tptr(U[2]), _tptr(p), float(dt),
                                                self._s()))
        return U

    def fractional_step(self, U, H, nu, dt, p=None, first_step=False, m=8, mom_rel_tol=1e-10, **project_kw):
        """One fractional step on the device: advection-diffusion half-step of the cell-centred
        U (in u^n, out u^{n+1}) and H (in H^{n-1}, out H^n), face interpolation of u*, the
        projection of the faces and the cell-centred correction.  Returns (faces, p,
        momentum stats, projection stats); the faces hold the projected U^{n+1}."""
        code, mst = self.momentum_step(U, H, nu, dt, first_step=first_step, m=m, rel_tol=mom_rel_tol)
        faces = self.cell_to_faces(U)
        p, pst = self.project(*faces, dt=dt, p=p, **project_kw)
        self.correct_cells(U, p, dt)
        return faces, p, mst, pst

    # moving bodies
    def move_geometry(self, verts, tris):
        """New vertex positions (same or new triangles): re-classify, rebuild the stencils and
        list the fresh cells.  Returns (counts, n_fresh)."""
        self.verts = np.ascontiguousarray(verts, dtype=np.float64)
        self.tris = np.ascontiguousarray(tris, dtype=np.int32)
        counts = np.zeros(3, dtype=np.int64)
        nf = np.zeros(1, dtype=np.int64)
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_move_geometry(self._h, _dp(self.verts), len(self.verts),
                                                C.c_void_p(self.tris.ctypes.data), len(self.tris), self._s(),
                                                C.c_void_p(counts.ctypes.data), C.c_void_p(nf.ctypes.data)))
        self.nfresh = int(nf[0])
        self.ng = int(counts[1])
        return counts, self.nfresh

    def fresh(self):
        n = self.nfresh
        d = dict(cell=np.empty(n, np.int32), bi=np.empty((n, 3)), ip=np.empty((n, 3)),
                 stencil=np.empty((n, 8), np.int32), beta=np.empty((n, 8)), beta_c=np.empty(n),
                 flags=np.empty(n, np.int32))
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_get_fresh(self._h, self._s(), *[C.c_void_p(d[k].ctypes.data) for k in
                                                                   ("cell", "bi", "ip", "stencil", "beta", "beta_c",
                                                                    "flags")]))
        return d

    def fill_fresh(self, U, ubi=None):
        """U: (3, nz, ny, nx) float64 device tensor, fresh cells set in place."""
        self._field(U, "U")
        arr = None if ubi is None else np.ascontiguousarray(ubi, dtype=np.float64).reshape(-1)
        if arr is not None and arr.size != 3 * self.nfresh:
            raise ValueError("need 3 values per fresh cell")
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_fill_fresh(self._h, _tptr(U[0]), _tptr(U[1]), _tptr(U[2]),
                                             None if arr is None else C.c_void_p(arr.ctypes.data), self._s()))
        return U

    # smoother timing
    def set_profiling(self, on=True, stride=1):
        """on: time fine-level sweeps; stride: time every stride-th one (see ibm.h)."""
        if stride < 1:
            raise ValueError("stride must be >= 1")
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_set_profiling(self._h, int(stride) if on else 0))

    def profile(self):
        vals = np.zeros(2, dtype=np.float64)
        cnts = np.zeros(2, dtype=np.int64)
        self._check(lib().ibm_get_profile(self._h, C.c_void_p(vals.ctypes.data), C.c_void_p(cnts.ctypes.data),
                                          C.c_void_p(vals.ctypes.data + 8), C.c_void_p(cnts.ctypes.data + 8)))
        return dict(ms_fp64=float(vals[0]), n_fp64=int(cnts[0]), ms_fp32=float(vals[1]), n_fp32=int(cnts[1]))

    # kernel-level hooks
    def debug_sweep(self, p, rhs, lam=0.0, n=1, refresh=False):
        self._field(p, "p")
        self._field(rhs, "rhs")
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_debug_sweep(self._h, _tptr(p), _tptr(rhs), float(lam), int(n), int(refresh),
                                              self._s()))
        return p

    def debug_vector(self, which):
        """Device copy of an internal FP64 cell field (see ibm_debug_vector)."""
        out = self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device)
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_debug_vector(self._h, int(which), _tptr(out), self._s()))
            self.torch.cuda.current_stream(self.device).synchronize() if self.stream is None else self.stream.synchronize()
        return out

    def debug_apply(self, p):
        out = self.torch.empty_like(p)
        with self.torch.cuda.device(self.device):
            self._check(lib().ibm_debug_apply(self._h, _tptr(self._field(p, "p")), _tptr(out), self._s()))
        return out


def grid_from_workload(wl, precision="fp64", device="cuda:0", stream=None):
    g = Grid(wl.xf, wl.yf, wl.zf, precision=precision, device=device, stream=stream)
    counts = g.setup(wl.verts, wl.tris)
    return g, counts


def upload_velocity(wl, device="cuda:0"):
    import torch
    return tuple(torch.from_numpy(np.ascontiguousarray(a)).to(device) for a in wl.velocity())
