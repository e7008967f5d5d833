"""Workloads run twice by tests/test_sanitizers.py: once in the test process with the regular
builds, once in a child process with builds instrumented by AddressSanitizer and
UndefinedBehaviorSanitizer (the child preloads the sanitizer runtime and names the
instrumented library in ORACLE_LIB or IBM_LIB).  Each writes its results to an .npz file;
the test compares the two.  No GPU: the library part calls only host entry points.

    python tests/sanitize_child.py oracle|library OUT.npz
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def oracle_case():
    """Every entry point of the C oracle on small workloads: a multi-body grid (classification,
    stencils, operator, sweeps, levels, all three solvers, projection), the three constructed
    edge workloads (degenerate, on-surface and vertex-ray branches), a moved body's fresh
    cells, a mesh with an odd column and the STREAM triad."""
    from oracle import OracleProblem
    from oracle.fresh import FreshOracle
    from oracle.momentum import srj_schedule
    from oracle.oracle import stream_triad_gbs, threads
    from paper_2505_17287_amd import inputs as I

    out = {}
    wl = I.multibody(32, n_bodies=2, level=3)
    P = OracleProblem.from_workload(wl)
    out["types"] = P.types()
    g = P.ghosts()
    for k, v in g.items():
        out["ghost_" + k] = v
    rng = np.random.default_rng(3)
    p = rng.standard_normal(P.shape)
    f = rng.standard_normal(P.shape)
    out["apply"] = P.apply_S(p)
    out["sweep"] = P.sweep(p, f, lam=0.1, nsweeps=2)
    out["refresh"] = P.ghost_refresh(p)
    out["levels"] = np.array([lv["dims"] for lv in P.levels()])
    for l in range(1, len(P.levels())):
        act, T = P.level_arrays(l)
        out["level%d_act" % l] = act
        out["level%d_T" % l] = np.stack(T)
    bi, tri = P.closest_point(np.array([0.05, -0.1, 0.2]))
    out["closest"] = np.append(bi, tri)
    u, v, w = wl.velocity()
    rhs = P.rhs(u, v, w)
    out["rhs"] = rhs
    for method, kw in (("vcycle", dict(fixed_cycles=3)), ("bicgstab", dict(rel_tol=1e-9)),
                       ("bicgstab_srj", dict(fixed_cycles=4, srj_omega=srj_schedule(0.99, 4)))):
        ps, st = P.solve(rhs, method=method, **kw)
        out["solve_" + method] = ps
        out["cycles_" + method] = np.array([st.cycles])
    u1, v1, w1, pp, st, _ = P.project(u, v, w, dt=0.5, rel_tol=1e-9, method="bicgstab")
    for k, a in (("u", u1), ("v", v1), ("w", w1), ("p", pp)):
        out["project_" + k] = a
    out["div"] = np.array([P.div_max(u1, v1, w1)])
    P.set_neumann(np.linspace(0.0, 1.0, len(g["cell"])))
    out["neumann_solve"] = P.solve(rhs, fixed_cycles=2)[0]
    for name in sorted(I.EDGE_CASES):
        E = OracleProblem.from_workload(I.EDGE_CASES[name](32))
        out["edge_%s_types" % name] = E.types()
        out["edge_%s_flags" % name] = E.ghosts()["flags"]
        out["edge_%s_beta" % name] = E.ghosts()["beta"]
    # a moved body: fresh cells with intercepts, weights and the fill
    h = float(np.min(np.diff(wl.xf)))
    P1 = OracleProblem(wl.xf, wl.yf, wl.zf)
    P1.set_mesh(wl.verts + np.array([0.6 * h, -0.3 * h, 0.2 * h]), wl.tris)
    P1.classify()
    P1.build_stencils()
    U0, _ = wl.cell_fields()
    F = FreshOracle(P.types(), P1)
    out["fresh"] = F.fill(np.array(U0, copy=True))
    # one triangle flipped: the columns it crosses have an odd number of crossings
    bad = np.ascontiguousarray(wl.tris, dtype=np.int32).copy()
    bad[5] = bad[5][::-1]
    B = OracleProblem(wl.xf, wl.yf, wl.zf)
    try:
        B.set_mesh(wl.verts, bad)
        out["bad_mesh"] = np.array([0])
    except Exception as e:  # the closedness check refuses it
        out["bad_mesh"] = np.array([getattr(e, "code", -99)])
    out["triad_positive"] = np.array([stream_triad_gbs(1 << 20, 1) > 0.0 and threads() >= 1])
    return out


def library_case():
    """The library's host entry points (no device work): grid creation with its argument
    checks and level planning, workspace sizes from the handle-free bound and from a handle,
    the level query, the SRJ schedule, the no-allocation entry point's host checks, state
    errors before a workspace is bound, options and error strings."""
    import ctypes as C

    from paper_2505_17287_amd import ibm
    from paper_2505_17287_amd import inputs as I

    L = ibm.lib()
    out = {}

    def create(nx, ny, nz, xf=None, yf=None, zf=None):
        xf = np.linspace(0, 1, nx + 1) if xf is None else xf
        yf = np.linspace(0, 1, ny + 1) if yf is None else yf
        zf = np.linspace(0, 1, nz + 1) if zf is None else zf
        h = C.c_void_p()
        code = L.ibm_create_grid(nx, ny, nz, ibm._dp(np.ascontiguousarray(xf, float)),
                                 ibm._dp(np.ascontiguousarray(yf, float)), ibm._dp(np.ascontiguousarray(zf, float)),
                                 C.byref(h))
        return code, h

    grids = [("wing", I.wing(64, 32, 32)), ("multi", I.multibody(48, n_bodies=1, level=1)),
             ("cyl", I.cylinder2d(64))]
    shapes = [(s, wl.shape, wl.xf, wl.yf, wl.zf) for s, wl in grids]
    shapes += [("odd", (7, 9, 5), None, None, None), ("flat", (16, 16, 1), None, None, None),
               ("big", (512, 256, 256), None, None, None), ("tiny", (2, 2, 1), None, None, None)]
    for name, (nx, ny, nz), xf, yf, zf in shapes:
        code, h = create(nx, ny, nz, xf, yf, zf)
        assert code == ibm.IBM_OK, name
        n = C.c_int()
        dims = np.zeros(96, np.int32)
        assert L.ibm_get_levels(h, C.byref(n), C.c_void_p(dims.ctypes.data)) == 0
        out["levels_" + name] = dims[:3 * n.value].copy()
        sizes = []
        for prec in (ibm.IBM_FP64, ibm.IBM_MIXED):
            for caps in ((3, 1, 0), (1000, 2000, 5000), (1 << 20, 1 << 21, 1 << 22)):
                sizes.append(L.ibm_grid_workspace_bytes(h, *caps, prec))
                sizes.append(L.ibm_workspace_bytes(nx, ny, nz, *caps, prec))
        out["ws_" + name] = np.array(sizes, dtype=np.uint64)
        # state and argument errors before a workspace is bound
        v = np.zeros(9)
        t = np.zeros(3, np.int32)
        st = [L.ibm_set_geometry(h, ibm._dp(v), 3, C.c_void_p(t.ctypes.data), 1, None),
              L.ibm_classify(h, None, None), L.ibm_set_profiling(h, -1), L.ibm_set_profiling(h, 0)]
        out["state_" + name] = np.array(st)
        L.ibm_destroy_grid(h)
    bad = np.linspace(0, 1, 9)
    bad[3] = bad[2]
    nan = np.linspace(0, 1, 9)
    nan[5] = np.nan
    out["create_errors"] = np.array([create(1, 8, 8)[0], create(8, 8, 8, xf=bad)[0], create(8, 8, 8, zf=nan)[0],
                                     create(2048, 2048, 1024)[0]])
    out["last_error"] = np.frombuffer(L.ibm_last_error(None), dtype=np.uint8)
    for rho, m in ((0.0, 1), (0.3, 2), (0.9, 8), (0.999, 64)):
        out["srj_%g_%d" % (rho, m)] = ibm.srj_schedule(rho, m)
    srj_err = []
    for rho, m in ((1.0, 4), (-0.1, 4), (0.5, 0), (0.5, ibm.IBM_SRJ_MAX + 1)):
        try:
            ibm.srj_schedule(rho, m)
            srj_err.append(0)
        except ibm.IBMError as e:
            srj_err.append(e.code)
    out["srj_errors"] = np.array(srj_err)
    dummy = np.zeros(16)
    p = C.c_void_p(dummy.ctypes.data)
    counts = np.zeros(3, np.int64)
    cp = C.c_void_p(counts.ctypes.data)
    out["noalloc"] = np.array([L.ibm_classify_noalloc(4096, 4096, 1, p, p, p, p, 3, p, 1, p, cp, None),
                               L.ibm_classify_noalloc(2048, 2048, 1024, p, p, p, p, 3, p, 1, p, cp, None),
                               L.ibm_classify_noalloc(8, 8, 8, p, p, p, p, 2, p, 1, p, cp, None),
                               L.ibm_classify_noalloc(8, 8, 8, p, p, p, None, 3, p, 1, p, cp, None),
                               L.ibm_classify_noalloc(1, 8, 8, p, p, p, p, 3, p, 1, p, cp, None)])
    o = ibm.make_opts()
    out["opts"] = np.array([o.rel_tol, o.max_cycles, o.nu1, o.nu2, o.coarsest_sweeps, o.breakdown_tol])
    L.ibm_destroy_grid(None)
    return out


if __name__ == "__main__":
    kind, path = sys.argv[1], sys.argv[2]
    res = {"oracle": oracle_case, "library": library_case}[kind]()
    np.savez(path, **res)
    print("done", kind, len(res), flush=True)
