"""C-ABI library checks that need no GPU: it loads, exports every function include/ibm.h
declares, and its host-only entry points validate their arguments."""
import ctypes as C

import numpy as np
import pytest

from paper_2505_17287_amd import ibm


def test_library_exports_every_declared_symbol():
    L = ibm.lib()
    names = ibm.declared_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def _create(nx, ny, nz, xf=None, yf=None, zf=None):
    xf = np.linspace(0, 1, nx + 1) if xf is None else xf
    yf = np.linspace(0, 1, ny + 1) if yf is None else yf
    zf = np.linspace(0, 1, nz + 1) if zf is None else zf
    h = C.c_void_p()
    code = ibm.lib().ibm_create_grid(nx, ny, nz, ibm._dp(np.ascontiguousarray(xf, float)),
                                     ibm._dp(np.ascontiguousarray(yf, float)), ibm._dp(np.ascontiguousarray(zf, float)),
                                     C.byref(h))
    return code, h


def test_create_grid_validates_arguments():
    L = ibm.lib()
    code, h = _create(8, 8, 8)
    assert code == ibm.IBM_OK and h.value
    L.ibm_destroy_grid(h)
    assert _create(1, 8, 8)[0] == ibm.IBM_E_ARG
    bad = np.linspace(0, 1, 9)
    bad[3] = bad[2]
    assert _create(8, 8, 8, xf=bad)[0] == ibm.IBM_E_ARG
    nan = np.linspace(0, 1, 9)
    nan[5] = np.nan
    assert _create(8, 8, 8, zf=nan)[0] == ibm.IBM_E_ARG
    assert b"strictly increasing" in L.ibm_last_error(None)


def test_profiling_switch_validates_its_argument():
    L = ibm.lib()
    code, h = _create(8, 8, 8)
    assert code == ibm.IBM_OK
    assert L.ibm_set_profiling(h, -1) == ibm.IBM_E_ARG
    assert L.ibm_set_profiling(h, 0) == ibm.IBM_OK  # off: no device work
    L.ibm_destroy_grid(h)


def test_workspace_bound_covers_every_plan():
    """The handle-free size is an upper bound of the exact size for stretched grids."""
    from paper_2505_17287_amd import inputs as I
    L = ibm.lib()
    for wl in (I.wing(64, 32, 32), I.multibody(48, n_bodies=1, level=1), I.cylinder2d(64)):
        nx, ny, nz = wl.shape
        code, h = _create(nx, ny, nz, wl.xf, wl.yf, wl.zf)
        assert code == 0
        for prec in (ibm.IBM_FP64, ibm.IBM_MIXED):
            exact = L.ibm_grid_workspace_bytes(h, 1000, 2000, 5000, prec)
            bound = L.ibm_workspace_bytes(nx, ny, nz, 1000, 2000, 5000, prec)
            assert 0 < exact <= bound
        L.ibm_destroy_grid(h)


def test_levels_follow_width_coarsening_rule():
    """Level plan and child maps of the library equal the oracle's (same rule, independent
    code): stretched, uniform, odd, flat and anisotropic grids."""
    from oracle import OracleProblem
    from paper_2505_17287_amd import inputs as I
    L = ibm.lib()
    grids = [I.wing(64, 32, 32), I.multibody(48, n_bodies=1, level=1), I.cylinder2d(64), I.multibody(96, n_bodies=1, level=1)]
    extra = [(np.linspace(0, 1, 34), np.linspace(0, 3, 25), np.linspace(0, 0.5, 9)),
             (np.cumsum(np.r_[0, 1.07 ** np.arange(40)]), np.linspace(0, 1, 17), np.linspace(0, 1, 6))]
    cases = [(wl.xf, wl.yf, wl.zf) for wl in grids] + extra
    for xf, yf, zf in cases:
        nx, ny, nz = len(xf) - 1, len(yf) - 1, len(zf) - 1
        code, h = _create(nx, ny, nz, xf, yf, zf)
        assert code == 0
        n = C.c_int()
        dims = np.zeros(96, np.int32)
        assert L.ibm_get_levels(h, C.byref(n), C.c_void_p(dims.ctypes.data)) == 0
        P = OracleProblem(xf, yf, zf)
        P.classify()
        ref = [lv["dims"] for lv in P.levels()]
        got = [tuple(int(x) for x in dims[3 * l:3 * l + 3]) for l in range(n.value)]
        assert got == ref
        for l in range(1, n.value):
            maps = P.level_map(l)
            for d in range(3):
                cs = np.zeros(got[l][d] + 1, np.int32)
                assert L.ibm_get_level_map(h, l, d, C.c_void_p(cs.ctypes.data)) == 0
                assert np.array_equal(cs, maps[d]), (l, d)
        assert L.ibm_get_level_map(h, 0, 0, C.c_void_p(dims.ctypes.data)) == ibm.IBM_E_ARG
        L.ibm_destroy_grid(h)


def test_options_defaults():
    o = ibm.make_opts()
    assert o.rel_tol == 1e-10 and o.max_cycles == 200 and (o.nu1, o.nu2, o.coarsest_sweeps) == (2, 2, 16)


def test_srj_schedule_host_call():
    """The library's schedule (host code, no device) equals the oracle's Chebyshev factors and
    rejects out-of-range arguments."""
    from oracle.momentum import srj_schedule as ref
    for rho, m in ((0.0, 1), (0.3, 2), (0.9, 8), (0.999, 64)):
        a = ibm.srj_schedule(rho, m)
        assert np.max(np.abs(a - ref(rho, m)) / ref(rho, m)) <= 1e-15
    for rho, m in ((1.0, 4), (-0.1, 4), (0.5, 0), (0.5, ibm.IBM_SRJ_MAX + 1)):
        with pytest.raises(ibm.IBMError):
            ibm.srj_schedule(rho, m)


def test_classify_noalloc_rejects_sizes_beyond_its_scratch():
    """Argument and size checks of the no-allocation classification run on the host before
    any device work: too many columns for the fixed scratch, too many cells, empty meshes."""
    L = ibm.lib()
    dummy = np.zeros(16)
    p = C.c_void_p(dummy.ctypes.data)
    counts = np.zeros(3, np.int64)
    cp = C.c_void_p(counts.ctypes.data)
    # 4096 x 4096 columns need 16.8M column counters: beyond the fixed scratch
    assert L.ibm_classify_noalloc(4096, 4096, 1, p, p, p, p, 3, p, 1, p, cp, None) == ibm.IBM_E_NOMEM
    assert b"scratch" in L.ibm_last_error(None)
    assert L.ibm_classify_noalloc(2048, 2048, 1024, p, p, p, p, 3, p, 1, p, cp, None) == ibm.IBM_E_ARG
    assert L.ibm_classify_noalloc(8, 8, 8, p, p, p, p, 2, p, 1, p, cp, None) == ibm.IBM_E_ARG
    assert L.ibm_classify_noalloc(8, 8, 8, p, p, p, None, 3, p, 1, p, cp, None) == ibm.IBM_E_ARG
    assert L.ibm_classify_noalloc(1, 8, 8, p, p, p, p, 3, p, 1, p, cp, None) == ibm.IBM_E_ARG
