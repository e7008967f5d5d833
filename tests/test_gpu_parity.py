"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element by element.

Discrete outputs (cell types, ghost lists, stencil member indices, flags) must be equal;
intercepts, normals and weights agree to 1e-12; the smoother and the operator agree bit for
bit when given the same inputs; solves agree to 1e-9 max-relative (FP64, same cycle count
and converged) and 1e-8 (mixed precision against a tightly converged oracle).
"""
import numpy as np
import pytest

from oracle import OracleProblem
from paper_2505_17287_amd import inputs as I

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _setup(wl, precision="fp64"):
    from paper_2505_17287_amd import ibm
    print("case", wl.name, wl.shape, flush=True)
    g = ibm.Grid(wl.xf, wl.yf, wl.zf, precision=precision)
    counts = g.setup(wl.verts, wl.tris)
    return g, counts


CASES = {
    "cylinder2d": lambda: I.cylinder2d(128),
    "wing_small": lambda: I.wing(96, 48, 48),
    "spheres48": lambda: I.multibody(48, n_bodies=3, level=3),
    "spheres_ragged": lambda: I.multibody(88, n_bodies=2, level=3),
    "wing_odd": lambda: I.wing(75, 42, 40),  # odd nx: unpaired column path of the smoother
}

_cache = {}


def _pair(name):
    if name not in _cache:
        wl = CASES[name]()
        P = OracleProblem.from_workload(wl)
        g, counts = _setup(wl)
        _cache[name] = (wl, P, g, counts)
    return _cache[name]


@pytest.mark.parametrize("name", sorted(CASES))
def test_classification_equal(name):
    _torch()
    wl, P, g, counts = _pair(name)
    t_ref = P.types()
    t_gpu = g.cell_types().cpu().numpy()
    assert np.array_equal(t_gpu, t_ref)
    assert tuple(counts) == tuple(int((t_ref == k).sum()) for k in range(3))


@pytest.mark.parametrize("name", sorted(CASES))
def test_ghost_stencils_match(name):
    _torch()
    wl, P, g, counts = _pair(name)
    ref = P.ghosts()
    got = g.ghosts()
    assert np.array_equal(got["cell"], ref["cell"])
    assert np.array_equal(got["flags"], ref["flags"])
    assert np.max(np.abs(got["bi"] - ref["bi"]), initial=0.0) <= 1e-12
    assert np.max(np.abs(got["n"] - ref["n"]), initial=0.0) <= 1e-12
    assert np.max(np.abs(got["ip"] - ref["ip"]), initial=0.0) <= 1e-12
    assert np.array_equal(got["stencil"], ref["stencil"])
    assert np.max(np.abs(got["beta"] - ref["beta"]), initial=0.0) <= 1e-12 * max(1.0, np.abs(ref["beta"]).max())


@pytest.mark.parametrize("name", sorted(CASES))
def test_operator_and_sweep_bitwise(name):
    torch = _torch()
    wl, P, g, counts = _pair(name)
    rng = np.random.default_rng(21)
    t = P.types()
    p0 = np.where(t == 2, 0.0, rng.standard_normal(P.shape))
    f = np.where(t == 0, rng.standard_normal(P.shape), 0.0)
    pd = torch.from_numpy(p0).cuda()
    fd = torch.from_numpy(f).cuda()
    Sg = g.debug_apply(pd).cpu().numpy()
    assert np.array_equal(Sg, P.apply_S(p0))
    for n in (1, 3):
        out = g.debug_sweep(pd.clone(), fd, lam=0.37, n=n, refresh=False).cpu().numpy()
        ref = P.sweep(p0, f, lam=0.37, nsweeps=n, refresh=False)
        assert np.array_equal(out, ref), np.max(np.abs(out - ref))
    # with ghost refresh the weights come from different (equivalent) formulas
    out = g.debug_sweep(pd.clone(), fd, lam=0.0, n=2, refresh=True).cpu().numpy()
    ref = P.sweep(p0, f, lam=0.0, nsweeps=2, refresh=True)
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


def _rel(a, b, mask):
    a = a - a[mask].mean()
    b = b - b[mask].mean()
    return np.max(np.abs(a[mask] - b[mask])) / np.max(np.abs(b[mask]))


@pytest.mark.parametrize("method", ["vcycle", "bicgstab"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_solve_fixed_cycles(name, method):
    """Same outer iteration, same number of steps: the iterates agree to rounding."""
    torch = _torch()
    wl, P, g, counts = _pair(name)
    u, v, w = wl.velocity()
    f = P.rhs(u, v, w)
    fd = torch.from_numpy(f).cuda()
    act = P.types() != 2
    for ncyc in (1, 3):
        pr, sr = P.solve(f, fixed_cycles=ncyc, method=method)
        pg, sg = g.poisson_solve(fd, fixed_cycles=ncyc, method=method)
        assert sg.cycles == ncyc
        assert _rel(pg.cpu().numpy(), pr, act) <= 1e-9


@pytest.mark.parametrize("method", ["vcycle", "bicgstab"])
@pytest.mark.parametrize("name", ["cylinder2d", "wing_small", "spheres48"])
def test_solve_converged(name, method):
    """Converged to 1e-12 both sides: the discrete solution and lambda agree to 1e-9."""
    torch = _torch()
    wl, P, g, counts = _pair(name)
    u, v, w = wl.velocity()
    f = P.rhs(u, v, w)
    fd = torch.from_numpy(f).cuda()
    act = P.types() != 2
    pr, sr = P.solve(f, rel_tol=1e-12, method="vcycle", max_cycles=400)
    pg, sg = g.poisson_solve(fd, rel_tol=1e-12, method=method, max_cycles=400)
    assert sg.status == 0 and sr.status == 0
    assert sg.rel_residual <= 1e-12
    assert _rel(pg.cpu().numpy(), pr, act) <= 1e-9
    assert abs(sg.lam - sr.lam) <= 1e-9 * max(abs(sr.lam), np.abs(f).max() * 1e-6)
    # at the default tolerance the stop decision agrees within one step
    pr2, sr2 = P.solve(f, rel_tol=1e-10, method=method)
    pg2, sg2 = g.poisson_solve(fd, rel_tol=1e-10, method=method)
    assert abs(sg2.cycles - sr2.cycles) <= 1


def _srj_omega(m=16):
    from oracle.momentum import srj_schedule
    return srj_schedule(max(0.0, np.cos(np.pi / m)), m)


@pytest.mark.parametrize("name", sorted(CASES))
def test_srj_preconditioned_fixed_cycles(name):
    """The paper's configuration (BiCGStab + scheduled relaxed Jacobi): same schedule, same
    number of steps, iterates agree to rounding."""
    torch = _torch()
    wl, P, g, counts = _pair(name)
    u, v, w = wl.velocity()
    f = P.rhs(u, v, w)
    fd = torch.from_numpy(f).cuda()
    act = P.types() != 2
    for ncyc in (1, 4):
        pr, sr = P.solve(f, fixed_cycles=ncyc, method="bicgstab_srj", srj_omega=_srj_omega(16))
        pg, sg = g.poisson_solve(fd, fixed_cycles=ncyc, method="bicgstab_srj", srj_sweeps=16)
        assert sg.cycles == ncyc
        assert _rel(pg.cpu().numpy(), pr, act) <= 1e-9


@pytest.mark.parametrize("name", ["cylinder2d", "spheres48"])
def test_srj_preconditioned_converged(name):
    """Converged to 1e-12: the same discrete solution as the multigrid-preconditioned solve."""
    torch = _torch()
    wl, P, g, counts = _pair(name)
    u, v, w = wl.velocity()
    f = P.rhs(u, v, w)
    fd = torch.from_numpy(f).cuda()
    act = P.types() != 2
    pr, sr = P.solve(f, rel_tol=1e-12, method="vcycle", max_cycles=400)
    pg, sg = g.poisson_solve(fd, rel_tol=1e-12, method="bicgstab_srj", srj_sweeps=16, max_cycles=3000)
    assert sg.status == 0 and sg.rel_residual <= 1e-12
    assert _rel(pg.cpu().numpy(), pr, act) <= 1e-9
    assert abs(sg.lam - sr.lam) <= 1e-9 * max(abs(sr.lam), np.abs(f).max() * 1e-6)
    print(name, "SRJ-BiCGStab steps", sg.cycles, flush=True)
    with pytest.raises(Exception):
        g.poisson_solve(fd, method="bicgstab_srj", srj_sweeps=0)


@pytest.mark.parametrize("name", ["wing_small", "spheres48", "cylinder2d"])
def test_projection_matches(name):
    torch = _torch()
    wl, P, g, counts = _pair(name)
    u, v, w = wl.velocity()
    ud, vd, wd = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (u, v, w))
    dt = 0.25
    pg, sg = g.project(ud, vd, wd, dt=dt, rel_tol=1e-12)
    u1, v1, w1, pr, sr, f = P.project(u, v, w, dt=dt, rel_tol=1e-12, max_cycles=400)
    for a, b in ((ud, u1), (vd, v1), (wd, w1)):
        assert np.max(np.abs(a.cpu().numpy() - b)) <= 1e-9 * np.max(np.abs(b))
    assert abs(sg.div_max - P.div_max(u1, v1, w1)) <= 1e-9 * max(1.0, sg.div_max)


_mixed = {}


@pytest.mark.parametrize("method", ["vcycle", "bicgstab"])
@pytest.mark.parametrize("name", ["wing_small", "spheres48", "cylinder2d"])
def test_mixed_precision_matches_tight_oracle(name, method):
    """FP32 V-cycles inside FP64 refinement / FP64 BiCGStab, to relative residual 1e-10:
    within 1e-8 of the oracle solved to 1e-13."""
    torch = _torch()
    if name not in _mixed:
        wl = CASES[name]()
        P = OracleProblem.from_workload(wl)
        g, _ = _setup(wl, precision="mixed")
        u, v, w = wl.velocity()
        f = P.rhs(u, v, w)
        pr, sr = P.solve(f, rel_tol=1e-13, max_cycles=400)
        _mixed[name] = (P, g, f, pr)
    P, g, f, pr = _mixed[name]
    pg, sg = g.poisson_solve(torch.from_numpy(f).cuda(), rel_tol=1e-10, precision="mixed", method=method)
    assert sg.status == 0 and sg.rel_residual <= 1e-10
    act = P.types() != 2
    err = _rel(pg.cpu().numpy(), pr, act)
    print("mixed", name, method, "steps", sg.cycles, "err", err)
    assert err <= 1e-8


def test_determinism_bitwise():
    torch = _torch()
    wl, P, g, counts = _pair("spheres48")
    u, v, w = wl.velocity()
    fd = torch.from_numpy(P.rhs(u, v, w)).cuda()
    a, _ = g.poisson_solve(fd)
    b, _ = g.poisson_solve(fd)
    assert torch.equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_determinism_bitwise_stretched(precision):
    """Run to run bitwise on a hierarchy that merges cells on part of each axis: the row-wise
    restrictions (fixed tiling, per-lane sums gathered in a fixed order, one partial per
    workgroup), the staged prolongations and the paired sweeps of odd coarse rows."""
    torch = _torch()
    from paper_2505_17287_amd import ibm
    wl = I.multibody(158, n_bodies=2, level=3)
    P = OracleProblem.from_workload(wl)
    g = ibm.Grid(wl.xf, wl.yf, wl.zf, precision=precision)
    g.setup(wl.verts, wl.tris)
    fd = torch.from_numpy(P.rhs(*wl.velocity())).cuda()
    a, sa = g.poisson_solve(fd, method="bicgstab", precision=precision)
    b, sb = g.poisson_solve(fd, method="bicgstab", precision=precision)
    assert sa.status == 0 and sa.cycles == sb.cycles
    assert torch.equal(a, b)
    g.close()


@pytest.mark.parametrize("stride", [1, 3])
def test_profiling_times_every_stride_th_sweep(stride):
    """Two fixed V(2,2) cycles run eight level-0 sweeps; profiling with a stride times the
    sweeps 0, stride, 2 stride, ... of them, each with a positive duration."""
    torch = _torch()
    wl, P, g, counts = _pair("spheres48")
    fd = torch.from_numpy(P.rhs(*wl.velocity())).cuda()
    g.set_profiling(True, stride=stride)
    g.poisson_solve(fd, fixed_cycles=2, method="vcycle")
    torch.cuda.synchronize()
    prof = g.profile()
    g.set_profiling(False)
    assert prof["n_fp64"] == (8 + stride - 1) // stride
    assert prof["ms_fp64"] > 0.0


@pytest.mark.parametrize("precision,method", [("fp64", "vcycle"), ("fp64", "bicgstab"), ("mixed", "vcycle"),
                                              ("mixed", "bicgstab"), ("fp64", "bicgstab_srj")])
def test_step_api_equals_blocking_solve(precision, method):
    """ibm_solve_begin / ibm_solve_step / ibm_solve_poll give, bit for bit, the pressure of the
    blocking ibm_poisson_solve with the same options (converged and at a fixed step count),
    with the same step count; poll reports -1 while idle between steps and never blocks."""
    import time
    torch = _torch()
    from paper_2505_17287_amd import ibm
    wl = CASES["spheres48"]()
    P = OracleProblem.from_workload(wl, stencils=False)
    g, _ = _setup(wl, precision="mixed")
    fd = torch.from_numpy(P.rhs(*wl.velocity())).cuda()
    for kw in (dict(rel_tol=1e-10), dict(fixed_cycles=3)):
        ref, st_ref = g.poisson_solve(fd, precision=precision, method=method, **kw)
        p = torch.empty_like(fd)
        g.solve_begin(fd, p, precision=precision, method=method, **kw)
        done, idle, polls = 0, 0, 0
        while done != 1:
            polls += 1
            assert polls < 200000
            done, st = g.solve_poll()
            if done == -1:
                idle += 1
                g.solve_step(1)
            elif done == 0:
                time.sleep(1e-4)
        torch.cuda.synchronize()
        assert st.status == st_ref.status and st.cycles == st_ref.cycles, (kw, st, st_ref)
        assert idle >= 1
        assert torch.equal(p, ref), (precision, method, kw)
    # all three fixed cycles enqueued by one step call (only the first is a solve's first)
    ref, st_ref = g.poisson_solve(fd, precision=precision, method=method, fixed_cycles=3)
    p = torch.empty_like(fd)
    g.solve_begin(fd, p, precision=precision, method=method, fixed_cycles=3)
    done, polls = 0, 0
    while done != 1:
        polls += 1
        assert polls < 200000
        done, st = g.solve_poll()
        if done == -1:
            g.solve_step(3)
        elif done == 0:
            time.sleep(1e-4)
    torch.cuda.synchronize()
    assert st.cycles == 3 and st_ref.cycles == 3
    assert torch.equal(p, ref), (precision, method, "one step call")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bicgstab_restart_path_matches_oracle(precision):
    """The near-breakdown restart forced from the host (breakdown_tol 0.3): at a fixed step
    count the GPU takes the same restarts as the oracle (FP64) and its iterate agrees to 1e-9;
    converged, both precisions reach the oracle's solution."""
    torch = _torch()
    wl, P, g, counts = _pair("spheres48")
    if precision == "mixed":
        g, _ = _setup(wl, precision="mixed")
    f = P.rhs(*wl.velocity())
    fd = torch.from_numpy(f).cuda()
    act = P.types() != 2
    if precision == "fp64":
        pr, sr = P.solve(f, fixed_cycles=6, method="bicgstab", breakdown_tol=0.3)
        pg, sg = g.poisson_solve(fd, fixed_cycles=6, method="bicgstab", breakdown_tol=0.3)
        assert sr.restarts >= 1 and sg.restarts == sr.restarts
        assert _rel(pg.cpu().numpy(), pr, act) <= 1e-9
    pr, sr = P.solve(f, rel_tol=1e-12, max_cycles=400, method="bicgstab")
    pg, sg = g.poisson_solve(fd, rel_tol=1e-12, max_cycles=400, method="bicgstab", precision=precision,
                             breakdown_tol=0.3)
    assert sg.status == 0 and sg.restarts >= 1
    assert _rel(pg.cpu().numpy(), pr, act) <= (1e-9 if precision == "fp64" else 1e-8)


def test_solve_stats_ghost_residual_and_setup_time():
    """ghost_residual_max is the largest ghost-equation residual of the returned pressure
    (recomputed here with the oracle's ghost equations); t_setup is the handle's last
    geometry set-up time."""
    torch = _torch()
    wl, P, g, counts = _pair("spheres48")
    fd = torch.from_numpy(P.rhs(*wl.velocity())).cuda()
    for method in ("vcycle", "bicgstab"):
        pg, sg = g.poisson_solve(fd, rel_tol=1e-10, method=method)
        p = pg.cpu().numpy()
        ref = P.ghost_refresh(p)
        gc = P.ghost_cells()
        want = np.max(np.abs(ref.ravel()[gc] - p.ravel()[gc]))
        assert abs(sg.ghost_residual_max - want) <= 1e-12 * max(1.0, np.abs(p).max())
        assert sg.ghost_residual_max <= 1e-6 * np.abs(p).max()
        assert 0.0 < sg.t_setup < 10.0


@pytest.mark.parametrize("method", ["vcycle", "bicgstab"])
def test_stretched_hierarchy_fixed_cycles(method):
    """A stretched grid whose hierarchy merges cells on part of each axis (the generic
    restriction and the staged prolongation of level 0) and whose level 1 has an odd row
    length and enough cells for the fused coarse sweep: iterates equal the oracle's at a
    fixed number of steps."""
    torch = _torch()
    from paper_2505_17287_amd import ibm
    wl = I.multibody(158, n_bodies=2, level=3)
    print("stretched hierarchy", wl.name, method, flush=True)
    P = OracleProblem.from_workload(wl)
    lv = P.levels()
    assert lv[1]["dims"][0] % 2 == 1 and np.prod(lv[1]["dims"]) >= 3 << 17
    g = ibm.Grid(wl.xf, wl.yf, wl.zf)
    g.setup(wl.verts, wl.tris)
    f = P.rhs(*wl.velocity())
    act = P.types() != 2
    fd = torch.from_numpy(f).cuda()
    for ncyc in (1, 2):
        pr, sr = P.solve(f, fixed_cycles=ncyc, method=method)
        pg, sg = g.poisson_solve(fd, fixed_cycles=ncyc, method=method)
        a = pg.cpu().numpy()
        a, b = a - a[act].mean(), pr - pr[act].mean()
        err = np.max(np.abs(a[act] - b[act])) / np.max(np.abs(b[act]))
        print(method, ncyc, "error", err, flush=True)
        assert err <= 1e-9
    g.close()


def _hierarchy_cases():
    """Grids whose level plans take the less common branches of the width-based coarsening:
    a stretched 2D grid (one z cell), the same at 1024^2 (its 586^2 level 1 takes the
    row-wise coarse restriction and the LDS-staged coarse prolongation in 2D), a tiny grid of
    odd counts below the merge limit on one axis, and a grid whose z cells are four times
    wider than x and y (z kept until the others catch up)."""
    cases = {}
    v, t = I.prism_mesh(0.5, 128, -1.0, 1.0)
    for name, n in (("cyl2d_stretched", 96), ("cyl2d_large", 1024)):
        xf = I.stretched_faces(-8.0, 8.0, -2.0, 2.0, n)
        h = float(np.min(np.diff(xf)))
        cases[name] = I.Workload(name, xf, xf.copy(), np.array([-h / 2, h / 2]), v, t, 3)
    vs, ts = I.icosphere(3)
    cases["tiny_odd"] = I.Workload("tiny_odd", np.linspace(-1, 1, 8), np.linspace(-1, 1, 6), np.linspace(-1, 1, 5),
                                   vs * 0.45 + np.array([0.05, -0.03, 0.02]), ts, 4)
    cases["coarse_z"] = I.Workload("coarse_z", np.linspace(-1, 1, 49), np.linspace(-1, 1, 49),
                                   np.linspace(-1, 1, 13), vs * 0.5, ts, 5)
    return cases


@pytest.mark.parametrize("name", ["cyl2d_stretched", "cyl2d_large", "tiny_odd", "coarse_z"])
@pytest.mark.parametrize("method", ["vcycle", "bicgstab"])
def test_hierarchy_branches_fixed_cycles(name, method):
    torch = _torch()
    from paper_2505_17287_amd import ibm
    wl = _hierarchy_cases()[name]
    print("hierarchy case", name, wl.shape, method, flush=True)
    P = OracleProblem.from_workload(wl)
    g = ibm.Grid(wl.xf, wl.yf, wl.zf)
    g.setup(wl.verts, wl.tris)
    assert np.array_equal(g.cell_types().cpu().numpy(), P.types())
    f = P.rhs(*wl.velocity())
    act = P.types() != 2
    fd = torch.from_numpy(f).cuda()
    for ncyc in (1, 3):
        pr, sr = P.solve(f, fixed_cycles=ncyc, method=method)
        pg, sg = g.poisson_solve(fd, fixed_cycles=ncyc, method=method)
        a = pg.cpu().numpy()
        a, b = a - a[act].mean(), pr - pr[act].mean()
        assert np.max(np.abs(a[act] - b[act])) <= 1e-9 * np.max(np.abs(b[act]))
    pr, sr = P.solve(f, rel_tol=1e-12, max_cycles=400, method="bicgstab")
    pg, sg = g.poisson_solve(fd, rel_tol=1e-12, max_cycles=400)
    assert sg.status == 0 and sr.status == 0
    a = pg.cpu().numpy()
    a, b = a - a[act].mean(), pr - pr[act].mean()
    assert np.max(np.abs(a[act] - b[act])) <= 1e-9 * np.max(np.abs(b[act]))
    g.close()
