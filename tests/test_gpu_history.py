"""A grid handle reused across geometries gives, bit for bit, what a fresh handle gives.

The serving loop keeps one handle per grid and slot and runs request after request on it,
each with its own body.  Every result must therefore be a function of the request alone.
The control is a fresh handle whose workspace starts with NaN in every floating-point
sub-buffer (ibm_debug_poison): a value the library reads before writing it would show up
there as NaN or as a difference in the bits.  Each geometry runs the same sequence of
calls on both handles (projection FP64 and mixed with BiCGStab, fixed-cycle V-cycle solves
in both precisions, a converged V-cycle solve, BiCGStab with the scheduled-Jacobi
preconditioner, an advection-diffusion half-step, a small move of the body with its fresh
cells), and every output is compared exactly: cell types, ghost data, pressures, corrected
velocities, statistics.  The reused handle
also changes mesh size between geometries, so its workspace is rebound on the way.
"""
import numpy as np
import pytest

from paper_2505_17287_amd import inputs as I

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _requests(n, count, trace_seed=5):
    """The first `count` requests of the seeded serving stream on the n^3 grid."""
    out, r = [], 0
    while len(out) < count:
        wl = I.serving_request(r, trace_seed=trace_seed, sizes=(64, 128))
        if wl.shape[0] == n:
            out.append(wl)
        r += 1
    return out


def _run(g, wl, torch):
    """Setup and the fixed sequence of solves on one handle; host copies of every output."""
    counts = g.setup(wl.verts, wl.tris)
    out = {"counts": np.asarray(counts).copy(), "types": g.cell_types().cpu().numpy()}
    gh = g.ghosts()
    for k, v in gh.items():
        out["ghost_" + k] = v
    uvw = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in wl.velocity()]
    for prec in ("fp64", "mixed"):
        u, v, w = (a.clone() for a in uvw)
        p, st = g.project(u, v, w, dt=1.0, precision=prec, method="bicgstab")
        out["proj_%s" % prec] = (p.cpu().numpy(), u.cpu().numpy(), v.cpu().numpy(), w.cpu().numpy(),
                                 st.status, st.cycles, st.rel_residual, st.lam, st.div_max)
    rng = np.random.default_rng(wl.seed % (1 << 31))
    f = torch.from_numpy(rng.uniform(-1.0, 1.0, g.shape)).cuda()
    for prec in ("fp64", "mixed"):
        p, st = g.poisson_solve(f, precision=prec, method="vcycle", fixed_cycles=3)
        out["vc_%s" % prec] = (p.cpu().numpy(), st.cycles, st.rel_residual, st.lam)
    p, st = g.poisson_solve(f, precision="fp64", method="vcycle", rel_tol=1e-9, max_cycles=300)
    out["vc_conv"] = (p.cpu().numpy(), st.status, st.cycles, st.rel_residual)
    p, st = g.poisson_solve(f, precision="fp64", method="bicgstab_srj", fixed_cycles=2)
    out["srj"] = (p.cpu().numpy(), st.cycles, st.rel_residual, st.lam)
    # advection-diffusion half-step (borrows the Krylov vectors of the workspace)
    U0, H0 = wl.cell_fields()
    U, H = torch.from_numpy(U0).cuda(), torch.from_numpy(H0).cuda()
    code, ms = g.momentum_step(U, H, 1e-3, 0.01, m=4, fixed_cycles=2)
    out["momentum"] = (U.cpu().numpy(), H.cpu().numpy(), code, ms.rel_residual)
    # a small rigid move: re-classification, fresh cells and their fill
    h = float(np.min(np.diff(wl.xf)))
    counts2, nf = g.move_geometry(wl.verts + np.array([0.31, -0.22, 0.13]) * h, wl.tris)
    out["move"] = (np.asarray(counts2).copy(), nf, g.cell_types().cpu().numpy())
    fr = g.fresh()
    for k, v in fr.items():
        out["fresh_" + k] = v
    g.fill_fresh(U)
    out["fill"] = U.cpu().numpy()
    return out


def _same(a, b, what):
    assert a.keys() == b.keys()
    for k in a:
        x, y = a[k], b[k]
        xs = x if isinstance(x, tuple) else (x,)
        ys = y if isinstance(y, tuple) else (y,)
        for q, (s, t) in enumerate(zip(xs, ys)):
            if isinstance(s, np.ndarray):
                assert s.dtype == t.dtype and s.shape == t.shape, (what, k, q)
                if s.dtype.kind == "f":
                    assert np.all(np.isfinite(s)), (what, k, q, "non-finite")
                    assert np.array_equal(s.view(np.uint8), t.view(np.uint8)), (what, k, q)
                else:
                    assert np.array_equal(s, t), (what, k, q)
            else:
                assert s == t or (s != s and t != t), (what, k, q, s, t)


@pytest.mark.parametrize("n", [64, 128])
def test_reused_handle_equals_poisoned_fresh_handle(n):
    torch = _torch()
    from paper_2505_17287_amd import ibm
    reqs = _requests(n, 4)
    print("history", n, [wl.name for wl in reqs], flush=True)
    wl0 = reqs[0]
    reused = ibm.Grid(wl0.xf, wl0.yf, wl0.zf, precision="mixed")
    try:
        for wl in reqs:
            print("geometry", wl.name, len(wl.tris), flush=True)
            got = _run(reused, wl, torch)
            fresh = ibm.Grid(wl.xf, wl.yf, wl.zf, precision="mixed", poison=True)
            try:
                ref = _run(fresh, wl, torch)
            finally:
                fresh.close()
            _same(got, ref, wl.name)
            assert got["proj_fp64"][4] == 0 and got["proj_mixed"][4] == 0
    finally:
        reused.close()


def test_poisoned_handle_matches_oracle_types_and_solve():
    """The poisoned handle is an ordinary handle otherwise: classification equals the
    oracle's and a converged projection agrees with it."""
    torch = _torch()
    from oracle import OracleProblem
    from paper_2505_17287_amd import ibm
    wl = I.multibody(48, n_bodies=3, level=3)
    P = OracleProblem.from_workload(wl)
    g = ibm.Grid(wl.xf, wl.yf, wl.zf, precision="mixed", poison=True)
    try:
        g.setup(wl.verts, wl.tris)
        assert np.array_equal(g.cell_types().cpu().numpy(), P.types())
        u, v, w = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in wl.velocity())
        p, st = g.project(u, v, w, dt=1.0, rel_tol=1e-12)
    finally:
        g.close()
    u1, v1, w1, pr, sr, f = P.project(*wl.velocity(), dt=1.0, rel_tol=1e-12)
    act = P.types() != 2
    pg = p.cpu().numpy()
    err = np.max(np.abs((pg - pg[act].mean())[act] - (pr - pr[act].mean())[act])) / np.max(np.abs(pr[act]))
    assert st.status == 0 and err <= 1e-9
