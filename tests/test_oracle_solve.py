"""Pins of the oracle's pressure solve and projection (CPU only).

Section 2.1 of the paper: fractional step (a pressure Poisson equation, then the velocity
correction), solved iteratively; Section 2.2: the ghost equations sit implicitly in the
linear system.  The multigrid result is pinned against
  * a DCT-II Neumann solve (uniform grid, no body),
  * fast diagonalisation by per-axis generalized eigenvectors (stretched grid, no body;
    Lynch, Rice and Thomas 1964),
  * dense LU of the bordered system [S 1; V^T 0][p; lambda] = [f; 0] on tiny grids with a
    body (every fluid, ghost and dead row assembled here from its definition),
  * a manufactured solution with exact Neumann data (orders of the ghost closure, the
    interior truncation and the solution),
and the projection against the identity D u^{n+1} = dt (lambda + r').
"""
import numpy as np
import pytest
import scipy.fft
import scipy.linalg
from scipy import ndimage

from oracle import OracleProblem
from paper_2505_17287_amd import inputs as I


def _vol(P):
    wx, wy, wz = (np.diff(f) for f in (P.xf, P.yf, P.zf))
    return wz[:, None, None] * wy[None, :, None] * wx[None, None, :]


def _nobody(xf, yf, zf):
    P = OracleProblem(xf, yf, zf)
    P.classify()
    P.build_stencils()
    return P


def test_uniform_nobody_matches_dct_solve():
    nx, ny, nz = 32, 24, 16
    h = (0.25, 0.4, 0.3)
    xf, yf, zf = (np.arange(n + 1) * hh for n, hh in zip((nx, ny, nz), h))
    P = _nobody(xf, yf, zf)
    f = np.random.default_rng(0).standard_normal((nz, ny, nx))
    p, st = P.solve(f, rel_tol=1e-13, max_cycles=60)
    assert st.cycles < 60
    fh = scipy.fft.dctn(f, type=2, norm="ortho")
    lam = np.zeros((nz, ny, nx))
    for ax, (n, hh) in enumerate(zip((nz, ny, nx), (h[2], h[1], h[0]))):
        k = np.arange(n)
        shp = [1, 1, 1]
        shp[ax] = n
        lam = lam - (4.0 / hh ** 2 * np.sin(np.pi * k / (2 * n)) ** 2).reshape(shp)
    ph = np.zeros_like(fh)
    ph[lam != 0] = fh[lam != 0] / lam[lam != 0]
    pref = scipy.fft.idctn(ph, type=2, norm="ortho")
    assert abs(st.lam - f.mean()) < 1e-13 * np.abs(f).max()
    assert np.max(np.abs(p - pref)) <= 1e-11 * np.max(np.abs(pref))


def _op1d(f):
    c = 0.5 * (f[1:] + f[:-1])
    w = np.diff(f)
    n = len(w)
    K = np.zeros((n, n))
    for i in range(n - 1):
        t = 1.0 / (c[i + 1] - c[i])
        K[i, i] -= t
        K[i + 1, i + 1] -= t
        K[i, i + 1] += t
        K[i + 1, i] += t
    return K, np.diag(w)


def test_stretched_nobody_matches_fast_diagonalisation():
    wl = I.wing(48, 32, 40)
    P = _nobody(wl.xf, wl.yf, wl.zf)
    f = np.random.default_rng(1).standard_normal(P.shape)
    p, st = P.solve(f, rel_tol=1e-13, max_cycles=150)
    assert st.status == 0
    Q = []
    M = []
    for fc in (wl.zf, wl.yf, wl.xf):
        K, W = _op1d(fc)
        mu, q = scipy.linalg.eigh(K, W)
        mu[np.argmax(mu)] = 0.0  # the constant mode
        Q.append((q, W))
        M.append(mu)
    vol = _vol(P)
    lam = np.sum(vol * f) / np.sum(vol)
    g = f - lam
    # coefficients: Q^{-1} = Q^T W per axis
    c = np.einsum("ai,ab,bjk->ijk", Q[0][0], Q[0][1], g)
    c = np.einsum("aj,ab,ibk->ijk", Q[1][0], Q[1][1], c)
    c = np.einsum("ak,ab,ijb->ijk", Q[2][0], Q[2][1], c)
    den = M[0][:, None, None] + M[1][None, :, None] + M[2][None, None, :]
    c = np.where(den != 0, c / np.where(den != 0, den, 1.0), 0.0)
    pref = np.einsum("ia,ajk->ijk", Q[0][0], c)
    pref = np.einsum("ja,iak->ijk", Q[1][0], pref)
    pref = np.einsum("ka,ija->ijk", Q[2][0], pref)
    pref -= np.sum(vol * pref) / np.sum(vol)
    assert abs(st.lam - lam) < 1e-12 * np.abs(f).max()
    assert np.max(np.abs(p - pref)) <= 1e-10 * np.max(np.abs(pref))


def dense_bordered_solution(P, f):
    """Assemble [S 1; V^T 0] row by row from the definitions and solve it densely."""
    t = P.types().ravel()
    g = P.ghosts()
    nz, ny, nx = P.shape
    n = nx * ny * nz
    xc, yc, zc = (0.5 * (a[1:] + a[:-1]) for a in (P.xf, P.yf, P.zf))
    wx, wy, wz = (np.diff(a) for a in (P.xf, P.yf, P.zf))
    A = np.zeros((n + 1, n + 1))
    b = np.zeros(n + 1)
    vol = _vol(P).ravel()
    fl = f.ravel()
    gi = {int(c): q for q, c in enumerate(g["cell"])}
    for idx in range(n):
        i, j, k = idx % nx, (idx // nx) % ny, idx // (nx * ny)
        if t[idx] == 0:
            for d, (ii, n_, cc, ww, stride) in enumerate(((i, nx, xc, wx, 1), (j, ny, yc, wy, nx), (k, nz, zc, wz, nx * ny))):
                for s in (-1, 1):
                    if 0 <= ii + s < n_:
                        a = 1.0 / (ww[ii] * abs(cc[ii + s] - cc[ii]))
                        A[idx, idx + s * stride] += a
                        A[idx, idx] -= a
            A[idx, n] = 1.0  # lambda
            b[idx] = fl[idx]
            A[n, idx] = vol[idx]
        elif t[idx] == 1:
            q = gi[idx]
            A[idx, idx] = 1.0
            if g["flags"][q] & 1:
                cnt = 0
                for dk in (-1, 0, 1):
                    for dj in (-1, 0, 1):
                        for di in (-1, 0, 1):
                            ii, jj, kk = i + di, j + dj, k + dk
                            if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz and t[(kk * ny + jj) * nx + ii] == 0:
                                cnt += 1
                for dk in (-1, 0, 1):
                    for dj in (-1, 0, 1):
                        for di in (-1, 0, 1):
                            ii, jj, kk = i + di, j + dj, k + dk
                            if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz and t[(kk * ny + jj) * nx + ii] == 0:
                                A[idx, (kk * ny + jj) * nx + ii] -= 1.0 / cnt
            else:
                for m in range(8):
                    if g["stencil"][q, m] >= 0:
                        A[idx, g["stencil"][q, m]] -= g["beta"][q, m]
                b[idx] = g["h"][q]
        else:
            A[idx, idx] = 1.0
    x = np.linalg.solve(A, b)
    return x[:n].reshape(P.shape), x[n]


def srj_pressure_schedule(m):
    """Relaxation factors of the SRJ preconditioner: the Chebyshev schedule on
    [1 - cos(pi/m), 1 + cos(pi/m)] (oracle.momentum.srj_schedule)."""
    from oracle.momentum import srj_schedule
    return srj_schedule(np.cos(np.pi / m), m)


@pytest.mark.parametrize("method", ["vcycle", "bicgstab", "bicgstab_srj"])
@pytest.mark.parametrize("case", ["sphere3d", "plate3d", "cylinder2d"])
def test_multigrid_equals_dense_bordered_solve(case, method):
    if case == "sphere3d":
        wl = I.sphere_small(8, level=3)
    elif case == "plate3d":
        v, t = I.box_mesh((0.03, -0.02, 0.01), (1.1, 0.9, 0.5), 20.0)
        f_ = I.uniform_faces(-1, 1, 10)
        wl = I.Workload("plate3d", f_, f_, f_, v, t, seed=3)
    else:
        f_ = I.uniform_faces(-1, 1, 12)
        v, t = I.prism_mesh(0.37, 64, -1, 1, center=(0.04, -0.03))
        wl = I.Workload("cyl", f_, f_, np.array([-0.08, 0.08]), v, t, seed=3)
    P = OracleProblem.from_workload(wl)
    assert P.ghosts()["cell"].size > 0
    rng = np.random.default_rng(5)
    f = rng.standard_normal(P.shape) * (P.types() == 0)
    # nonzero Neumann data so the ghost right-hand sides are exercised
    P.set_neumann(rng.standard_normal(len(P.ghost_cells())))
    kw = dict(srj_omega=srj_pressure_schedule(8)) if method == "bicgstab_srj" else {}
    p, st = P.solve(f, rel_tol=1e-13, max_cycles=200, method=method, **kw)
    assert st.status == 0
    pd, lam = dense_bordered_solution(P, f)
    act = P.types() != 2
    assert abs(st.lam - lam) <= 1e-11 * max(1.0, abs(lam))
    assert np.max(np.abs(p[act] - pd[act])) <= 1e-11 * np.max(np.abs(pd[act]))
    assert np.all(p[~act] == 0.0)


def test_gauge_and_lambda_properties():
    wl = I.multibody(32, n_bodies=2, level=3)
    P = OracleProblem.from_workload(wl)
    u, v, w = wl.velocity()
    f = P.rhs(u, v, w)
    fl = P.types() == 0
    vol = _vol(P)
    p, st = P.solve(f, rel_tol=1e-12)
    # zero V-weighted mean over the fluid cells
    assert abs(np.sum(vol[fl] * p[fl])) <= 1e-12 * np.sum(vol[fl] * np.abs(p[fl]))
    # independent of a constant added to the initial guess
    p2, st2 = P.solve(f, p0=np.full(P.shape, 3.7), rel_tol=1e-12)
    assert np.max(np.abs(p2 - p)) <= 1e-9 * np.max(np.abs(p))
    # the projection right-hand side telescopes: sum V f = net flux through the fluid
    # region's faces with non-fluid cells (the walls carry none)
    # no body: sum V f = 0 exactly up to round-off
    Pn = _nobody(wl.xf, wl.yf, wl.zf)
    fn = Pn.rhs(u, v, w)
    assert abs(np.sum(vol * fn)) <= 1e-13 * np.sum(vol * np.abs(fn))
    pn, stn = Pn.solve(fn)
    assert abs(stn.lam) <= 1e-12 * np.abs(fn).max()


def test_projection_identity_and_idempotence():
    wl = I.multibody(32, n_bodies=2, level=3)
    P = OracleProblem.from_workload(wl)
    u, v, w = wl.velocity()
    dt = 0.5
    u1, v1, w1, p, st, f = P.project(u, v, w, dt=dt, rel_tol=1e-12)
    fl = P.types() == 0
    div = P.rhs(u1, v1, w1, dt=1.0)
    # D u^{n+1} = dt (lambda + r'), with |r'| <= tol * |f'|
    assert np.max(np.abs(div[fl] - dt * st.lam)) <= 1e-9 * np.max(np.abs(f))
    # faces touching no fluid cell keep their values
    t = P.types()
    nf_x = np.zeros(u.shape, bool)
    nf_x[:, :, 1:-1] = (t[:, :, 1:] != 0) & (t[:, :, :-1] != 0)
    assert np.array_equal(u1[nf_x], u[nf_x])
    # a second projection changes nothing beyond the tolerance
    u2, v2, w2, p2, st2, f2 = P.project(u1, v1, w1, dt=dt, rel_tol=1e-12)
    assert np.max(np.abs(u2 - u1)) <= 1e-8 * np.max(np.abs(u))


def _mms_case(n, stretched=False):
    wl = I.mms_workload(n, stretched=stretched, level=5)
    P = OracleProblem.from_workload(wl)
    g = P.ghosts()
    gx, gy, gz = I.mms_grad(g["bi"][:, 0], g["bi"][:, 1], g["bi"][:, 2])
    P.set_neumann(gx * g["n"][:, 0] + gy * g["n"][:, 1] + gz * g["n"][:, 2])
    xc, yc, zc = (0.5 * (a[1:] + a[:-1]) for a in (wl.xf, wl.yf, wl.zf))
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    t = P.types()
    fl = t == 0
    f = np.where(fl, I.mms_source(X, Y, Z), 0.0)
    ex = I.mms_exact(X, Y, Z)
    h = np.max(np.diff(wl.xf[(wl.xf > -0.6) & (wl.xf < 0.6)]))
    return wl, P, g, t, fl, f, ex, h


def _mms_error(n, stretched=False):
    wl, P, g, t, fl, f, ex, h = _mms_case(n, stretched)
    p, st = P.solve(f, rel_tol=1e-12, max_cycles=100)
    assert st.status == 0 and np.sum(g["flags"] & 1) == 0
    vol = _vol(P)
    err = p - ex
    err = err - np.sum(vol[fl] * err[fl]) / np.sum(vol[fl])
    # ghost equations applied to the exact solution: error against its smooth extension
    pe = np.where(t == 2, 0.0, ex)
    pg = P.ghost_refresh(pe)
    gerr = np.max(np.abs(pg.ravel()[g["cell"]] - ex.ravel()[g["cell"]]))
    tau = np.abs(f - P.apply_S(pg))
    # fluid rows next to a ghost (a face neighbour) and rows at least 3 cells from every ghost
    face = np.zeros((3, 3, 3), bool)
    face[1, 1, :] = face[1, :, 1] = face[:, 1, 1] = True
    near = ndimage.binary_dilation(t == 1, structure=face) & fl
    far = ~ndimage.binary_dilation(t == 1, structure=np.ones((3, 3, 3), bool), iterations=3) & fl
    return dict(h=h, l2=np.sqrt(np.sum(vol[fl] * err[fl] ** 2) / np.sum(vol[fl])), linf=np.max(np.abs(err[fl])),
                lam=abs(st.lam), ghost=gerr, trunc=np.max(tau[far]), near=np.max(tau[near]),
                near_int=np.sum(vol[near] * tau[near]))


def _order(a, b, key):
    return np.log(a[key] / b[key]) / np.log(a["h"] / b["h"])


@pytest.mark.parametrize("stretched", [False, True])
def test_manufactured_solution_orders(stretched):
    """p = cos(pi x) cos(pi y) cos(pi z) on [-1,1]^3 (zero normal derivative on the box)
    around a sphere, with exact normal-derivative data at the body intercepts, on 32^3, 64^3
    and 96^3.

    The image-point closure (Eq. 2 with the Neumann row of Eq. 3) gives the ghost values to
    second order, and the interior rows are second-order consistent on uniform grids.  But a
    ghost value with an O(h^2) error enters the flux of the face it shares with a fluid cell
    divided by h^2 (the flux over the cell volume), so the fluid rows next to the body keep
    an O(1) truncation error that does not decay; it fills a layer one cell thick, of volume
    O(h), so its integral is O(h), and the pressure error and the compatibility shift lambda
    converge at first order.  These measured orders (and the O(1) layer that explains them)
    are asserted within about 0.1 of their values; the second order of the interior is not
    reachable with a trilinear (second-order) ghost closure of a Neumann condition."""
    res = [_mms_error(n, stretched) for n in (32, 64, 96)]
    for a, b in zip(res[:-1], res[1:]):
        assert _order(a, b, "ghost") >= 1.85
        if not stretched:  # cell-centred rows on a stretched family are only supraconvergent
            assert _order(a, b, "trunc") >= 1.9
        assert 0.9 <= _order(a, b, "l2") <= 1.15
        assert 0.75 <= _order(a, b, "linf") <= 1.15
        assert 0.8 <= _order(a, b, "lam") <= 1.1
        # the mechanism: O(1) truncation next to the body, O(h) once integrated over its layer
        assert -0.25 <= _order(a, b, "near") <= 0.15
        assert 0.7 <= _order(a, b, "near_int") <= 1.1
    for r in res:
        assert 3.0 <= r["near"] <= 9.0
    # first order with a steady constant: error / h within 10 % across the family
    c = [r["l2"] / r["h"] for r in res]
    assert max(c) / min(c) < 1.1
    assert res[-1]["l2"] < 0.002 and res[-1]["linf"] < 0.01


def test_bicgstab_restarts_reach_the_same_solution():
    """With a breakdown threshold so large that near-breakdowns are declared often, the
    oracle's BiCGStab restarts its shadow residual several times and still converges to the
    dense bordered solution (the restart changes the Krylov path, not the fixed point)."""
    wl = I.sphere_small(8, level=3)
    P = OracleProblem.from_workload(wl)
    rng = np.random.default_rng(12)
    f = rng.standard_normal(P.shape) * (P.types() == 0)
    p0, s0 = P.solve(f, rel_tol=1e-13, max_cycles=300, method="bicgstab")
    p1, s1 = P.solve(f, rel_tol=1e-13, max_cycles=300, method="bicgstab", breakdown_tol=0.9)
    assert s0.status == 0 and s1.status == 0
    assert s0.restarts == 0 and s1.restarts >= 2
    pd, lam = dense_bordered_solution(P, f)
    act = P.types() != 2
    for p in (p0, p1):
        assert np.max(np.abs(p[act] - pd[act])) <= 1e-11 * np.max(np.abs(pd[act]))
