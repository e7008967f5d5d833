"""Pins of the advection-diffusion oracle (CPU only).

Section 2.1 (central differences, Adams-Bashforth, implicit viscous term solved by scheduled
relaxed Jacobi) and Section 2.2 (ghost rows from the image-point interpolant, Eq. 2 and
Eq. 3, with the Dirichlet condition at the body intercept).  Each pin is fixed by the
mathematics, not by retyping the oracle:
  - the Dirichlet weights reproduce every trilinear function given in physical coordinates
    (member centres and the body intercept in, image point out); without the ghost in its
    box they are the tensor-product trilinear weights;
  - the ghost row reproduces a linear field at the ghost centre (mirror through BI);
  - the conservative convective term of a linear velocity field is exact at cells away
    from the walls, and telescopes to zero over a closed box;
  - the viscous operator equals the C oracle's pressure operator on fluid rows;
  - the schedule is min-max optimal (Chebyshev equioscillation, 1/T_m(1/rho));
  - Crank-Nicolson of a cosine eigenmode divides it by 1 + a |lambda|;
  - SRJ converges to the direct sparse solve of the assembled system, in 3D and 2D.
"""
import math

import numpy as np
import pytest

from oracle import OracleProblem
from oracle.momentum import MomentumOracle, srj_cycle_bound, srj_rho, srj_schedule
from paper_2505_17287_amd import inputs as I

_cache = {}


def _mo(name):
    if name not in _cache:
        wl = {"sphere": lambda: I.sphere_small(16, radius=0.45, level=3),
              "wing": lambda: I.wing(80, 48, 48),
              "cyl": lambda: I.cylinder2d(128)}[name]()
        P = OracleProblem.from_workload(wl)
        _cache[name] = (wl, MomentumOracle(P))
    return _cache[name]


def _centres(mo):
    return mo.m["xc"], mo.m["yc"], mo.m["zc"]


def _xyz(mo, cell):
    k, j, i = np.unravel_index(int(cell), (mo.nz, mo.ny, mo.nx))
    xc, yc, zc = _centres(mo)
    return np.array([xc[i], yc[j], zc[k]])


@pytest.mark.parametrize("name", ["sphere", "wing", "cyl"])
def test_dirichlet_weights_reproduce_trilinear(name):
    wl, mo = _mo(name)
    G = mo.G
    rng = np.random.default_rng(5)
    nchk = 0
    for g in range(len(G["cell"])):
        if mo.degenerate[g] or (G["flags"][g] & 2):  # clamped image points use clamped coordinates
            continue
        c = rng.standard_normal(8)

        def q(x):
            x0, y0, z0 = x
            if mo.two_d:
                return c[0] * x0 * y0 + c[1] * x0 + c[2] * y0 + c[3]
            return (c[0] * x0 * y0 * z0 + c[1] * x0 * y0 + c[2] * y0 * z0 + c[3] * x0 * z0 + c[4] * x0 + c[5] * y0
                    + c[6] * z0 + c[7])
        ip = G["ip"][g].copy()
        bi = G["bi"][g].copy()
        if mo.two_d:
            ip[2] = bi[2] = _xyz(mo, G["cell"][g])[2]
        s = sum(mo.beta[g, m] * q(_xyz(mo, mo.members[g, m])) for m in range(8) if mo.members[g, m] >= 0)
        s += mo.beta_g[g] * q(bi)
        scale = max(1.0, max(abs(q(_xyz(mo, mo.members[g, m]))) for m in range(8) if mo.members[g, m] >= 0))
        assert abs(s - q(ip)) <= 1e-11 * scale * max(1.0, np.abs(mo.beta[g]).sum() + abs(mo.beta_g[g]))
        assert abs(mo.beta[g].sum() + mo.beta_g[g] - 1.0) <= 1e-12
        nchk += 1
    assert nchk >= 10


def test_weights_without_self_are_trilinear():
    wl, mo = _mo("sphere")
    G = mo.G
    xc, yc, zc = _centres(mo)
    n = 0
    for g in range(len(G["cell"])):
        if mo.degenerate[g] or np.sum(mo.members[g] >= 0) < 8:
            continue
        i0 = np.unravel_index(int(mo.members[g, 0]), (mo.nz, mo.ny, mo.nx))[::-1]
        ip = G["ip"][g]
        t = [min(max((ip[0] - xc[i0[0]]) / (xc[i0[0] + 1] - xc[i0[0]]), 0), 1),
             min(max((ip[1] - yc[i0[1]]) / (yc[i0[1] + 1] - yc[i0[1]]), 0), 1),
             min(max((ip[2] - zc[i0[2]]) / (zc[i0[2] + 1] - zc[i0[2]]), 0), 1)]
        for m in range(8):
            a, b, cc = m & 1, (m >> 1) & 1, (m >> 2) & 1
            w = (t[0] if a else 1 - t[0]) * (t[1] if b else 1 - t[1]) * (t[2] if cc else 1 - t[2])
            assert abs(mo.beta[g, m] - w) <= 1e-13
        assert mo.beta_g[g] == 0.0
        n += 1
    assert n > 0


@pytest.mark.parametrize("name", ["sphere", "cyl"])
def test_ghost_row_reproduces_linear_field(name):
    """u = c0 + c.x, u_BI = u(BI): the ghost row gives 2 u(BI) - u(IP) = u(x_g) (BI is the
    midpoint of x_g and IP), whatever box the interpolant uses."""
    wl, mo = _mo(name)
    xc, yc, zc = _centres(mo)
    X = np.meshgrid(zc, yc, xc, indexing="ij")
    c0, cv = 0.3, np.array([0.7, -1.1, 0.4 if not mo.two_d else 0.0])
    lin = c0 + cv[0] * X[2] + cv[1] * X[1] + cv[2] * X[0]
    U = np.stack([lin, 2.0 * lin, -lin])
    G = mo.G
    ubi = np.zeros((len(G["cell"]), 3))
    for g in range(len(G["cell"])):
        bi = G["bi"][g]
        v = c0 + cv[0] * bi[0] + cv[1] * bi[1] + (cv[2] * bi[2] if not mo.two_d else 0.0)
        ubi[g] = (v, 2.0 * v, -v)
    out = mo.ghost_rows(U, ubi, src=U)
    n = 0
    for g in range(len(G["cell"])):
        if mo.degenerate[g] or (G["flags"][g] & 2):
            continue
        cell = int(G["cell"][g])
        at = (slice(None),) + np.unravel_index(cell, (mo.nz, mo.ny, mo.nx))
        exact = U[at]
        got = out[at]
        assert np.max(np.abs(got - exact)) <= 1e-11 * max(1.0, np.abs(U).max())
        n += 1
    assert n > 10


def _nobody(xf, yf, zf):
    P = OracleProblem(xf, yf, zf)
    P.classify()
    P.build_stencils()
    return MomentumOracle(P)


def test_convective_term_of_linear_field_is_exact():
    """u_i = c_i + G_ij x_j: -d(u_i u_j)/dx_j = -((G u)_i + u_i tr G) at every cell whose
    six faces are interior (stretched grid, no body)."""
    wl = I.wing(20, 16, 12)
    mo = _nobody(wl.xf, wl.yf, wl.zf)
    xc, yc, zc = _centres(mo)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    rng = np.random.default_rng(2)
    Gm = rng.standard_normal((3, 3))
    c = rng.standard_normal(3)
    U = np.stack([c[i] + Gm[i, 0] * X + Gm[i, 1] * Y + Gm[i, 2] * Z for i in range(3)])
    H = mo.convective(U)
    exact = -(np.einsum("ij,j...->i...", Gm, U) + U * np.trace(Gm))
    inner = (slice(None), slice(1, -1), slice(1, -1), slice(1, -1))
    assert np.max(np.abs(H[inner] - exact[inner])) <= 1e-11 * np.max(np.abs(exact))


def test_convective_term_telescopes():
    """No body, no flux through the box: sum_c V_c H_c = 0 for any field."""
    wl = I.wing(20, 16, 12)
    mo = _nobody(wl.xf, wl.yf, wl.zf)
    U = I.cell_velocity(3, 20, 16, 12)
    H = mo.convective(U)
    for q in range(3):
        assert abs(np.sum(mo.vol * H[q])) <= 1e-12 * np.sum(mo.vol * np.abs(H[q]))


def test_viscous_operator_is_the_pressure_operator():
    wl, mo = _mo("wing")
    rng = np.random.default_rng(4)
    phi = rng.standard_normal(mo.types.shape)
    fl = mo.types == 0
    a = mo.laplacian(phi)
    b = mo.P.apply_S(phi)
    assert np.max(np.abs(a[fl] - b[fl])) <= 1e-12 * np.max(np.abs(b[fl]))
    # the direct neighbour sum and the diagonal make up the same operator
    c = mo.neighbour_sum(phi) - mo.diag_sum() * phi
    assert np.max(np.abs(c[fl] - b[fl])) <= 1e-12 * np.max(np.abs(b[fl]))


@pytest.mark.parametrize("rho,m", [(0.3, 2), (0.6, 5), (0.9, 8), (0.99, 16)])
def test_srj_schedule_is_minmax(rho, m):
    w = srj_schedule(rho, m)
    assert len(w) == m
    kap = np.linspace(1.0 - rho, 1.0 + rho, 200001)
    amp = np.ones_like(kap)
    for x in w:
        amp *= 1.0 - x * kap
    bound = srj_cycle_bound(rho, m)
    assert abs(np.max(np.abs(amp)) - bound) <= 1e-6 * bound
    # equioscillation: m + 1 alternating extrema of equal magnitude, at the interval ends
    assert abs(abs(amp[0]) - bound) <= 1e-9 * max(bound, 1e-300) + 1e-15
    assert abs(abs(amp[-1]) - bound) <= 1e-9 * max(bound, 1e-300) + 1e-15
    assert bound < rho ** m  # beats plain Jacobi


def test_crank_nicolson_of_cosine_mode():
    """Uniform grid, no body: L cos-mode = lambda mode, so (I - a L)^{-1} mode =
    mode / (1 + a |lambda|), both by SRJ and by the direct solve."""
    nx, ny, nz = 12, 10, 8
    h = (0.3, 0.5, 0.4)
    mo = _nobody(np.arange(nx + 1) * h[0], np.arange(ny + 1) * h[1], np.arange(nz + 1) * h[2])
    kx, ky, kz = 3, 2, 1
    i, j, l = np.arange(nx), np.arange(ny), np.arange(nz)
    mode = (np.cos(np.pi * kz * (l + 0.5) / nz)[:, None, None] * np.cos(np.pi * ky * (j + 0.5) / ny)[None, :, None]
            * np.cos(np.pi * kx * (i + 0.5) / nx)[None, None, :])
    lam = -(4 / h[0] ** 2 * np.sin(np.pi * kx / (2 * nx)) ** 2 + 4 / h[1] ** 2 * np.sin(np.pi * ky / (2 * ny)) ** 2
            + 4 / h[2] ** 2 * np.sin(np.pi * kz / (2 * nz)) ** 2)
    alpha = 0.05
    b = np.stack([mode, 2 * mode, -mode])
    exact = b / (1.0 + alpha * abs(lam))
    rho = srj_rho(mo.m, alpha)
    U, cyc, rel, _ = mo.solve(b, np.zeros_like(b), alpha, srj_schedule(rho, 6), rel_tol=1e-14, max_cycles=500)
    assert np.max(np.abs(U - exact)) <= 1e-12
    assert np.max(np.abs(mo.exact_solve(b, alpha) - exact)) <= 1e-12


@pytest.mark.parametrize("name", ["sphere", "cyl"])
def test_srj_converges_to_direct_solve(name):
    wl, mo = _mo(name)
    nx, ny, nz = mo.nx, mo.ny, mo.nz
    U0, Hold = I.cell_velocity(11, nx, ny, nz), I.cell_velocity(12, nx, ny, nz)
    nu, dt = 0.05, 0.02
    G = mo.G
    ubi = np.tile(np.array([0.2, -0.1, 0.05]), (len(G["cell"]), 1))
    Us, H, cyc, rel = mo.step(U0, Hold, nu, dt, first=False, m=6, ubi=ubi, rel_tol=1e-13, max_cycles=400)
    assert rel <= 1e-13
    U = np.array(U0, copy=True)
    U[:, mo.types == 2] = 0.0
    U = mo.ghost_rows(U, ubi, src=U.copy())
    b = mo.cn_rhs(U, mo.convective(U), Hold, nu, dt, False)
    ref = mo.exact_solve(b, 0.5 * nu * dt, ubi)
    act = mo.types != 2
    assert np.max(np.abs(Us[:, act] - ref[:, act])) <= 1e-10 * np.max(np.abs(ref))
    # the solution satisfies every assembled row
    A = mo.assemble(0.5 * nu * dt)
    for q in range(3):
        r = A @ Us[q].ravel()
        fl = (mo.types == 0).ravel()
        assert np.max(np.abs(r[fl] - b[q].ravel()[fl])) <= 1e-10 * np.max(np.abs(b[q]))


def test_schedule_beats_plain_jacobi_on_the_step():
    wl, mo = _mo("sphere")
    nx, ny, nz = mo.nx, mo.ny, mo.nz
    U0, Hold = I.cell_velocity(21, nx, ny, nz), I.cell_velocity(22, nx, ny, nz)
    nu, dt = 1.0, 0.05  # strongly implicit: a d = O(10)
    alpha = 0.5 * nu * dt
    rho = srj_rho(mo.m, alpha)
    assert rho > 0.9
    m = 8
    _, _, c_srj, r_srj = mo.step(U0, Hold, nu, dt, first=True, m=m, rel_tol=1e-10, max_cycles=200)
    _, _, c_jac, r_jac = mo.step(U0, Hold, nu, dt, first=True, omegas=np.ones(m), rel_tol=1e-10, max_cycles=200)
    assert r_srj <= 1e-10
    assert c_srj < c_jac


def test_crank_nicolson_step_on_2d_modes():
    """2D, no body, uniform grid: u^n = (0, 0, w) has no convective term (no z faces, zero
    in-plane velocity), so one step is exact Crank-Nicolson on cosine eigenmodes:
      u* = w (1 - a|l1|)/(1 + a|l1|) - (dt/2) H^{n-1} / (1 + a|l2|)
    for w a mode with eigenvalue l1 and every component of H^{n-1} a mode with l2."""
    n, h = 16, 0.25
    f = np.arange(n + 1) * h
    mo = _nobody(f, f.copy(), np.array([-h / 2, h / 2]))
    i = np.arange(n)

    def mode(kx, ky):
        return (np.cos(np.pi * ky * (i + 0.5) / n)[:, None] * np.cos(np.pi * kx * (i + 0.5) / n)[None, :])[None]

    def lam(kx, ky):
        return -(4 / h ** 2) * (np.sin(np.pi * kx / (2 * n)) ** 2 + np.sin(np.pi * ky / (2 * n)) ** 2)
    m1, l1 = mode(3, 1), lam(3, 1)
    m2, l2 = mode(1, 4), lam(1, 4)
    U = np.stack([np.zeros_like(m1), np.zeros_like(m1), 0.7 * m1])
    Hold = np.stack([m2, m2, m2])
    nu, dt = 0.2, 0.1
    a = 0.5 * nu * dt
    Us, H, cyc, rel = mo.step(U, Hold, nu, dt, first=False, m=4, rel_tol=1e-14, max_cycles=400)
    assert np.max(np.abs(H)) == 0.0
    hold = -0.5 * dt * m2 / (1.0 + a * abs(l2))
    exact = np.stack([hold, hold, 0.7 * m1 * (1.0 - a * abs(l1)) / (1.0 + a * abs(l1)) + hold])
    assert np.max(np.abs(Us - exact)) <= 1e-12
