"""Pins of the fractional-step composition oracle (oracle/fractional.py), CPU only.

- face interpolation: a field linear in x, y, z (different coefficients per component) is
  reproduced exactly at every interior face of a stretched grid, and the wall faces are 0
  (a transposed weight, a wrong axis or a wrong wall value fails it);
- cell correction: with a pressure linear in x on a body-free stretched grid, the oracle's
  own face correction (oracle.c) changes every interior x-face by dt c, so the cell update is
  dt c away from the walls and dt c / 2 next to them, v and w unchanged (a wrong sign, a
  missing halving or a correction applied to the wrong component fails it);
- the composed step on a body: the corrected faces satisfy the projection identity
  D U^{n+1} = dt lambda on fluid cells, only fluid cells change in the cell correction, and
  the cell correction is a mean of face corrections (bounded by the largest of them).
"""
import numpy as np

from oracle import OracleProblem
from oracle.fractional import cell_to_faces, correct_cells, fractional_step
from oracle.momentum import MomentumOracle
from paper_2505_17287_amd import inputs as I


def _stretched():
    wl = I.wing(40, 24, 20)
    return wl.xf, wl.yf, wl.zf


def test_faces_of_a_linear_field_are_exact():
    xf, yf, zf = _stretched()
    xc, yc, zc = (0.5 * (a[1:] + a[:-1]) for a in (xf, yf, zf))
    coef = np.array([[0.3, 1.7, -0.4, 2.1], [-1.2, 0.5, 3.3, -0.7], [2.0, -0.9, 0.8, 1.4]])

    def lin(d, x, y, z):
        a, b, c, e = coef[d]
        return a + b * x + c * y + e * z

    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    U = np.stack([lin(d, X, Y, Z) for d in range(3)])
    uf, vf, wf = cell_to_faces(xf, yf, zf, U)
    assert uf.shape == (len(zc), len(yc), len(xc) + 1)
    assert vf.shape == (len(zc), len(yc) + 1, len(xc))
    assert wf.shape == (len(zc) + 1, len(yc), len(xc))
    Zu, Yu, Xu = np.meshgrid(zc, yc, xf[1:-1], indexing="ij")
    Zv, Yv, Xv = np.meshgrid(zc, yf[1:-1], xc, indexing="ij")
    Zw, Yw, Xw = np.meshgrid(zf[1:-1], yc, xc, indexing="ij")
    scale = np.abs(U).max()
    assert np.max(np.abs(uf[:, :, 1:-1] - lin(0, Xu, Yu, Zu))) <= 1e-13 * scale
    assert np.max(np.abs(vf[:, 1:-1, :] - lin(1, Xv, Yv, Zv))) <= 1e-13 * scale
    assert np.max(np.abs(wf[1:-1, :, :] - lin(2, Xw, Yw, Zw))) <= 1e-13 * scale
    for a, ax in ((uf, 2), (vf, 1), (wf, 0)):
        assert not np.take(a, [0, a.shape[ax] - 1], axis=ax).any()


def test_cell_correction_of_a_linear_pressure():
    xf, yf, zf = _stretched()
    P = OracleProblem(xf, yf, zf)
    P.classify()  # no body: every cell fluid
    nz, ny, nx = P.shape
    xc = 0.5 * (xf[1:] + xf[:-1])
    c, dt = 0.8, 0.25
    p = np.broadcast_to(c * xc, (nz, ny, nx)).copy()
    rng = np.random.default_rng(11)
    before = [rng.uniform(-1, 1, s) for s in ((nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx))]
    for a, ax in zip(before, (2, 1, 0)):  # walls 0, as the face interpolation leaves them
        idx = [slice(None)] * 3
        idx[ax] = [0, a.shape[ax] - 1]
        a[tuple(idx)] = 0.0
    after = P.correct(*before, p, dt=dt)
    Us = rng.uniform(-1, 1, (3, nz, ny, nx))
    U1 = correct_cells(P.types(), Us, before, after)
    want = np.full(nx, dt * c)
    want[0] = want[-1] = 0.5 * dt * c
    assert np.max(np.abs((Us[0] - U1[0]) - want[None, None, :])) <= 1e-12
    assert np.array_equal(U1[1], Us[1]) or np.max(np.abs(U1[1] - Us[1])) <= 1e-15
    assert np.max(np.abs(U1[2] - Us[2])) <= 1e-15


def test_composed_step_on_a_body():
    wl = I.multibody(32, n_bodies=2, level=3)
    P = OracleProblem.from_workload(wl)
    mo = MomentumOracle(P)
    U0, H0 = wl.cell_fields()
    nu, dt = 1e-2, 0.5 * float(np.min(np.diff(wl.xf)))
    U1, H, faces, p, st = fractional_step(P, mo, U0, H0, nu, dt, first=True, mom_rel_tol=1e-12, rel_tol=1e-12,
                                          max_cycles=400, method="bicgstab")
    assert st.status == 0
    t = P.types()
    fl = t == 0
    div = P.rhs(*faces, dt=1.0)
    Us, _, _, _ = mo.step(U0, H0, nu, dt, first=True, rel_tol=1e-12)
    before = cell_to_faces(P.xf, P.yf, P.zf, Us)
    f = P.rhs(*before, dt=dt)
    assert np.max(np.abs(div[fl] - dt * st.lam)) <= 1e-9 * np.max(np.abs(f)) * dt
    # only fluid cells move; each moves by a mean of two face corrections
    assert np.array_equal(U1[:, ~fl], Us[:, ~fl])
    for d, ax in enumerate((2, 1, 0)):
        dU = np.abs(before[d] - faces[d])
        n = dU.shape[ax] - 1
        bound = np.maximum(np.take(dU, np.arange(0, n), axis=ax), np.take(dU, np.arange(1, n + 1), axis=ax))
        assert np.all(np.abs(U1[d] - Us[d]) <= bound + 1e-15)
