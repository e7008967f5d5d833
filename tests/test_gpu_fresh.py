"""GPU parity of the fresh cells of a moved body (Section 2.2) against the oracle.

The fresh list (cells ghost or dead before the move, fluid after it) is compared exactly,
intercepts and image points to 1e-12, box members exactly, weights to 1e-13 (GPU tensor
product against the oracle's LU), and the filled values to 1e-12: a 3D sphere and the 2D
cylinder moved by a fraction of a cell, two moves in a row, a move by zero, and the
multi-body 256^3 workload with every body translated.
"""
import numpy as np
import pytest

from oracle import OracleProblem
from oracle.fresh import FreshOracle
from paper_2505_17287_amd import inputs as I

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _oracle(wl, verts_old, verts_new):
    P0 = OracleProblem(wl.xf, wl.yf, wl.zf)
    P0.set_mesh(verts_old, wl.tris)
    P0.classify()
    P1 = OracleProblem(wl.xf, wl.yf, wl.zf)
    P1.set_mesh(verts_new, wl.tris)
    P1.classify()
    P1.build_stencils()
    return P1, FreshOracle(P0.types(), P1)


def _compare(g, F, P1, U0, ubi):
    torch = _torch()
    assert np.array_equal(g.cell_types().cpu().numpy(), P1.types())
    d = g.fresh()
    assert np.array_equal(d["cell"].astype(np.int64), F.cells)
    if len(F.cells) == 0:
        return
    assert np.max(np.abs(d["bi"] - F.bi)) <= 1e-12
    assert np.max(np.abs(d["ip"] - F.ip)) <= 1e-12
    deg = (d["flags"] & 1) != 0
    assert np.array_equal(deg, F.degenerate)
    ok = ~deg
    assert np.array_equal(np.where(F.members[ok] >= 0, F.members[ok], -1), d["stencil"][ok])
    assert np.max(np.abs(d["beta"][ok] - F.beta[ok]), initial=0.0) <= 1e-13
    assert np.max(np.abs(d["beta_c"][ok] - F.beta_c[ok]), initial=0.0) <= 1e-13
    U = torch.from_numpy(np.ascontiguousarray(U0)).cuda()
    g.fill_fresh(U, ubi)
    ref = F.fill(U0, ubi)
    assert np.max(np.abs(U.cpu().numpy() - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("name", ["sphere", "cylinder2d"])
def test_fresh_cells_match_oracle(name):
    _torch()
    from paper_2505_17287_amd import ibm
    if name == "sphere":
        wl, h = I.sphere_small(24, radius=0.45, level=3), 2.0 / 24
        shifts = [(0.6 * h, -0.25 * h, 0.1 * h), (0.3 * h, 0.5 * h, -0.4 * h)]
    else:
        wl, h = I.cylinder2d(128), 16.0 / 128
        shifts = [(0.7 * h, 0.3 * h, 0.0), (-0.5 * h, 0.6 * h, 0.0)]
    print("case", wl.name, flush=True)
    g = ibm.Grid(wl.xf, wl.yf, wl.zf)
    g.setup(wl.verts, wl.tris)
    verts = wl.verts.copy()
    U0, _ = wl.cell_fields()
    rng = np.random.default_rng(3)
    for sh in shifts:  # two moves in a row: the second is relative to the first
        new = verts + np.asarray(sh)
        counts, nf = g.move_geometry(new, wl.tris)
        P1, F = _oracle(wl, verts, new)
        assert nf == len(F.cells) > 0
        ubi = rng.uniform(-0.3, 0.3, size=(nf, 3))
        _compare(g, F, P1, U0, ubi)
        verts = new
    # a changed triangle list is checked again: one flipped triangle is refused
    bad = wl.tris.copy()
    bad[0] = bad[0][::-1]
    with pytest.raises(ibm.IBMError):
        g.move_geometry(verts, bad)
    # a move by zero leaves no fresh cell and the fill changes nothing
    counts, nf = g.move_geometry(verts, wl.tris)
    assert nf == 0
    torch = _torch()
    U = torch.from_numpy(np.ascontiguousarray(U0)).cuda()
    g.fill_fresh(U)
    assert np.array_equal(U.cpu().numpy(), U0)
    g.close()


def test_fresh_cells_multibody_256():
    _torch()
    from paper_2505_17287_amd import ibm
    wl = I.multibody(256)
    h = float(np.min(np.diff(wl.xf)))
    print("case", wl.name, flush=True)
    g = ibm.Grid(wl.xf, wl.yf, wl.zf)
    g.setup(wl.verts, wl.tris)
    new = wl.verts + np.array([0.3 * h, -0.2 * h, 0.1 * h])
    counts, nf = g.move_geometry(new, wl.tris)
    print("fresh cells", nf, flush=True)
    P1, F = _oracle(wl, wl.verts, new)
    assert nf == len(F.cells) > 1000
    U0, _ = wl.cell_fields()
    _compare(g, F, P1, U0, None)
    g.close()
