"""Pins of the oracle's multigrid hierarchy (coarsening by cell width), CPU only.

- a uniform grid is halved outright (coarse cell I holds fine 2I and 2I+1; an odd count
  keeps its last cell whole); an axis twice as coarse as the others is kept (semi-coarsening)
  until the others catch up;
- every level holds at most half the cells of the level above it, so the coarse levels
  together never exceed the grid (the workspace bound relies on it);
- the narrowest cells merge first: on a stretched axis no cell kept whole is narrower than
  half of the widest merged pair, and every kept cell is well above the smallest width;
- what the rule is for: on the stretched multi-body grid without bodies the V-cycle
  contracts by at most 0.25 per cycle at 96^3 and 0.22 at 128^3 (the per-axis halving of
  the same levels gave 0.30-0.36 and kept degrading with the aspect ratio).
"""
import numpy as np
import pytest

from oracle import OracleProblem
from paper_2505_17287_amd import inputs as I


def _levels(xf, yf, zf):
    P = OracleProblem(xf, yf, zf)
    P.classify()
    return P, P.levels()


def test_uniform_axes_are_halved():
    for n in (64, 33):
        f = np.linspace(-1.0, 1.0, n + 1)
        P, lv = _levels(f, f, np.linspace(0.0, 16.0 / n, 9))  # the same spacing on all axes
        (csx, csy, csz) = P.level_map(1)
        half = (n + 1) // 2
        assert lv[1]["dims"] == (half, half, 4)
        want = np.minimum(2 * np.arange(half + 1), n)
        assert np.array_equal(csx, want) and np.array_equal(csy, want)
        assert np.array_equal(csz, [0, 2, 4, 6, 8])
    f = np.linspace(-1.0, 1.0, 65)
    P, lv = _levels(f, f, np.linspace(0.0, 0.5, 9))  # z cells twice as wide
    assert lv[1]["dims"] == (32, 32, 8) and lv[2]["dims"] == (16, 16, 4)


@pytest.mark.parametrize("wl", [I.wing(96, 48, 48), I.multibody(64, n_bodies=1, level=1), I.cylinder2d(64)],
                         ids=["wing", "multibody", "cylinder"])
def test_levels_shrink_by_half(wl):
    P, lv = _levels(wl.xf, wl.yf, wl.zf)
    cells = [int(np.prod(l["dims"])) for l in lv]
    assert len(cells) >= 3
    for a, b in zip(cells, cells[1:]):
        assert 2 * b <= a or b < a  # at most half, or the last levels of a tiny grid
    assert sum(cells[1:]) <= cells[0]
    for l in range(1, len(lv)):
        for d, cs in enumerate(P.level_map(l)):
            assert cs[0] == 0 and cs[-1] == lv[l - 1]["dims"][d]
            assert np.all(np.diff(cs) >= 1) and np.all(np.diff(cs) <= 2)


def test_narrowest_cells_merge_first():
    wl = I.multibody(96, n_bodies=1, level=1)
    P, lv = _levels(wl.xf, wl.yf, wl.zf)
    w = np.diff(wl.xf)
    cs = P.level_map(1)[0]
    counts = np.diff(cs)
    merged = [w[a] + w[a + 1] for a, c in zip(cs[:-1], counts) if c == 2]
    kept = [w[a] for a, c in zip(cs[:-1], counts) if c == 1]
    assert merged and kept
    # a cell is kept whole only where it is already wider than the narrowest cells
    assert min(kept) >= 0.5 * max(merged) * 0.999
    assert min(kept) > 1.5 * w.min()


@pytest.mark.parametrize("n,bound", [(96, 0.25), (128, 0.22)])
def test_vcycle_contracts_on_the_stretched_grid(n, bound):
    wl = I.multibody(n)
    P = OracleProblem(wl.xf, wl.yf, wl.zf)
    P.classify()  # no body: the stretched shell alone
    rng = np.random.default_rng(0)
    f = rng.standard_normal(P.shape)
    r2 = P.solve(f, fixed_cycles=2, method="vcycle")[1].rel_residual
    r6 = P.solve(f, fixed_cycles=6, method="vcycle")[1].rel_residual
    rate = (r6 / r2) ** 0.25
    assert rate <= bound, rate
