"""Pins of the oracle's special branches on constructed geometry (Section 2.2).

Each workload places bodies on the grid so that one branch is taken many times:
  - edge_slot: two boxes separated by a slot narrower than a cell, one of them 0.7 h from a
    wall -> degenerate ghosts (a dead member or no fluid member in the image-point box) and
    clamped image points (beyond the outermost cell centre);
  - edge_aligned: box faces exactly through cell centres -> centres on the surface,
    classified by the edge-ownership rule (x, y faces) or the open crossing interval
    (z faces), and ghosts on the surface with the facet-normal fallback;
  - edge_vertices: polyhedra with vertices on column centres -> rays through vertices and
    along projected edges.

Independent checks: the generalized winding number (at the centre, or at the centre moved
by (+d, -d^2, 0) for centres on a vertical face, which is what edge ownership means), the
closed-form nearest point of an axis-aligned box, the definitions of the image point, the
box, the clamping and the degenerate test recomputed from the intercept and normal, exact
reproduction of trilinear functions, and a dense solve of the bordered system assembled
with the degenerate rows written out from their definition.
"""
import numpy as np
import pytest

from oracle import OracleProblem
from paper_2505_17287_amd import inputs as I

from test_oracle_geometry import cell_centres, winding_number
from test_oracle_solve import dense_bordered_solution

FLAG_DEG, FLAG_CLAMP, FLAG_NFALL, FLAG_SELF = 1, 2, 4, 8


def _problem(wl, stencils=True):
    P = OracleProblem(wl.xf, wl.yf, wl.zf)
    P.set_mesh(wl.verts, wl.tris)
    P.classify()
    if stencils:
        P.build_stencils()
    return P


def _on_surface(pts, verts, tris, tol=1e-12):
    """Points lying (closed) on some facet: in its plane and inside it (barycentric test)."""
    out = np.zeros(len(pts), bool)
    for a, b, c in tris:
        A, B, C = verts[a], verts[b], verts[c]
        nrm = np.cross(B - A, C - A)
        nn = np.linalg.norm(nrm)
        plane = np.abs((pts - A) @ nrm) <= tol * nn
        if not plane.any():
            continue
        P = pts[plane]
        v0, v1, v2 = C - A, B - A, P - A
        d00, d01, d11 = v0 @ v0, v0 @ v1, v1 @ v1
        d20, d21 = v2 @ v0, v2 @ v1
        den = d00 * d11 - d01 * d01
        u = (d11 * d20 - d01 * d21) / den
        v = (d00 * d21 - d01 * d20) / den
        ins = (u >= -tol) & (v >= -tol) & (u + v <= 1 + tol)
        idx = np.flatnonzero(plane)
        out[idx[ins]] = True
    return out


def _on_horizontal_facet(pts, verts, tris, tol=0.0):
    """Points lying (closed) on a facet whose plane is z = const."""
    out = np.zeros(len(pts), bool)
    for a, b, c in tris:
        A, B, C = verts[a], verts[b], verts[c]
        if not (A[2] == B[2] == C[2]):
            continue
        on = pts[:, 2] == A[2]

        def side(P0, P1):
            return (P1[0] - P0[0]) * (pts[:, 1] - P0[1]) - (P1[1] - P0[1]) * (pts[:, 0] - P0[0])
        s1, s2, s3 = side(A, B), side(B, C), side(C, A)
        inside = ((s1 >= -tol) & (s2 >= -tol) & (s3 >= -tol)) | ((s1 <= tol) & (s2 <= tol) & (s3 <= tol))
        out |= on & inside
    return out


@pytest.mark.parametrize("n", [16, 32])
@pytest.mark.parametrize("name", sorted(I.EDGE_CASES))
def test_edge_classification(name, n):
    """Zero odd columns; every centre off the surface agrees with the winding number; a centre
    on a horizontal facet is fluid (open crossing interval); a centre on a vertical facet is
    classified as the centre moved by (+d, -d^2, 0) (edge ownership: left edges and top edges
    own their points)."""
    wl = I.EDGE_CASES[name](n)
    P = _problem(wl, stencils=False)
    assert P.odd_columns() == 0
    solid = (P.types() != 0).ravel()
    pts = cell_centres(wl)
    on = _on_surface(pts, wl.verts, wl.tris)
    off = ~on
    wn = winding_number(pts[off], wl.verts, wl.tris)
    assert np.all(np.abs(wn - np.round(wn)) < 1e-9)
    assert np.array_equal(solid[off], np.round(wn) == 1)
    horiz = _on_horizontal_facet(pts, wl.verts, wl.tris)
    assert not np.any(solid[on & horiz])
    rest = on & ~horiz
    if rest.any():
        h = 2.0 / n
        d = 1e-6 * h
        moved = pts[rest] + np.array([d, -d * d / h, 0.0])
        wm = winding_number(moved, wl.verts, wl.tris)
        assert np.all(np.abs(wm - np.round(wm)) < 1e-6)
        assert np.array_equal(solid[rest], np.round(wm) == 1)
    if name == "aligned":
        assert on.sum() > 0 and (on & horiz).sum() > 0 and rest.sum() > 0
    if name == "vertices":
        # the constructed rays do pass through vertices: some vertex lies on a column centre
        xc = 0.5 * (wl.xf[1:] + wl.xf[:-1])
        yc = 0.5 * (wl.yf[1:] + wl.yf[:-1])
        assert np.any(np.isin(wl.verts[:, 0], xc) & np.isin(wl.verts[:, 1], yc))


def _box_nearest(x, lo, hi):
    """Closed-form nearest surface point of an axis-aligned box from a point inside it and
    the gap to the second-nearest face (to skip ties)."""
    gaps = np.concatenate([x - lo, hi - x])
    order = np.argsort(gaps)
    d = order[0]
    q = x.copy()
    q[d % 3] = lo[d % 3] if d < 3 else hi[d % 3]
    return q, gaps[order[1]] - gaps[order[0]]


def _recompute(P, wl, g, q):
    """Image point, box, clamping, self slot and degenerate test of ghost q recomputed from
    its intercept and normal by their definitions."""
    xc, yc, zc = (0.5 * (f[1:] + f[:-1]) for f in (wl.xf, wl.yf, wl.zf))
    cs = (xc, yc, zc)
    nx, ny, nz = len(xc), len(yc), len(zc)
    t = P.types().ravel()
    cell = int(g["cell"][q])
    ijk = (cell % nx, (cell // nx) % ny, cell // (nx * ny))
    xg = np.array([cs[d][ijk[d]] for d in range(3)])
    bi, nrm = g["bi"][q], g["n"][q]
    on_surface = bool(g["flags"][q] & FLAG_NFALL)
    ip = xg.copy() if on_surface else 2.0 * bi - xg
    lo = []
    for d in range(3):
        if on_surface:
            l0 = ijk[d] if nrm[d] >= 0 else ijk[d] - 1
        else:
            l0 = int(np.searchsorted(cs[d], ip[d], side="right")) - 1
        lo.append(int(np.clip(l0, 0, len(cs[d]) - 2)))
    h = np.array([cs[d][lo[d] + 1] - cs[d][lo[d]] for d in range(3)])
    xi = np.array([(ip[d] - cs[d][lo[d]]) / h[d] for d in range(3)])
    clamped = bool(np.any(xi < 0) or np.any(xi > 1))
    members = []
    for m in range(8):
        a, b, c = m & 1, (m >> 1) & 1, (m >> 2) & 1
        members.append(((lo[2] + c) * ny + lo[1] + b) * nx + lo[0] + a)
    mt = t[members]
    self_m = members.index(cell) if cell in members else -1
    deg = bool(np.any(mt == 2) or not np.any(mt == 0))
    if self_m >= 0 and not deg:
        xb = (bi - np.array([cs[d][lo[d]] for d in range(3)])) / h
        bits = [(self_m >> d) & 1 for d in range(3)]
        fac = [xb[d] if bits[d] else 1.0 - xb[d] for d in range(3)]
        dn = sum(nrm[d] * (1.0 if bits[d] else -1.0) / h[d] * np.prod([fac[e] for e in range(3) if e != d])
                 for d in range(3))
        deg = not (dn < 0.0)
    flags = (FLAG_DEG if deg else 0) | (FLAG_CLAMP if clamped else 0) | (FLAG_NFALL if on_surface else 0)
    if self_m >= 0 and not deg:
        flags |= FLAG_SELF
    return dict(xg=xg, ip=ip, lo=lo, xi=np.clip(xi, 0, 1), members=members, self_m=self_m, flags=flags)


@pytest.mark.parametrize("name", sorted(I.EDGE_CASES))
def test_edge_ghost_branches_follow_their_definitions(name):
    """Every flag bit, image point and stencil member recomputed from the intercept and
    normal; intercepts of the box workloads against the closed-form nearest face."""
    wl = I.EDGE_CASES[name](32)
    P = _problem(wl)
    g = P.ghosts()
    seen = 0
    for q in range(len(g["cell"])):
        r = _recompute(P, wl, g, q)
        assert g["flags"][q] == r["flags"], (q, g["flags"][q], r["flags"])
        assert np.array_equal(g["ip"][q], r["ip"]) or np.max(np.abs(g["ip"][q] - r["ip"])) < 1e-15
        seen |= r["flags"]
        if r["flags"] & FLAG_DEG:
            assert np.all(g["stencil"][q] == -1) and np.all(g["beta"][q] == 0.0)
        else:
            st = g["stencil"][q]
            for m in range(8):
                assert st[m] == (-1 if m == r["self_m"] else r["members"][m])
        if r["flags"] & FLAG_NFALL:
            # on the surface: the centre is its own intercept, the normal is the facet's (an
            # axis for these boxes), and the box lies on the normal's side
            assert np.array_equal(g["bi"][q], r["xg"]) and g["dl"][q] == 0.0
            assert np.sum(np.abs(g["n"][q]) == 1.0) == 1 and np.sum(g["n"][q] == 0.0) == 2
    if name in ("slot", "aligned"):
        # intercepts against the nearest face of the box holding the ghost (ties skipped)
        boxes = [(wl.verts[8 * b:8 * b + 8].min(axis=0), wl.verts[8 * b:8 * b + 8].max(axis=0))
                 for b in range(len(wl.verts) // 8)]
        checked = 0
        for q in range(len(g["cell"])):
            x = _recompute(P, wl, g, q)["xg"]
            for lo, hi in boxes:
                if np.all(x >= lo) and np.all(x <= hi):
                    bi, tie = _box_nearest(x, lo, hi)
                    if tie > 1e-9:
                        assert np.max(np.abs(g["bi"][q] - bi)) < 1e-15
                        checked += 1
        assert checked > 0.5 * len(g["cell"])
    expect = {"slot": FLAG_DEG | FLAG_CLAMP | FLAG_SELF, "aligned": FLAG_NFALL | FLAG_SELF, "vertices": FLAG_SELF}
    assert seen & expect[name] == expect[name]


@pytest.mark.parametrize("name", sorted(I.EDGE_CASES))
def test_edge_weights_reproduce_trilinear_functions(name):
    """For every non-degenerate ghost and trilinear q: sum_{m != g} beta_m q(x_m) +
    beta_g dq/dn(BI) = q(IP'), IP' the image point moved into its box (the clamped point;
    the centre itself for a ghost on the surface)."""
    wl = I.EDGE_CASES[name](32)
    P = _problem(wl)
    g = P.ghosts()
    xc, yc, zc = (0.5 * (f[1:] + f[:-1]) for f in (wl.xf, wl.yf, wl.zf))
    nx, ny = len(xc), len(yc)
    rng = np.random.default_rng(9)
    coef = rng.standard_normal((4, 8))
    nclamped = 0
    for q in range(len(g["cell"])):
        if g["flags"][q] & FLAG_DEG:
            continue
        r = _recompute(P, wl, g, q)
        lo = np.array([xc[r["lo"][0]], yc[r["lo"][1]], zc[r["lo"][2]]])
        hs = np.array([xc[r["lo"][0] + 1], yc[r["lo"][1] + 1], zc[r["lo"][2] + 1]]) - lo
        target = lo + r["xi"] * hs
        nclamped += bool(g["flags"][q] & FLAG_CLAMP)
        st, beta, bg, bi, n = g["stencil"][q], g["beta"][q], g["beta_g"][q], g["bi"][q], g["n"][q]
        assert abs(np.sum(beta[st >= 0]) - 1.0) < 1e-12
        for a in coef:
            def qf(x):
                X, Y, Z = x
                return a[0] + a[1] * X + a[2] * Y + a[3] * Z + a[4] * X * Y + a[5] * Y * Z + a[6] * X * Z + a[7] * X * Y * Z

            def dq(x):
                X, Y, Z = x
                return np.array([a[1] + a[4] * Y + a[6] * Z + a[7] * Y * Z, a[2] + a[4] * X + a[5] * Z + a[7] * X * Z,
                                 a[3] + a[5] * Y + a[6] * X + a[7] * X * Y])
            pts = [np.array([xc[c % nx], yc[(c // nx) % ny], zc[c // (nx * ny)]]) for c in st]
            val = sum(beta[m] * qf(pts[m]) for m in range(8) if st[m] >= 0) + bg * np.dot(n, dq(bi))
            assert abs(val - qf(target)) < 1e-11 * (1.0 + np.max(np.abs(a)) * 10)
    if name == "slot":
        assert nclamped > 0


def _dense_system(P, f):
    """The bordered matrix and right-hand side assembled by dense_bordered_solution (rows
    from their definitions; degenerate ghosts: mean of the fluid 26-neighbours)."""
    held = {}
    solve = np.linalg.solve

    def keep(A, b):
        held["A"], held["b"] = A.copy(), b.copy()
        return solve(A, b)
    np.linalg.solve = keep
    try:
        dense_bordered_solution(P, f)
    finally:
        np.linalg.solve = solve
    return held["A"], held["b"]


@pytest.mark.parametrize("method", ["vcycle", "bicgstab"])
def test_aligned_solve_equals_dense_bordered_solve(method):
    """Ghosts on the surface (one-sided Neumann rows): the multigrid and BiCGStab solutions
    equal the dense solve of the bordered system, with nonzero Neumann data."""
    wl = I.edge_aligned(12)
    P = _problem(wl)
    assert np.sum(P.ghosts()["flags"] & FLAG_NFALL) > 0
    rng = np.random.default_rng(6)
    f = rng.standard_normal(P.shape) * (P.types() == 0)
    P.set_neumann(rng.standard_normal(len(P.ghost_cells())))
    p, st = P.solve(f, rel_tol=1e-13, max_cycles=300, method=method)
    assert st.status == 0
    pd, lam = dense_bordered_solution(P, f)
    act = P.types() != 2
    assert abs(st.lam - lam) <= 1e-11 * max(1.0, abs(lam))
    assert np.max(np.abs(p[act] - pd[act])) <= 1e-10 * np.max(np.abs(pd[act]))


def test_slot_system_is_singular_and_the_solve_satisfies_it():
    """Across a slot narrower than a cell, the image-point box of a ghost on one wall holds
    just that ghost and the ghost facing it on the other wall, so their rows read
    p_A - p_B = -h g_A and p_B - p_A = -h g_B: dependent.  The bordered system is singular
    and consistent only for compatible Neumann data (here g = 0, the projection's).  The
    BiCGStab solution (degenerate ghosts included) satisfies every row of the dense system,
    assembled with the degenerate rows written from their definition."""
    wl = I.edge_slot(12)
    P = _problem(wl)
    assert np.sum(P.ghosts()["flags"] & FLAG_DEG) > 0
    rng = np.random.default_rng(6)
    f = rng.standard_normal(P.shape) * (P.types() == 0)
    A, b = _dense_system(P, f)
    sv = np.linalg.svd(A, compute_uv=False)
    assert np.sum(sv < 1e-10 * sv[0]) >= 1
    p, st = P.solve(f, rel_tol=1e-13, max_cycles=300, method="bicgstab")
    assert st.status == 0
    x = np.concatenate([p.ravel(), [st.lam]])
    assert np.max(np.abs(A @ x - b)) <= 1e-10 * np.max(np.abs(b))
