"""Seeded synthetic inputs shared by the HIP path, its tests and the oracle.

This module only *generates* inputs: face coordinates of stretched Cartesian grids,
closed triangulated bodies and face-velocity fields.  It holds none of the method's
arithmetic (no metrics, classification, stencils or solver steps), so it can feed both
the GPU library and the CPU oracle without coupling them.

Workloads follow the paper's cases in shape only (Section 3.2: 2D cylinder, finite
rectangular wing; Section 3.3: multi-body array): the paper's CAD bodies and flow data are
not available, so closed synthetic bodies of the same character stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------------------
# grids
# ----------------------------------------------------------------------------------------


def _grow(h0: float, length: float, ratio: float, ramp: float) -> list[float]:
    """Cell widths growing away from a uniform core until they span ``length``.

    h_k = h_{k-1} * exp(ln(ratio) * tanh(k / ramp)); the list is rescaled so its sum is
    exactly ``length`` (the adjacent ratio stays <= ratio up to that rescale).
    """
    if length <= 0.0:
        return []
    widths: list[float] = []
    h = h0
    total = 0.0
    k = 0
    while total < length:
        k += 1
        h = h * math.exp(math.log(ratio) * math.tanh(k / ramp))
        widths.append(h)
        total += h
    s = length / total
    return [w * s for w in widths]


def stretched_faces(lo: float, hi: float, core_lo: float, core_hi: float, n: int,
                    ratio: float = 1.049, ramp: float = 8.0) -> np.ndarray:
    """Face coordinates (n+1) of a grid that is uniform on [core_lo, core_hi] and
    stretches geometrically (tanh-ramped ratio <= ``ratio``) towards both walls.

    The core cell count is the smallest one for which the total reaches n; surplus cells
    are removed from the ends of the longer side, which is then rescaled to fit.
    """
    assert lo < core_lo < core_hi < hi and n >= 4
    core = core_hi - core_lo
    best = None
    for nc in range(1, n + 1):
        hc = core / nc
        left = _grow(hc, core_lo - lo, ratio, ramp)
        right = _grow(hc, hi - core_hi, ratio, ramp)
        tot = nc + len(left) + len(right)
        if tot >= n:
            best = (nc, left, right, tot)
            break
    if best is None:
        raise ValueError("cannot reach the requested cell count")
    nc, left, right, tot = best
    extra = tot - n
    while extra > 0:
        if len(left) >= len(right) and left:
            left = left[:-1]
            left = [w * (core_lo - lo) / sum(left) for w in left] if left else left
        elif right:
            right = right[:-1]
            right = [w * (hi - core_hi) / sum(right) for w in right] if right else right
        extra -= 1
    hc = core / nc
    widths = list(reversed(left)) + [hc] * nc + right
    assert len(widths) == n
    f = np.empty(n + 1, dtype=np.float64)
    f[0] = lo
    f[1:] = lo + np.cumsum(widths)
    # pin the core ends and the far wall exactly
    nl = len(left)
    f[nl] = core_lo
    f[nl + 1:nl + nc] = core_lo + hc * np.arange(1, nc)
    f[nl + nc] = core_hi
    f[nl + nc + 1:] = core_hi + np.cumsum(right)
    f[-1] = hi
    assert np.all(np.diff(f) > 0)
    return f


def uniform_faces(lo: float, hi: float, n: int) -> np.ndarray:
    return np.linspace(lo, hi, n + 1, dtype=np.float64)


# ----------------------------------------------------------------------------------------
# closed triangle meshes (outward orientation: counter-clockwise seen from outside)
# ----------------------------------------------------------------------------------------


def box_mesh(center=(0.0, 0.0, 0.0), size=(1.0, 2.0, 0.08), pitch_deg: float = 15.0):
    """Rectangular plate (chord along x, span along y, thickness along z) rotated about
    the y axis so the leading edge (x < 0 side) goes up: 8 vertices, 12 triangles."""
    lx, ly, lz = (s / 2.0 for s in size)
    corners = np.array([[sx * lx, sy * ly, sz * lz]
                        for sz in (-1, 1) for sy in (-1, 1) for sx in (-1, 1)], dtype=np.float64)
    # vertex v = ix + 2*iy + 4*iz ; outward quads (CCW from outside)
    quads = [
        (0, 2, 3, 1),  # z-
        (4, 5, 7, 6),  # z+
        (0, 1, 5, 4),  # y-
        (2, 6, 7, 3),  # y+
        (0, 4, 6, 2),  # x-
        (1, 3, 7, 5),  # x+
    ]
    tris = []
    for a, b, c, d in quads:
        tris.append((a, b, c))
        tris.append((a, c, d))
    t = math.radians(pitch_deg)
    # rotation about +y by -t lifts the x<0 edge (leading edge up)
    c, s = math.cos(-t), math.sin(-t)
    rot = np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])
    verts = corners @ rot.T + np.asarray(center, dtype=np.float64)
    return verts.astype(np.float64), np.asarray(tris, dtype=np.int32)


def prism_mesh(radius: float = 0.5, n_sides: int = 256, z0: float = -1.0, z1: float = 1.0,
               center=(0.0, 0.0)):
    """Regular n-gon prism with centre-fan caps (4n triangles): a circular cylinder
    along z for 2D runs."""
    th = 2.0 * math.pi * np.arange(n_sides) / n_sides
    x = center[0] + radius * np.cos(th)
    y = center[1] + radius * np.sin(th)
    bot = np.stack([x, y, np.full(n_sides, z0)], axis=1)
    top = np.stack([x, y, np.full(n_sides, z1)], axis=1)
    verts = np.concatenate([bot, top, [[center[0], center[1], z0]], [[center[0], center[1], z1]]])
    cb, ct = 2 * n_sides, 2 * n_sides + 1
    tris = []
    for i in range(n_sides):
        j = (i + 1) % n_sides
        tris.append((i, j, n_sides + j))
        tris.append((i, n_sides + j, n_sides + i))
        tris.append((cb, j, i))
        tris.append((ct, n_sides + i, n_sides + j))
    return verts.astype(np.float64), np.asarray(tris, dtype=np.int32)


def icosphere(level: int):
    """Unit icosphere by midpoint subdivision: 10*4^level+2 vertices, 20*4^level faces."""
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0), (0, -1, p), (0, 1, p), (0, -1, -p),
         (0, 1, -p), (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    verts = [np.asarray(a, dtype=np.float64) / np.linalg.norm(a) for a in v]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
             (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
             (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    for _ in range(level):
        cache: dict[tuple[int, int], int] = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.asarray(verts, dtype=np.float64), np.asarray(faces, dtype=np.int32)


def _real_sph_harm(l: int, m: int, theta: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Orthonormal real spherical harmonic (theta polar, phi azimuth)."""
    from scipy.special import lpmv
    am = abs(m)
    norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
    leg = lpmv(am, l, np.cos(theta))
    if m == 0:
        return norm * leg
    if m > 0:
        return math.sqrt(2.0) * norm * leg * np.cos(am * phi)
    return math.sqrt(2.0) * norm * leg * np.sin(am * phi)


def perturbed_sphere(rng: np.random.Generator, level: int, radius: float, center,
                     lmax: int = 6, amp: float = 0.15):
    """Icosphere whose radius is R(1 + amp * s / max|s|), s a random real spherical-harmonic
    series with l = 1..lmax and N(0,1) coefficients."""
    v, t = icosphere(level)
    theta = np.arccos(np.clip(v[:, 2], -1.0, 1.0))
    phi = np.arctan2(v[:, 1], v[:, 0])
    s = np.zeros(len(v))
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            s += rng.standard_normal() * _real_sph_harm(l, m, theta, phi)
    r = radius * (1.0 + amp * s / np.max(np.abs(s)))
    verts = v * r[:, None] + np.asarray(center, dtype=np.float64)
    return verts, t


def merge_meshes(meshes):
    vs, ts, off = [], [], 0
    for v, t in meshes:
        vs.append(v)
        ts.append(t + off)
        off += len(v)
    return np.concatenate(vs).astype(np.float64), np.concatenate(ts).astype(np.int32)


def place_bodies(rng: np.random.Generator, k: int, box_lo: float, box_hi: float,
                 rmin: float = 0.3, rmax: float = 0.8, gap: float = 0.1, max_tries: int = 100000):
    """Radii ~ U[rmin, rmax]; centres uniform in the box shrunk by 1.15R; accept a body
    iff its centre is at least 1.15(R_i + R_j) + gap from every accepted one."""
    out = []
    tries = 0
    while len(out) < k:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("body placement failed")
        R = rng.uniform(rmin, rmax)
        m = 1.15 * R
        c = rng.uniform(box_lo + m, box_hi - m, size=3)
        if all(np.linalg.norm(c - c2) >= 1.15 * (R + R2) + gap for c2, R2 in out):
            out.append((c, R))
    return out


# ----------------------------------------------------------------------------------------
# velocity fields (MAC faces)
# ----------------------------------------------------------------------------------------


def face_velocity(seed: int, nx: int, ny: int, nz: int):
    """Face-normal velocities u[nz][ny][nx+1], v[nz][ny+1][nx], w[nz+1][ny][nx]:
    i.i.d. U[-1,1] on interior faces, zero on the domain walls (and w == 0 in 2D)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=(nz, ny, nx + 1))
    v = rng.uniform(-1.0, 1.0, size=(nz, ny + 1, nx))
    w = rng.uniform(-1.0, 1.0, size=(nz + 1, ny, nx))
    u[:, :, 0] = 0.0
    u[:, :, -1] = 0.0
    v[:, 0, :] = 0.0
    v[:, -1, :] = 0.0
    w[0, :, :] = 0.0
    w[-1, :, :] = 0.0
    if nz == 1:
        w[:] = 0.0
    return u, v, w


def cell_velocity(seed: int, nx: int, ny: int, nz: int, n_modes: int = 6, amplitude: float = 1.0):
    """Cell-centred velocity components, shape (3, nz, ny, nx): per component a sum of
    ``n_modes`` seeded low-wavenumber (0..3 per axis) products of cosines in index space,
    scaled so the largest magnitude is ``amplitude``; w == 0 in 2D."""
    rng = np.random.default_rng(seed)
    out = np.zeros((3, nz, ny, nx))
    idx = [(np.arange(n) + 0.5) / n for n in (nx, ny, nz)]
    for c in range(3):
        for _ in range(n_modes):
            kx, ky, kz = rng.integers(0, 4, size=3)
            ph = rng.uniform(0.0, 2.0 * np.pi, size=3)
            a = rng.standard_normal()
            fx = np.cos(2.0 * np.pi * kx * idx[0] + ph[0])
            fy = np.cos(2.0 * np.pi * ky * idx[1] + ph[1])
            fz = np.cos(2.0 * np.pi * kz * idx[2] + ph[2]) if nz > 1 else np.ones(1)
            out[c] += a * (fz[:, None, None] * fy[None, :, None]) * fx[None, None, :]
        mx = np.max(np.abs(out[c]))
        if mx > 0.0:
            out[c] *= amplitude / mx
    if nz == 1:
        out[2] = 0.0
    return out


# ----------------------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------------------


@dataclass
class Workload:
    name: str
    xf: np.ndarray
    yf: np.ndarray
    zf: np.ndarray
    verts: np.ndarray
    tris: np.ndarray
    seed: int
    dt: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (len(self.xf) - 1, len(self.yf) - 1, len(self.zf) - 1)

    @property
    def ncells(self):
        nx, ny, nz = self.shape
        return nx * ny * nz

    def velocity(self):
        nx, ny, nz = self.shape
        return face_velocity(self.seed, nx, ny, nz)

    def cell_fields(self):
        """(u^n, H^{n-1}) of an advection-diffusion step: two seeded smooth cell-centred
        fields of order 1 (seeds 1000 + seed and 2000 + seed)."""
        nx, ny, nz = self.shape
        return (cell_velocity(1000 + self.seed, nx, ny, nz),
                cell_velocity(2000 + self.seed, nx, ny, nz))


def cylinder2d(n: int = 128) -> Workload:
    """2D circular cylinder: uniform n x n on [-8,8]^2, one z cell of width h; circle of
    radius 0.5 at the origin as a 256-gon prism spanning the z cell (Section 3.2.1 shape)."""
    xf = uniform_faces(-8.0, 8.0, n)
    h = 16.0 / n
    zf = np.array([-h / 2.0, h / 2.0])
    v, t = prism_mesh(0.5, 256, -1.0, 1.0)
    return Workload("cylinder2d_%dx%d" % (n, n), xf, xf.copy(), zf, v, t, seed=0)


def wing(nx: int = 256, ny: int = 128, nz: int = 128, seed: int = 1) -> Workload:
    """Finite rectangular wing (Section 3.2.2 shape): plate chord 1, span 2, thickness
    0.08 at 15 degrees on [-5,5]^3, grid uniform on the body bounding box +/- 0.15 and
    stretched (ratio <= 1.05) to the walls."""
    v, t = box_mesh((0.0, 0.0, 0.0), (1.0, 2.0, 0.08), 15.0)
    lo, hi = v.min(axis=0), v.max(axis=0)
    xf = stretched_faces(-5.0, 5.0, lo[0] - 0.15, hi[0] + 0.15, nx)
    yf = stretched_faces(-5.0, 5.0, lo[1] - 0.15, hi[1] + 0.15, ny)
    zf = stretched_faces(-5.0, 5.0, lo[2] - 0.15, hi[2] + 0.15, nz)
    return Workload("wing_%dx%dx%d" % (nx, ny, nz), xf, yf, zf, v, t, seed=seed)


def multibody(n: int = 384, n_bodies: int = 8, level: int = 5, geo_seed: int = 4,
              rhs_seed: int = 40, domain: float = 4.0, core: float = 2.3) -> Workload:
    """Array of closed bodies (Section 3.3.2 shape): ``n_bodies`` perturbed icospheres
    (spherical-harmonic l <= 6, amplitude 0.15R, R ~ U[0.3,0.8]) placed without overlap
    in the core of an n^3 grid on [-domain, domain]^3, uniform core +/- ``core``."""
    rng = np.random.default_rng(geo_seed)
    placed = place_bodies(rng, n_bodies, -core, core)
    meshes = [perturbed_sphere(rng, level, R, c) for c, R in placed]
    v, t = merge_meshes(meshes)
    f = stretched_faces(-domain, domain, -core, core, n)
    return Workload("multibody%d_%d^3" % (n_bodies, n), f, f.copy(), f.copy(), v, t,
                    seed=rhs_seed, meta={"bodies": [(c.tolist(), R) for c, R in placed]})


def serving_request(req_id: int, trace_seed: int = 5, sizes=(64, 128, 192, 256)) -> Workload:
    """One request of the serving stream: grid n^3 with n uniform from ``sizes`` and
    1-4 level-4 perturbed icospheres; seeds derive from the request id."""
    rng = np.random.default_rng([trace_seed, req_id])
    n = int(rng.choice(sizes))
    k = int(rng.integers(1, 5))
    wl = multibody(n=n, n_bodies=k, level=4, geo_seed=int(rng.integers(1 << 30)),
                   rhs_seed=int(rng.integers(1 << 30)))
    wl.name = "req%d_%d^3_%dbody" % (req_id, n, k)
    return wl


def mms_workload(n: int = 32, stretched: bool = False, level: int = 5) -> Workload:
    """Manufactured-solution case on [-1,1]^3: icosphere of radius 0.45 centred at
    (0.05,-0.03,0.02); exact p = cos(pi x) cos(pi y) cos(pi z)."""
    v, t = icosphere(level)
    v = v * 0.45 + np.array([0.05, -0.03, 0.02])
    if stretched:
        f = stretched_faces(-1.0, 1.0, -0.55, 0.55, n, ratio=1.08, ramp=4.0)
    else:
        f = uniform_faces(-1.0, 1.0, n)
    return Workload("mms_%d" % n, f, f.copy(), f.copy(), v, t, seed=0)


def mms_exact(x, y, z):
    return np.cos(np.pi * x) * np.cos(np.pi * y) * np.cos(np.pi * z)


def mms_grad(x, y, z):
    pi = np.pi
    return (-pi * np.sin(pi * x) * np.cos(pi * y) * np.cos(pi * z),
            -pi * np.cos(pi * x) * np.sin(pi * y) * np.cos(pi * z),
            -pi * np.cos(pi * x) * np.cos(pi * y) * np.sin(pi * z))


def mms_source(x, y, z):
    return -3.0 * np.pi ** 2 * mms_exact(x, y, z)


def sphere_small(n: int = 8, radius: float = 0.3, center=(0.07, -0.04, 0.03), level: int = 3) -> Workload:
    """Tiny 3D case for dense brute-force checks: sphere in [-1,1]^3 on an n^3 grid."""
    v, t = icosphere(level)
    v = v * radius + np.asarray(center)
    f = uniform_faces(-1.0, 1.0, n)
    return Workload("sphere%d" % n, f, f.copy(), f.copy(), v, t, seed=7)


# ----------------------------------------------------------------------------------------
# constructed edge cases: bodies placed on the grid so that every special branch of the
# classification and of the ghost stencils is taken (uniform n^3 grid on [-1, 1]^3, n even,
# so cell centres -1 + (i + 1/2) h are exact binary fractions)
# ----------------------------------------------------------------------------------------


def aabb_mesh(lo, hi):
    """Axis-aligned box with exactly the given corner coordinates (12 outward triangles)."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    corners = np.array([[(hi if (v >> d) & 1 else lo)[d] for d in range(3)] for v in range(8)], dtype=np.float64)
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    tris = [t for a, b, c, d in quads for t in ((a, b, c), (a, c, d))]
    return corners, np.asarray(tris, dtype=np.int32)


def convex_hull_mesh(verts, faces):
    """The given triangles of a convex polyhedron, each reordered to face outward (away from
    the vertex centroid)."""
    v = np.asarray(verts, dtype=np.float64)
    c = v.mean(axis=0)
    out = []
    for a, b, d in faces:
        nrm = np.cross(v[b] - v[a], v[d] - v[a])
        out.append((a, b, d) if np.dot(nrm, v[a] - c) > 0 else (a, d, b))
    return v, np.asarray(out, dtype=np.int32)


def _centres(n):
    h = 2.0 / n
    return h, -1.0 + h * (np.arange(n) + 0.5)


def edge_slot(n: int = 32) -> Workload:
    """Two boxes separated by a slot narrower than a cell (no cell centre in it), so the
    image points of the ghost cells along the slot mouth fall into solid boxes (degenerate
    ghosts); the left box ends 0.7 h from the x = -1 wall, so the image points of its wall-side
    ghosts lie beyond the outermost cell centre (clamped)."""
    h, _ = _centres(n)
    ylo, yhi, zlo, zhi = -1.0 + 2.3 * h, 1.0 - 3.4 * h, -1.0 + 2.6 * h, 1.0 - 2.2 * h
    a = aabb_mesh((-1.0 + 0.7 * h, ylo, zlo), (-0.32 * h, yhi, zhi))
    b = aabb_mesh((0.32 * h, ylo, zlo), (1.0 - 1.7 * h, yhi, zhi))
    v, t = merge_meshes([a, b])
    f = uniform_faces(-1.0, 1.0, n)
    return Workload("edge_slot_%d" % n, f, f.copy(), f.copy(), v, t, seed=11)


def edge_aligned(n: int = 32) -> Workload:
    """Boxes whose faces pass exactly through cell centres: box 1 its x and z faces, box 2 its
    y faces (the others between centres).  Centres on the surface are classified by the
    edge-ownership rule (x and y faces) and the open crossing interval (z faces); the ghosts
    on the surface take the facet normal."""
    h, c = _centres(n)

    def at(k32):  # the cell centre at k/32 of the grid
        return c[int(k32 * n) // 32]

    b1 = aabb_mesh((at(6), -1.0 + 0.29 * 2.0 + 0.3 * h, at(10)), (at(20), 1.0 - 0.27 * 2.0 - 0.4 * h, at(21)))
    b2 = aabb_mesh((1.0 - 0.23 * 2.0 - 0.4 * h, at(7), -1.0 + 0.3 * 2.0 + 0.3 * h),
                   (1.0 - 0.07 * 2.0 - 0.3 * h, at(23), 1.0 - 0.32 * 2.0 - 0.2 * h))
    v, t = merge_meshes([b1, b2])
    f = uniform_faces(-1.0, 1.0, n)
    return Workload("edge_aligned_%d" % n, f, f.copy(), f.copy(), v, t, seed=12)


def edge_vertices(n: int = 32) -> Workload:
    """An octahedron and a tetrahedron whose vertices lie on column centres (x_i, y_j), with
    z between centres, so column rays pass exactly through vertices and along projected
    edges."""
    h, c = _centres(n)

    def at(k32):
        return c[int(k32 * n) // 32]

    i0, j0 = int(10 * n) // 32, int(9 * n) // 32
    m = max(2, int(6 * n) // 32)  # equatorial half-width in cells
    xo, yo, zo, a, b = c[i0], c[j0], -1.0 + 2 * (n // 5) * (2.0 / n) / 2.0, m * h, 5.37 * h * max(1, n // 32)
    ov = [(xo + a, yo, zo), (xo - a, yo, zo), (xo, yo + a, zo), (xo, yo - a, zo), (xo, yo, zo + b), (xo, yo, zo - b)]
    of = [(0, 2, 4), (2, 1, 4), (1, 3, 4), (3, 0, 4), (2, 0, 5), (1, 2, 5), (3, 1, 5), (0, 3, 5)]
    oct_ = convex_hull_mesh(ov, of)
    tv = [(at(18), at(17), 0.23 + 0.5 * h), (at(28), at(20), 0.41), (at(20), at(28), 0.37), (at(22), at(22), 0.93 - 0.2 * h)]
    tet = convex_hull_mesh(tv, [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)])
    v, t = merge_meshes([oct_, tet])
    f = uniform_faces(-1.0, 1.0, n)
    return Workload("edge_vertices_%d" % n, f, f.copy(), f.copy(), v, t, seed=13)


EDGE_CASES = {"slot": edge_slot, "aligned": edge_aligned, "vertices": edge_vertices}


CONFIGS = {
    "cylinder2d": lambda: cylinder2d(128),
    "wing": lambda: wing(256, 128, 128, seed=1),
    "wing_large": lambda: wing(512, 256, 256, seed=2),
    "multibody384": lambda: multibody(384),
    "multibody256": lambda: multibody(256),
}
