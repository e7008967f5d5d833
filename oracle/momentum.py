"""Oracle of the advection-diffusion half-step with Dirichlet ghost rows (test infrastructure).

Only tests/, the package's smoke check and the benchmark's CPU baseline use this module.
It is plain FP64 numpy, written from the paper's description, and shares no code with the
GPU library; it reuses the C oracle (oracle.c) for what that already pins: classification,
body intercepts, image points, interpolation boxes and the 1D grid metrics.

What is computed (Section 2.1: fractional step, central differences on the non-uniform
Cartesian grid, Adams-Bashforth in time, the advection-diffusion equation solved by
scheduled relaxed Jacobi; Section 2.2: ghost cells with the image-point interpolation of
Eq. 2 and Eq. 3, here with the Dirichlet condition at the body intercept):

  velocity  cell-centred components U = (u, v, w), array shape (3, nz, ny, nx); dead
            cells hold 0, ghost cells carry the values of their ghost equations.
  H         convective term -d(u_i u_j)/dx_j in conservative form: face values by linear
            interpolation between the two adjacent centres, flux = (normal velocity at the
            face) x (component at the face) x face area, summed over the six faces and
            divided by the cell volume; no flux through the walls of the box.
  L         the flux-form Laplacian of the pressure operator (same coefficients, no flux
            through the box walls).
  step      Adams-Bashforth for H, Crank-Nicolson for the viscous term:
              (I - a L) u* = u^n + dt (3/2 H^n - 1/2 H^{n-1}) + a L u^n,  a = nu dt / 2,
            on fluid rows (the first step takes H^{n-1} = H^n).  Before H^n and L u^n are
            formed, the ghost rows are applied once to u^n.
  ghost row Dirichlet value u_BI at the body intercept, mirrored image point (BI is the
            midpoint of ghost centre and IP): u_g = 2 u_BI - u_IP, with u_IP from the
            trilinear interpolant of the box whose own row (if the ghost is a member) is the
            Dirichlet condition at BI, i.e. Vandermonde row b(xi_BI):
              u_g + sum_{m != g} beta_m u_m = (2 - beta_g) u_BI,  beta = V^{-T} b(xi_IP).
            A degenerate ghost (dead member or no fluid member) uses the mean of its fluid
            26-neighbours for u_IP.
  SRJ       Jacobi on the fluid rows with a schedule of relaxation factors
              u <- (1 - w_k) u + w_k (b + a sum_f a_f u_nb) / (1 + a sum_f a_f),
            every sweep followed by one pass of the ghost rows (ghost members taken from the
            values before the sweep).  The schedule: the reciprocals of the M Chebyshev
            nodes of the interval [1 - rho, 1 + rho] that holds the spectrum of the
            Jacobi-scaled operator, rho = max a d / (1 + a d), d the diagonal flux sum; this
            is the min-max optimal set of M factors, which the SRJ schemes approach as their
            number of distinct factors grows.  Order: largest and smallest alternately.
"""
from __future__ import annotations

import math

import numpy as np

from .oracle import OracleProblem

T_FLUID, T_GHOST, T_DEAD = 0, 1, 2
GF_DEGENERATE = 1


def srj_rho(metrics: dict, alpha: float) -> float:
    """Half-width of the interval [1 - rho, 1 + rho] containing the spectrum of D^{-1} A for
    A = I - alpha L (Gershgorin: the off-diagonal row sum equals the diagonal flux sum)."""
    d = (np.max(metrics["axm"] + metrics["axp"]) + np.max(metrics["aym"] + metrics["ayp"])
         + np.max(metrics["azm"] + metrics["azp"]))
    ad = alpha * d
    return ad / (1.0 + ad)


def srj_schedule(rho: float, m: int) -> np.ndarray:
    """Relaxation factors 1/kappa_k, kappa_k the Chebyshev nodes of [1 - rho, 1 + rho]
    (kappa_k = 1 + rho cos((2k - 1) pi / (2m)), k = 1..m), ordered largest factor, smallest
    factor, second largest, second smallest, ..."""
    k = np.arange(1, m + 1)
    kappa = 1.0 + rho * np.cos((2 * k - 1) * np.pi / (2 * m))
    w = np.sort(1.0 / kappa)[::-1]  # descending
    out = []
    lo, hi = 0, m - 1
    while lo <= hi:
        out.append(w[lo])
        if lo != hi:
            out.append(w[hi])
        lo += 1
        hi -= 1
    return np.array(out)


def srj_cycle_bound(rho: float, m: int) -> float:
    """max over [1 - rho, 1 + rho] of |prod_k (1 - kappa / kappa_k)| for the Chebyshev
    nodes: 1 / T_m(1 / rho)."""
    return 1.0 / math.cosh(m * math.acosh(1.0 / rho)) if rho > 0.0 else 0.0


class MomentumOracle:
    """Advection-diffusion half-step on an OracleProblem with classification and stencils."""

    def __init__(self, P: OracleProblem):
        self.P = P
        self.nx, self.ny, self.nz = P.nx, P.ny, P.nz
        self.two_d = P.nz == 1
        self.m = P.metrics()
        self.types = P.types()
        self.G = P.ghosts()
        self.xf, self.yf, self.zf = P.xf, P.yf, P.zf
        self.wx, self.wy, self.wz = np.diff(P.xf), np.diff(P.yf), np.diff(P.zf)
        self.vol = (self.wz[:, None, None] * self.wy[None, :, None]) * self.wx[None, None, :]
        self._weights()

    # -------------------------------------------------------------------------------- ghosts
    def _box(self, ip):
        """Lower corner of the interpolation box of an image point and its local
        coordinates (per axis: the largest centre index with x_i <= x_IP, clamped to
        [0, n - 2]; local coordinate clamped to [0, 1])."""
        lo, xi = [], []
        for c, x in ((self.m["xc"], ip[0]), (self.m["yc"], ip[1]), (self.m["zc"], ip[2])):
            n = len(c)
            if n == 1:
                lo.append(0)
                xi.append(0.0)
                continue
            i0 = int(np.searchsorted(c, x, side="right")) - 1
            i0 = min(max(i0, 0), n - 2)
            lo.append(i0)
            xi.append(min(max((x - c[i0]) / (c[i0 + 1] - c[i0]), 0.0), 1.0))
        return lo, xi

    def _local(self, lo, x):
        out = []
        for d, c in enumerate((self.m["xc"], self.m["yc"], self.m["zc"])):
            if len(c) == 1:
                out.append(0.0)
            else:
                out.append((x[d] - c[lo[d]]) / (c[lo[d] + 1] - c[lo[d]]))
        return out

    def _basis(self, x, y, z):
        if self.two_d:
            return np.array([x * y, x, y, 1.0])
        return np.array([x * y * z, x * y, y * z, x * z, x, y, z, 1.0])

    def _weights(self):
        """Dirichlet weights of every non-degenerate ghost by LU of the transposed
        Vandermonde system (Eq. 3 with the Dirichlet row at BI)."""
        G = self.G
        ng = len(G["cell"])
        nm = 4 if self.two_d else 8
        self.beta = np.zeros((ng, 8))
        self.beta_g = np.zeros(ng)
        self.members = np.full((ng, 8), -1, dtype=np.int64)
        self.degenerate = (G["flags"] & GF_DEGENERATE) != 0
        shp = (self.nz, self.ny, self.nx)
        for g in range(ng):
            if self.degenerate[g]:
                continue
            lo, xi = self._box(G["ip"][g])
            xb = self._local(lo, G["bi"][g])
            cell = int(G["cell"][g])
            V = np.zeros((nm, nm))
            self_slot = -1
            for m in range(nm):
                a, b, c = m & 1, (m >> 1) & 1, (m >> 2) & 1
                mid = int(np.ravel_multi_index((lo[2] + c, lo[1] + b, lo[0] + a), shp))
                if mid == cell:
                    self_slot = m
                    V[m] = self._basis(*xb)
                else:
                    self.members[g, m] = mid
                    V[m] = self._basis(float(a), float(b), float(c))
            # the box must be the one of the Neumann stencil (same members, same own slot)
            assert np.array_equal(np.where(self.members[g, :nm] >= 0, self.members[g, :nm], -1),
                                  np.where(G["stencil"][g, :nm] >= 0, G["stencil"][g, :nm], -1))
            beta = np.linalg.solve(V.T, self._basis(*xi))
            for m in range(nm):
                if m == self_slot:
                    self.beta_g[g] = beta[m]
                else:
                    self.beta[g, m] = beta[m]

    def _fluid_neighbour_mean(self, U, cell):
        k, j, i = np.unravel_index(cell, (self.nz, self.ny, self.nx))
        sl = (slice(max(k - 1, 0), k + 2), slice(max(j - 1, 0), j + 2), slice(max(i - 1, 0), i + 2))
        fl = self.types[sl] == T_FLUID
        n = int(fl.sum())
        return np.array([U[q][sl][fl].sum() / n if n else 0.0 for q in range(3)])

    def ghost_rows(self, U, ubi=None, src=None):
        """One pass of the Dirichlet ghost rows: u_g = (2 - beta_g) u_BI - sum beta_m u_m,
        fluid members from U, ghost members from src (the values before the pass; U itself
        when src is None)."""
        U = np.array(U, dtype=np.float64, copy=True)
        S = U if src is None else src
        ng = len(self.G["cell"])
        ub = np.zeros((ng, 3)) if ubi is None else np.asarray(ubi, dtype=np.float64).reshape(ng, 3)
        Uf = [u.ravel() for u in U]
        Sf = [s.ravel() for s in S]
        tf = self.types.ravel()
        new = np.zeros((ng, 3))
        for g in range(ng):
            cell = int(self.G["cell"][g])
            if self.degenerate[g]:
                new[g] = 2.0 * ub[g] - self._fluid_neighbour_mean(U, cell)
                continue
            acc = np.zeros(3)
            for m in range(8):
                q = self.members[g, m]
                if q < 0:
                    continue
                src_f = Sf if tf[q] == T_GHOST else Uf
                acc += self.beta[g, m] * np.array([src_f[c][q] for c in range(3)])
            new[g] = (2.0 - self.beta_g[g]) * ub[g] - acc
        for g in range(ng):
            cell = int(self.G["cell"][g])
            for c in range(3):
                Uf[c][cell] = new[g, c]
        return U

    # -------------------------------------------------------------------------- operators
    def laplacian(self, phi):
        """(L phi)_c = sum over the six faces of a_f (phi_nb - phi_c); a_f per unit volume,
        no flux through the box walls."""
        m = self.m
        out = np.zeros_like(phi)
        if self.nx > 1:
            d = phi[:, :, 1:] - phi[:, :, :-1]
            out[:, :, :-1] += m["axp"][None, None, :-1] * d
            out[:, :, 1:] -= m["axm"][None, None, 1:] * d
        if self.ny > 1:
            d = phi[:, 1:, :] - phi[:, :-1, :]
            out[:, :-1, :] += m["ayp"][None, :-1, None] * d
            out[:, 1:, :] -= m["aym"][None, 1:, None] * d
        if self.nz > 1:
            d = phi[1:] - phi[:-1]
            out[:-1] += m["azp"][:-1, None, None] * d
            out[1:] -= m["azm"][1:, None, None] * d
        return out

    def neighbour_sum(self, phi):
        """sum over the six faces of a_f phi_nb (no wall faces)."""
        m = self.m
        out = np.zeros_like(phi)
        if self.nx > 1:
            out[:, :, :-1] += m["axp"][None, None, :-1] * phi[:, :, 1:]
            out[:, :, 1:] += m["axm"][None, None, 1:] * phi[:, :, :-1]
        if self.ny > 1:
            out[:, :-1, :] += m["ayp"][None, :-1, None] * phi[:, 1:, :]
            out[:, 1:, :] += m["aym"][None, 1:, None] * phi[:, :-1, :]
        if self.nz > 1:
            out[:-1] += m["azp"][:-1, None, None] * phi[1:]
            out[1:] += m["azm"][1:, None, None] * phi[:-1]
        return out

    def diag_sum(self):
        """sum_f a_f per cell (wall faces excluded)."""
        m = self.m
        dx = m["axm"].copy()
        dx[0] = 0.0
        px = m["axp"].copy()
        px[-1] = 0.0
        dy = m["aym"].copy()
        dy[0] = 0.0
        py = m["ayp"].copy()
        py[-1] = 0.0
        dz = m["azm"].copy()
        dz[0] = 0.0
        pz = m["azp"].copy()
        pz[-1] = 0.0
        if self.nz == 1:
            dz[:] = 0.0
            pz[:] = 0.0
        return (dz + pz)[:, None, None] + (dy + py)[None, :, None] + (dx + px)[None, None, :]

    def _face_interp(self, c, f):
        """Weights (w_lo, w_hi) of the linear interpolation to the interior faces f[1:-1]
        from the centres on either side."""
        h = c[1:] - c[:-1]
        return (c[1:] - f[1:-1]) / h, (f[1:-1] - c[:-1]) / h

    def convective(self, U):
        """H_i = -(1/V) sum_faces +/- A_f U_n,f (u_i)_f, interior faces only."""
        u = U
        H = np.zeros_like(u)
        # x faces
        if self.nx > 1:
            wl, wh = self._face_interp(self.m["xc"], self.xf)
            face = wl[None, None, None, :] * u[:, :, :, :-1] + wh[None, None, None, :] * u[:, :, :, 1:]
            area = (self.wz[:, None] * self.wy[None, :])[None, :, :, None]
            flux = face[0][None] * face * area
            H[:, :, :, :-1] -= flux
            H[:, :, :, 1:] += flux
        if self.ny > 1:
            wl, wh = self._face_interp(self.m["yc"], self.yf)
            face = wl[None, None, :, None] * u[:, :, :-1, :] + wh[None, None, :, None] * u[:, :, 1:, :]
            area = (self.wz[:, None] * self.wx[None, :])[None, :, None, :]
            flux = face[1][None] * face * area
            H[:, :, :-1, :] -= flux
            H[:, :, 1:, :] += flux
        if self.nz > 1:
            wl, wh = self._face_interp(self.m["zc"], self.zf)
            face = wl[None, :, None, None] * u[:, :-1] + wh[None, :, None, None] * u[:, 1:]
            area = (self.wy[:, None] * self.wx[None, :])[None, None, :, :]
            flux = face[2][None] * face * area
            H[:, :-1] -= flux
            H[:, 1:] += flux
        H /= self.vol[None]
        H[:, self.types != T_FLUID] = 0.0
        return H

    def cn_rhs(self, U, H, Hold, nu, dt, first):
        a = 0.5 * nu * dt
        Hp = H if first else Hold
        b = U + dt * (1.5 * H - 0.5 * Hp) + a * np.stack([self.laplacian(U[q]) for q in range(3)])
        b[:, self.types != T_FLUID] = 0.0
        return b

    # ------------------------------------------------------------------------------ solve
    def srj_sweep(self, U, b, alpha, omega, ubi=None):
        """One relaxed Jacobi sweep of the fluid rows, then one pass of the ghost rows.
        Returns the new iterate and sum over fluid rows of r^2 at the input iterate."""
        fl = self.types == T_FLUID
        ds = self.diag_sum()
        new = np.array(U, copy=True)
        r2 = 0.0
        for q in range(3):
            num = b[q] + alpha * self.neighbour_sum(U[q])
            den = 1.0 + alpha * ds
            r = num - den * U[q]
            r2 += float(np.sum(r[fl] ** 2))
            upd = (1.0 - omega) * U[q] + omega * (num / den)
            new[q][fl] = upd[fl]
        new = self.ghost_rows(new, ubi, src=U)
        return new, r2

    def solve(self, b, U0, alpha, omegas, ubi=None, rel_tol=1e-10, max_cycles=200, fixed_cycles=0):
        """SRJ cycles (each the whole schedule) from U0.  The stop test after a cycle uses
        the residual of the input of its last sweep."""
        fl = self.types == T_FLUID
        bn = math.sqrt(float(sum(np.sum(b[q][fl] ** 2) for q in range(3))))
        U = np.array(U0, copy=True)
        hist = []
        ncyc = fixed_cycles if fixed_cycles > 0 else max_cycles
        cycles = 0
        rel = float("nan")
        for _ in range(ncyc):
            for w in omegas:
                U, r2 = self.srj_sweep(U, b, alpha, w, ubi)
            cycles += 1
            rel = math.sqrt(r2) / bn if bn > 0 else 0.0
            hist.append(rel)
            if fixed_cycles <= 0 and rel <= rel_tol:
                break
        return U, cycles, rel, np.array(hist)

    def step(self, U, Hold, nu, dt, first=False, omegas=None, m=8, ubi=None, rel_tol=1e-10, max_cycles=200,
             fixed_cycles=0):
        """One half-step: ghost rows on u^n, H^n, right-hand side, SRJ solve.  Returns
        (u*, H^n, cycles, rel)."""
        U = np.array(U, dtype=np.float64, copy=True)
        U[:, self.types == T_DEAD] = 0.0
        U = self.ghost_rows(U, ubi, src=U.copy())
        H = self.convective(U)
        b = self.cn_rhs(U, H, Hold, nu, dt, first)
        alpha = 0.5 * nu * dt
        if omegas is None:
            omegas = srj_schedule(srj_rho(self.m, alpha), m)
        Us, cycles, rel, _ = self.solve(b, U, alpha, omegas, ubi, rel_tol, max_cycles, fixed_cycles)
        return Us, H, cycles, rel

    # --------------------------------------------------------------- assembled system (pin)
    def assemble(self, alpha):
        """Sparse matrix of one component's system over all cells: fluid rows
        (1 + a d) u_c - a sum a_f u_nb, ghost rows u_g + sum beta_m u_m (degenerate: + mean
        of the fluid neighbours), dead rows identity."""
        import scipy.sparse as sp
        nz, ny, nx = self.types.shape
        N = nx * ny * nz
        tf = self.types.ravel()
        rows, cols, vals = [], [], []
        ds = self.diag_sum().ravel()
        m = self.m
        idx = np.arange(N).reshape(nz, ny, nx)

        def add(r, c, v):
            rows.append(r)
            cols.append(c)
            vals.append(v)
        fl = np.flatnonzero(tf == T_FLUID)
        add(fl, fl, 1.0 + alpha * ds[fl])
        kk, jj, ii = np.unravel_index(fl, (nz, ny, nx))
        for cond, nb, coef in ((ii > 0, fl - 1, m["axm"][ii]), (ii < nx - 1, fl + 1, m["axp"][ii]),
                               (jj > 0, fl - nx, m["aym"][jj]), (jj < ny - 1, fl + nx, m["ayp"][jj]),
                               (kk > 0, fl - nx * ny, m["azm"][kk]), (kk < nz - 1, fl + nx * ny, m["azp"][kk])):
            add(fl[cond], nb[cond], -alpha * coef[cond])
        dead = np.flatnonzero(tf == T_DEAD)
        add(dead, dead, np.ones(len(dead)))
        for g, cell in enumerate(self.G["cell"]):
            cell = int(cell)
            add(np.array([cell]), np.array([cell]), np.array([1.0]))
            if self.degenerate[g]:
                k, j, i = np.unravel_index(cell, (nz, ny, nx))
                sl = (slice(max(k - 1, 0), k + 2), slice(max(j - 1, 0), j + 2), slice(max(i - 1, 0), i + 2))
                nbs = idx[sl][self.types[sl] == T_FLUID]
                if len(nbs):
                    add(np.full(len(nbs), cell), nbs, np.full(len(nbs), 1.0 / len(nbs)))
                continue
            mem = self.members[g]
            sel = mem >= 0
            add(np.full(int(sel.sum()), cell), mem[sel], self.beta[g][sel])
        r = np.concatenate([np.atleast_1d(x) for x in rows])
        c = np.concatenate([np.atleast_1d(x) for x in cols])
        v = np.concatenate([np.atleast_1d(x) for x in vals])
        return sp.csr_matrix((v, (r, c)), shape=(N, N))

    def exact_solve(self, b, alpha, ubi=None):
        """Direct sparse solve of the three component systems (scipy)."""
        import scipy.sparse.linalg as spl
        A = self.assemble(alpha)
        ng = len(self.G["cell"])
        ub = np.zeros((ng, 3)) if ubi is None else np.asarray(ubi, dtype=np.float64).reshape(ng, 3)
        out = np.zeros_like(b)
        for q in range(3):
            rhs = np.array(b[q], copy=True).ravel()
            rhs[self.types.ravel() != T_FLUID] = 0.0
            for g, cell in enumerate(self.G["cell"]):
                rhs[int(cell)] = (2.0 * ub[g, q] if self.degenerate[g]
                                  else (2.0 - self.beta_g[g]) * ub[g, q])
            out[q] = spl.spsolve(A.tocsc(), rhs).reshape(b[q].shape)
        return out
