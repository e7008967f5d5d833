"""Oracle of fresh cells after a body moves (test infrastructure).

Only tests/, the package's smoke check and the benchmark's CPU baseline use this module.
Plain FP64 numpy on top of the C oracle (oracle.c), which already pins classification and
the closest point on the mesh; it shares no code with the GPU library.

Section 2.2 of the paper: when a body moves, cells inside it at the previous step that are
in the fluid now ("fresh cells") carry no history, and their values are set by the same
image-point machinery as the ghost cells, with the body's velocity at the intercept.
Readings (the paper gives no formula):
  fresh    old type ghost or dead, new type fluid.
  BI       closest point of the moved surface to the cell centre (2D: in the cell plane).
  IP       2 x_c - BI: the cell centre is the midpoint of BI and IP, so the value at the
           centre is the mean of the intercept value and the image-point value:
             u_c = (u_BI + u_IP) / 2,  u_IP = sum_m beta_m u_m  (trilinear, Eq. 2)
           over the 8 (2D: 4) cells around IP (per axis the largest centre <= x_IP, clamped
           to [0, n-2]; local coordinates clamped to [0, 1]).  When the fresh cell is one of
           them its own term moves to the left side:
             u_c = (u_BI + sum_{m != c} beta_m u_m) / (2 - beta_c).
           Members take their values from the field before the pass (other fresh cells
           included).  A box with a dead cell or without a fluid cell is degenerate: u_c is
           the mean of the fluid, non-fresh 26-neighbours (u_BI if there is none).
  weights  from the Vandermonde system of Eq. 3 with the plain basis rows, solved by LU.
"""
from __future__ import annotations

import numpy as np

from .oracle import OracleProblem

T_FLUID, T_GHOST, T_DEAD = 0, 1, 2


class FreshOracle:
    """Fresh cells of the move old_types -> P (an OracleProblem classified on the moved mesh)."""

    def __init__(self, old_types: np.ndarray, P: OracleProblem, limit: int | None = None):
        """limit: process only the first `limit` fresh cells (a bounded timing sample)."""
        self.P = P
        self.m = P.metrics()
        self.types = P.types()
        self.nz, self.ny, self.nx = self.types.shape
        self.two_d = self.nz == 1
        self.fresh_mask = (old_types != T_FLUID) & (self.types == T_FLUID)
        self.cells = np.flatnonzero(self.fresh_mask.ravel()).astype(np.int64)
        self.n_all = len(self.cells)
        if limit is not None:
            self.cells = self.cells[:limit]
        n = len(self.cells)
        self.bi = np.zeros((n, 3))
        self.ip = np.zeros((n, 3))
        self.members = np.full((n, 8), -1, dtype=np.int64)
        self.beta = np.zeros((n, 8))
        self.beta_c = np.zeros(n)
        self.degenerate = np.zeros(n, dtype=bool)
        for q, cell in enumerate(self.cells):
            self._one(q, int(cell))

    def _centre(self, cell):
        k, j, i = np.unravel_index(cell, (self.nz, self.ny, self.nx))
        return np.array([self.m["xc"][i], self.m["yc"][j], self.m["zc"][k]])

    def _basis(self, x, y, z):
        if self.two_d:
            return np.array([x * y, x, y, 1.0])
        return np.array([x * y * z, x * y, y * z, x * z, x, y, z, 1.0])

    def _one(self, q, cell):
        xc = self._centre(cell)
        bi, _ = self.P.closest_point(xc)
        if self.two_d:
            bi[2] = xc[2]
        ip = 2.0 * xc - bi
        self.bi[q], self.ip[q] = bi, ip
        lo, xi = [], []
        for c, x in ((self.m["xc"], ip[0]), (self.m["yc"], ip[1]), (self.m["zc"], ip[2])):
            if len(c) == 1:
                lo.append(0)
                xi.append(0.0)
                continue
            i0 = int(np.searchsorted(c, x, side="right")) - 1
            i0 = min(max(i0, 0), len(c) - 2)
            lo.append(i0)
            xi.append(min(max((x - c[i0]) / (c[i0 + 1] - c[i0]), 0.0), 1.0))
        nm = 4 if self.two_d else 8
        V = np.zeros((nm, nm))
        mem = []
        for m in range(nm):
            a, b, c = m & 1, (m >> 1) & 1, (m >> 2) & 1
            mid = int(np.ravel_multi_index((lo[2] + c, lo[1] + b, lo[0] + a), self.types.shape))
            mem.append(mid)
            V[m] = self._basis(float(a), float(b), float(c))
        tf = self.types.ravel()
        if any(tf[x] == T_DEAD for x in mem) or not any(tf[x] == T_FLUID for x in mem):
            self.degenerate[q] = True
            return
        beta = np.linalg.solve(V.T, self._basis(*xi))
        for m in range(nm):
            if mem[m] == cell:
                self.beta_c[q] = beta[m]
            else:
                self.members[q, m] = mem[m]
                self.beta[q, m] = beta[m]

    def fill(self, U, ubi=None):
        """U: (3, nz, ny, nx); returns a copy with every fresh cell set (one pass, members
        from U)."""
        U = np.array(U, dtype=np.float64, copy=True)
        src = [u.ravel().copy() for u in U]
        n = len(self.cells)
        ub = np.zeros((n, 3)) if ubi is None else np.asarray(ubi, dtype=np.float64).reshape(n, 3)
        tf = self.types.ravel()
        fresh = self.fresh_mask.ravel()
        out = np.zeros((n, 3))
        for q, cell in enumerate(self.cells):
            if self.degenerate[q]:
                k, j, i = np.unravel_index(int(cell), self.types.shape)
                acc, cnt = np.zeros(3), 0
                for dk in (-1, 0, 1):
                    for dj in (-1, 0, 1):
                        for di in (-1, 0, 1):
                            kk, jj, ii = k + dk, j + dj, i + di
                            if not (0 <= kk < self.nz and 0 <= jj < self.ny and 0 <= ii < self.nx):
                                continue
                            x = int(np.ravel_multi_index((kk, jj, ii), self.types.shape))
                            if tf[x] == T_FLUID and not fresh[x]:
                                acc += np.array([src[c][x] for c in range(3)])
                                cnt += 1
                out[q] = acc / cnt if cnt else ub[q]
                continue
            s = np.zeros(3)
            for m in range(8):
                x = self.members[q, m]
                if x >= 0:
                    s += self.beta[q, m] * np.array([src[c][x] for c in range(3)])
            out[q] = (ub[q] + s) / (2.0 - self.beta_c[q])
        for q, cell in enumerate(self.cells):
            for c in range(3):
                U[c].ravel()[int(cell)] = out[q, c]
        return U
