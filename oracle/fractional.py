"""Oracle of one whole fractional step (test infrastructure).

Only tests/, the package's smoke check and the benchmark's CPU baseline use this module.
Plain FP64 numpy, written from the method's description; it shares no code with the GPU
library and composes the two oracles that are pinned on their own: the advection-diffusion
half-step (oracle/momentum.py) and the projection (oracle.c).

Section 2.1 splits a time step of the Navier-Stokes equations into an advection-diffusion
equation and a pressure Poisson equation.  The half-step advances cell-centred velocity
components; the projection corrects face-normal velocities.  The paper names the split, not
the variable arrangement, so the composition is a reading (the collocated arrangement with
face-normal velocities on the faces of the cells):

  1. u* = the advection-diffusion half-step of u^n (cell-centred);
  2. U*_f on every interior face = the value at the face of the straight line through the
     two adjacent cell centres (the interpolation the convective term already uses), 0 on
     the walls of the box;
  3. the projection of U*: right-hand side, pressure solve, face correction -> p, U^{n+1};
  4. on fluid cells u^{n+1}_c = u*_c - (dU_{c-1/2} + dU_{c+1/2}) / 2 along each axis, where
     dU_f = U*_f - U^{n+1}_f is the change the projection made on face f (0 on the walls);
     ghost and dead cells keep u* (the next half-step resets the ghost rows).
"""
from __future__ import annotations

import numpy as np

from .momentum import T_FLUID

# component d lives on the faces normal to axis d; its cell index runs along array axis 2 - d
_AXIS = (2, 1, 0)


def cell_to_faces(xf, yf, zf, U):
    """Step 2: three face arrays (u: (nz, ny, nx+1), v: (nz, ny+1, nx), w: (nz+1, ny, nx))."""
    faces = []
    for d, f in enumerate((np.asarray(xf, float), np.asarray(yf, float), np.asarray(zf, float))):
        ax = _AXIS[d]
        comp = np.asarray(U[d], dtype=np.float64)
        n = comp.shape[ax]
        shape = list(comp.shape)
        shape[ax] = n + 1
        out = np.zeros(shape)
        if n > 1:
            c = 0.5 * (f[:-1] + f[1:])
            frac = (f[1:-1] - c[:-1]) / (c[1:] - c[:-1])  # how far face q lies from centre q-1 to q
            bshape = [1, 1, 1]
            bshape[ax] = n - 1
            lo = np.take(comp, np.arange(0, n - 1), axis=ax)
            hi = np.take(comp, np.arange(1, n), axis=ax)
            idx = [slice(None)] * 3
            idx[ax] = slice(1, n)
            out[tuple(idx)] = lo + frac.reshape(bshape) * (hi - lo)
        faces.append(out)
    return faces


def correct_cells(types, Ustar, faces_before, faces_after):
    """Step 4: the cell-centred u^{n+1} from u* and the face fields before and after the
    projection."""
    out = np.array(Ustar, dtype=np.float64, copy=True)
    fluid = np.asarray(types) == T_FLUID
    for d in range(3):
        ax = _AXIS[d]
        dU = np.asarray(faces_before[d], float) - np.asarray(faces_after[d], float)
        n = dU.shape[ax] - 1
        mean = 0.5 * (np.take(dU, np.arange(0, n), axis=ax) + np.take(dU, np.arange(1, n + 1), axis=ax))
        out[d] = np.where(fluid, out[d] - mean, out[d])
    return out


def fractional_step(P, mo, U, Hold, nu, dt, first=False, m=8, mom_rel_tol=1e-10, **project_kw):
    """One whole step on the oracle problem P (classified, stencils built) with the momentum
    oracle mo.  Returns (u^{n+1} cells, H^n, faces U^{n+1}, p, projection stats)."""
    Us, H, _, _ = mo.step(U, Hold, nu, dt, first=first, m=m, rel_tol=mom_rel_tol)
    before = cell_to_faces(P.xf, P.yf, P.zf, Us)
    u1, v1, w1, p, st, _ = P.project(*before, dt=dt, **project_kw)
    U1 = correct_cells(P.types(), Us, before, (u1, v1, w1))
    return U1, H, (u1, v1, w1), p, st
