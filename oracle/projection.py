"""Oracle: the two steps either side of the pressure solve (FP64, numpy).

TEST INFRASTRUCTURE ONLY.  Nothing in the solver library imports or calls this.

Paper section 2.1: each Runge-Kutta stage solves the Poisson equation with the
divergence of (u/dt + R) as source (eqs. (poisson1), (poisson2)) and then projects the
velocity with the pressure gradient scaled by 1/rho (eqs. (runge1), (runge2)).  In the
finite-volume form of eq. (integral2) the velocity lives on cell faces (the normal
component, low-face storage like the face coefficients), so that:
  * divergence  f_c = (1/h) sum over the faces of c of (+-) (U_f + dt R_f) / dt, the sign
    + on the high face and - on the low face; closed faces (body, walls) carry no flux;
  * projection  U_f <- o_f (U_f + dt R_f - dt beta_f (p_hi - p_lo) / h).
With beta_f the face product of the solve, div(projected U) = div(U + dt R) - dt A p,
which vanishes when A p = div(U + dt R) / dt: the discrete projection is exact.
"""
from __future__ import annotations

import numpy as np

from .operator import Level, open_faces


def predicted(u, r, dt):
    """U + dt R on every face (R may be None)."""
    if r is None:
        return tuple(np.asarray(c, np.float64) for c in u)
    return tuple(np.asarray(a, np.float64) + dt * np.asarray(b, np.float64) for a, b in zip(u, r))


def divergence(u, lev: Level, dt: float = 1.0, r=None):
    """f_c = div(U + dt R)_c / dt on active cells, 0 elsewhere."""
    ux, uy, uz = predicted(u, r, dt)
    ox, oy, oz = open_faces(lev.mask)
    Fx = np.where(ox, ux, 0.0)
    Fy = np.where(oy, uy, 0.0)
    Fz = np.where(oz, uz, 0.0)
    Fz_hi = np.zeros_like(Fz)
    Fz_hi[:-1] = Fz[1:]
    div = (np.roll(Fx, -1, axis=2) - Fx) + (np.roll(Fy, -1, axis=1) - Fy) + (Fz_hi - Fz)
    return np.where(lev.mask, div / (lev.h * dt), 0.0)


def project(u, p, lev: Level, dt: float = 1.0, r=None):
    """U_f <- o_f (U_f + dt R_f - dt beta_f (p_hi - p_lo) / h) on the low faces."""
    ux, uy, uz = predicted(u, r, dt)
    ox, oy, oz = open_faces(lev.mask)
    gx = (p - np.roll(p, 1, axis=2)) / lev.h
    gy = (p - np.roll(p, 1, axis=1)) / lev.h
    gz = np.zeros_like(p)
    gz[1:] = (p[1:] - p[:-1]) / lev.h
    return (np.where(ox, ux - dt * lev.bx * gx, 0.0),
            np.where(oy, uy - dt * lev.by * gy, 0.0),
            np.where(oz, uz - dt * lev.bz * gz, 0.0))
