"""Oracle: adjoint of the pressure solve and the face-coefficient gradient (FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the solver library imports or calls this.

Not in the paper, which never differentiates its solver; this is the gradient of
a loss through the solve of section 3.1 written out from the definition of p*:
  p = A(beta)^+ P f  (zero active mean, 0 in the body),  L = sum_b w_b . p_b.
  * dL/df = mu, with A mu = P w (same symmetric operator, same gauge);
  * dL/dbeta_f = o_f h^-2 (mu_R - mu_L)(p_R - p_L)  (sum over the batch), which is
    -grad(lambda).grad(p) with lambda = -mu;
  * with beta_f = o_f 2/(rho_L + rho_R):  dbeta_f/drho_L = dbeta_f/drho_R = -beta_f^2/2,
    so dL/drho_c = -1/2 sum over the faces f of c of beta_f^2 dL/dbeta_f.
"""
from __future__ import annotations

import numpy as np

from .multigrid import Hierarchy, solve
from .operator import Level, open_faces


def face_gradient(mu, p, lev: Level):
    """(gx, gy, gz) on low faces: o_f h^-2 (mu_hi - mu_lo)(p_hi - p_lo); 0 on closed faces."""
    mu = np.asarray(mu)
    p = np.asarray(p)
    if mu.ndim == 3:
        mu, p = mu[None], p[None]
    h2 = lev.h * lev.h
    ox, oy, oz = open_faces(lev.mask)
    gx = np.zeros(mu.shape[1:])
    gy = np.zeros(mu.shape[1:])
    gz = np.zeros(mu.shape[1:])
    for m_b, p_b in zip(mu, p):
        gx += (m_b - np.roll(m_b, 1, axis=2)) * (p_b - np.roll(p_b, 1, axis=2))
        gy += (m_b - np.roll(m_b, 1, axis=1)) * (p_b - np.roll(p_b, 1, axis=1))
        gz[1:] += (m_b[1:] - m_b[:-1]) * (p_b[1:] - p_b[:-1])
    return (np.where(ox, gx / h2, 0.0), np.where(oy, gy / h2, 0.0), np.where(oz, gz / h2, 0.0))


def density_gradient(g, lev: Level):
    """dL/drho_c = -1/2 sum_{faces f of c} beta_f^2 dL/dbeta_f (faces from rho)."""
    gx, gy, gz = g
    tx = lev.bx ** 2 * gx
    ty = lev.by ** 2 * gy
    tz = lev.bz ** 2 * gz
    tz_hi = np.zeros_like(tz)
    tz_hi[:-1] = tz[1:]
    return -0.5 * (tx + np.roll(tx, -1, axis=2) + ty + np.roll(ty, -1, axis=1) + tz + tz_hi)


def adjoint_solve(hier: Hierarchy, w, tol: float = 1e-12, max_cycles: int = 200):
    """mu_b solving A mu_b = P w_b for every batch item (the operator is symmetric)."""
    w = np.asarray(w, np.float64)
    if w.ndim == 3:
        return solve(hier, w, tol=tol, max_cycles=max_cycles)[0]
    return np.stack([solve(hier, wb, tol=tol, max_cycles=max_cycles)[0] for wb in w])


def gradients(hier: Hierarchy, p, w, tol: float = 1e-12):
    """(dL/df, dL/drho) for L = sum_b w_b . p_b at the converged solutions p."""
    mu = adjoint_solve(hier, w, tol)
    g = face_gradient(mu, p, hier.fine)
    return mu, density_gradient(g, hier.fine)
