"""Oracle: direct solvers for the discrete pressure Poisson problem (FP64).

TEST INFRASTRUCTURE ONLY.  Nothing in the solver library imports or calls this.

Multigrid converges to one exactly defined vector, so the plain definition of the
result is a linear solve:  p* is the unique vector with
    A p* = P f,   sum over active cells of p* = 0,   p* = 0 in the body,
where A is the finite-volume operator of eq. (integral2) (see oracle.operator) and
P f removes the active mean of f (the compatibility condition implied by mass
conservation, eq. (mass), on a closed domain).  Three independent routes:
  * bordered dense system (numpy.linalg.solve), tiny grids;
  * bordered sparse system (scipy.sparse.linalg.spsolve), up to about 32^3;
  * FFT in x, y plus a tridiagonal (Thomas) solve in z, for coefficients that
    depend on z only and no body (the flat-interface workloads), any size.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operator import Level, assemble, project


def _bordered(A, mask):
    """[[A + I_body, 1_active], [1_active^T, 0]]: pins p = 0 in the body and the gauge."""
    m = mask.ravel().astype(np.float64)
    n = m.size
    body = sp.diags(1.0 - m)
    top = sp.hstack([A + body, sp.csr_matrix(m.reshape(n, 1))])
    bot = sp.hstack([sp.csr_matrix(m.reshape(1, n)), sp.csr_matrix((1, 1))])
    return sp.vstack([top, bot]).tocsr()


def solve_dense(lev: Level, f):
    M = _bordered(assemble(lev), lev.mask).toarray()
    rhs = np.concatenate([project(np.asarray(f, np.float64), lev.mask).ravel(), [0.0]])
    x = np.linalg.solve(M, rhs)
    return x[:-1].reshape(f.shape)


def solve_sparse(lev: Level, f):
    M = _bordered(assemble(lev), lev.mask).tocsc()
    rhs = np.concatenate([project(np.asarray(f, np.float64), lev.mask).ravel(), [0.0]])
    x = spla.spsolve(M, rhs, permc_spec="MMD_AT_PLUS_A")   # symmetric fill-reducing order
    return x[:-1].reshape(f.shape)


def z_profiles(lev: Level):
    """(bx_k, by_k, bz_k) if the coefficients depend on k only and there is no body."""
    if not lev.mask.all():
        raise ValueError("FFT solver needs a body-free grid")
    out = []
    for b in (lev.bx, lev.by, lev.bz):
        col = b[:, :1, :1]
        if not np.array_equal(b, np.broadcast_to(col, b.shape)):
            raise ValueError("FFT solver needs coefficients that depend on z only")
        out.append(col[:, 0, 0].copy())
    return out


def solve_fft_z(lev: Level, f):
    """Exact solve for z-only coefficients: 2-D real FFT in (y, x), Thomas in z.

    Mode (a, b) turns the x and y second differences into -4 sin^2(pi a/N) and
    -4 sin^2(pi b/N); what is left is one tridiagonal system in z per mode, strictly
    diagonally dominant except for the mean mode (0, 0), which is the 1-D Neumann
    problem solved by integrating the face flux from the bottom wall.
    """
    bxk, byk, bzk = z_profiles(lev)
    N = lev.N
    h2 = lev.h * lev.h
    fh = np.fft.rfft2(project(np.asarray(f, np.float64), lev.mask), axes=(1, 2))  # [k, b, a]
    a = np.arange(N // 2 + 1)
    b = np.arange(N)
    sa = np.sin(np.pi * a / N) ** 2
    sb = np.sin(np.pi * b / N) ** 2
    lower = bzk / h2                                   # coupling of k to k-1 (0 at k=0)
    upper = np.concatenate([bzk[1:], [0.0]]) / h2      # coupling of k to k+1 (0 at top)
    shift = 4.0 * (byk[:, None, None] * sb[None, :, None] + bxk[:, None, None] * sa[None, None, :]) / h2
    diag = -(lower + upper)[:, None, None] - shift     # [k, b, a]
    # Thomas elimination over k, vectorised over modes (mode (0,0) handled below).
    d = diag.astype(np.complex128).copy()
    r = fh.copy()
    d[:, 0, 0] = 1.0                                   # placeholder, overwritten below
    for k in range(1, N):
        w = lower[k] / d[k - 1]
        d[k] = d[k] - w * upper[k - 1]
        r[k] = r[k] - w * r[k - 1]
    x = np.empty_like(r)
    x[N - 1] = r[N - 1] / d[N - 1]
    for k in range(N - 2, -1, -1):
        x[k] = (r[k] - upper[k] * x[k + 1]) / d[k]
    # mean mode: h^-2 (F_{k+1} - F_k) = f_k with F_k = bz_k (p_k - p_{k-1}), F_0 = 0
    f00 = fh[:, 0, 0]
    F = np.concatenate([[0.0], np.cumsum(h2 * f00)])   # F[k] for k = 0..N
    p00 = np.zeros(N, dtype=np.complex128)
    for k in range(1, N):
        p00[k] = p00[k - 1] + F[k] / bzk[k]
    x[:, 0, 0] = p00
    p = np.fft.irfft2(x, s=(N, N), axes=(1, 2))
    return p - p.mean()
