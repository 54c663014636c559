"""Oracle: geometric multigrid for the pressure Poisson equation (numpy, FP64/FP32).

TEST INFRASTRUCTURE ONLY.  Nothing in the solver library imports or calls this.

Paper section 3.1 fixes only the idea: fine grids remove high-wavenumber residual
error, coarse grids low-wavenumber error, and the face product (1/rho) x (cut area)
is formed on the finest grid and moved to the coarse grids as one unit (rather than
restricting the cell-centre density, which over-smooths a sharp interface).  Every
other choice is a reading, written here plainly:
  * smoother: red-black Gauss-Seidel, red = (i + j + k) even; pre-smoothing runs
    red then black, post-smoothing black then red; cells with no open face skipped;
  * cycle: V(2,2), one V-cycle per outer iteration;
  * restriction: mean of the 8 children (cell-centred full weighting);
  * prolongation: trilinear, 1-D weights 3/4 (parent) and 1/4 (nearer neighbour),
    periodic in x and y, the parent standing in for a missing z neighbour;
    corrections are added on active fine cells only;
  * coefficient coarsening: a coarse face takes the mean of its 4 coincident fine
    faces; a coarse cell is active when any child is active and it keeps an open face;
    the spacing doubles;
  * coarsest grid 4^3, solved with the FP64 pseudo-inverse of its dense operator
    (symmetric eigendecomposition, eigenvalues below 1e-12 max|lambda| dropped) after
    removing the active mean of the right-hand side;
  * stopping: relative residual ||P f - A p||_2 / ||P f||_2 after every cycle;
  * gauge: the returned p has zero mean over active cells and is 0 in the body.
Mixed precision (not in the paper): one FP32 V-cycle per step of FP64 iterative
refinement; the residual, the update and the coarsest solve stay FP64.  The FP32 face
coefficients of the coarse grids are the FP64 ones rounded to nearest; the finest FP32
grid either rounds its FP64 coefficients too (fp32_levels) or forms them in single
precision from fl32(rho) (fp32_levels_from_rho), within two float32 ulps of rounding.

Pins: every step (smoother, transfers, coarsening, coarsest solve) against closed
forms, identities and library routines, and the converged solution against the exact
solvers of oracle.exact.  Parity unpinned: the convergence rate, i.e. the residual
history cycle by cycle.  The paper prints no history, so only the GPU's agreement
with this module pins it.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .operator import Level, apply, close_faces, diagonal, neighbour_sum, project

COARSEST = 4
PINV_RTOL = 1e-12


def _scalar(x, dtype):
    return dtype.type(x)


def colour_mask(N: int, colour: int) -> np.ndarray:
    k, j, i = np.indices((N, N, N))
    return ((i + j + k) % 2) == colour


RED, BLACK = 0, 1


def rbgs_half(p, f, lev: Level, colour: int):
    """Gauss-Seidel on one colour: p_c <- (S_c - h^2 f_c) / D_c where D_c > 0.

    Cells of one colour only neighbour the other colour, so updating all of them
    at once from the current p is exactly a Gauss-Seidel pass over that colour.
    """
    dt = p.dtype
    D = diagonal(lev)
    S = neighbour_sum(p, lev)
    sel = colour_mask(lev.N, colour) & (D > 0)
    out = p.copy()
    h2 = _scalar(lev.h * lev.h, dt)
    out[sel] = (S[sel] - h2 * f[sel]) / D[sel]
    return out


def smooth(p, f, lev: Level, sweeps: int, order):
    for _ in range(sweeps):
        for colour in order:
            p = rbgs_half(p, f, lev, colour)
    return p


def residual(p, f, lev: Level):
    """r = f - A p on active cells, 0 elsewhere."""
    return np.where(lev.mask, f - apply(p, lev), 0.0).astype(p.dtype, copy=False)


def restrict(r):
    """Coarse value = mean of the 8 children."""
    N = r.shape[0]
    n = N // 2
    return r.reshape(n, 2, n, 2, n, 2).mean(axis=(1, 3, 5)).astype(r.dtype, copy=False)


def _interp_axis(e, axis, periodic):
    """1-D linear interpolation to the children along one axis (weights 3/4, 1/4)."""
    dt = e.dtype
    w3, w1 = _scalar(0.75, dt), _scalar(0.25, dt)
    if periodic:
        lo = np.roll(e, 1, axis=axis)
        hi = np.roll(e, -1, axis=axis)
    else:
        lo = np.concatenate([np.take(e, [0], axis=axis), np.take(e, np.arange(e.shape[axis] - 1), axis=axis)], axis=axis)
        hi = np.concatenate([np.take(e, np.arange(1, e.shape[axis]), axis=axis), np.take(e, [e.shape[axis] - 1], axis=axis)], axis=axis)
    even = w3 * e + w1 * lo      # lower child: nearer neighbour is the one below
    odd = w3 * e + w1 * hi       # upper child: nearer neighbour is the one above
    shape = list(e.shape)
    shape[axis] *= 2
    out = np.empty(shape, dtype=dt)
    sl_even = [slice(None)] * e.ndim
    sl_odd = [slice(None)] * e.ndim
    sl_even[axis] = slice(0, None, 2)
    sl_odd[axis] = slice(1, None, 2)
    out[tuple(sl_even)] = even
    out[tuple(sl_odd)] = odd
    return out


def prolong(e):
    """Trilinear interpolation of a coarse field to the fine grid (tensor product)."""
    out = _interp_axis(e, 2, True)
    out = _interp_axis(out, 1, True)
    return _interp_axis(out, 0, False)


def prolong_add(p, e, lev_fine: Level):
    return p + np.where(lev_fine.mask, prolong(e), 0.0).astype(p.dtype, copy=False)


def coarsen(lev: Level) -> Level:
    """Move the face products to the next coarser grid (section 3.1, as one unit)."""
    n = lev.N // 2
    bx = lev.bx[:, :, 0::2].reshape(n, 2, n, 2, n).mean(axis=(1, 3))
    by = lev.by[:, 0::2, :].reshape(n, 2, n, n, 2).mean(axis=(1, 4))
    bz = lev.bz[0::2, :, :].reshape(n, n, 2, n, 2).mean(axis=(2, 4))
    any_child = lev.mask.reshape(n, 2, n, 2, n, 2).any(axis=(1, 3, 5))
    coarse = Level(bx, by, bz, any_child, 2.0 * lev.h)
    coarse.mask = any_child & (diagonal(coarse) > 0)
    return coarse


def dense_operator(lev: Level) -> np.ndarray:
    """Dense matrix of A, column by column from `apply` on unit vectors."""
    n = lev.N ** 3
    A = np.empty((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        A[:, c] = apply(e.reshape(lev.N, lev.N, lev.N), lev).ravel()
    return A


def pseudo_inverse(A: np.ndarray, rtol: float = PINV_RTOL) -> np.ndarray:
    """A^+ of a symmetric matrix from its eigendecomposition."""
    lam, V = np.linalg.eigh(A)
    keep = np.abs(lam) > rtol * np.abs(lam).max()
    inv = np.zeros_like(lam)
    inv[keep] = 1.0 / lam[keep]
    return (V * inv) @ V.T


@dataclasses.dataclass
class Hierarchy:
    levels: list
    coarse_pinv: np.ndarray   # FP64 pseudo-inverse of the coarsest operator

    @property
    def fine(self) -> Level:
        return self.levels[0]


def setup(bx, by, bz, mask, h, coarsest: int = COARSEST) -> Hierarchy:
    """Build the level hierarchy from finest-grid face coefficients and the body mask.

    Faces touching the body and the bottom wall are zeroed; a fluid cell left with
    no open face is treated as inactive (it has no equation to solve).
    """
    m = np.asarray(mask).astype(bool)
    bx, by, bz = close_faces(np.asarray(bx, np.float64), np.asarray(by, np.float64),
                             np.asarray(bz, np.float64), m)
    lev = Level(bx, by, bz, m, float(h))
    lev.mask = m & (diagonal(lev) > 0)
    levels = [lev]
    while levels[-1].N > coarsest:
        levels.append(coarsen(levels[-1]))
    return Hierarchy(levels, pseudo_inverse(dense_operator(levels[-1])))


def coarse_solve(hier: Hierarchy, f):
    """e = A_c^+ (f - active mean of f) on the coarsest grid, always in FP64."""
    lev = hier.levels[-1]
    f64 = np.asarray(f, np.float64)
    fh = project(f64, lev.mask)
    return (hier.coarse_pinv @ fh.ravel()).reshape(f.shape).astype(f.dtype)


def vcycle(hier: Hierarchy, p, f, levels=None, l: int = 0, nu1: int = 2, nu2: int = 2):
    """One V(nu1, nu2) cycle on level l for A_l p = f (levels may be an FP32 copy)."""
    levels = hier.levels if levels is None else levels
    lev = levels[l]
    if l == len(levels) - 1:
        return coarse_solve(hier, f)
    p = smooth(p, f, lev, nu1, (RED, BLACK))
    fc = restrict(residual(p, f, lev))
    ec = vcycle(hier, np.zeros_like(fc), fc, levels, l + 1, nu1, nu2)
    p = prolong_add(p, ec, lev)
    return smooth(p, f, lev, nu2, (BLACK, RED))


def relres(p, fhat, lev: Level, nf: float) -> float:
    r = residual(p, fhat, lev)
    return float(np.sqrt(np.sum(r * r))) / nf


# A projected right-hand side below this fraction of ||f|| (fluid cells) is rounding
# left by the mean removal: P f = 0, whose solution is p = 0 (f = 0, f constant).
ZERO_RHS = 64.0 * np.finfo(np.float64).eps


def zero_range(f, fhat, mask) -> bool:
    """True when P f is zero to rounding: ||P f|| <= ZERO_RHS ||f|| over the fluid cells."""
    nf_all = float(np.sqrt(np.sum(np.where(mask, np.asarray(f, np.float64), 0.0) ** 2)))
    return not float(np.sqrt(np.sum(fhat * fhat))) > ZERO_RHS * nf_all


def solve(hier: Hierarchy, f, p0=None, tol: float = 1e-10, max_cycles: int = 100):
    """FP64 V-cycles until the relative residual reaches tol.

    Returns (p, hist) with hist[0] the relative residual of the initial guess; a right-
    hand side with no component in the range of A (zero_range) returns (0, [0]).
    """
    lev = hier.fine
    fhat = project(np.asarray(f, np.float64), lev.mask)
    if zero_range(f, fhat, lev.mask):
        return np.zeros_like(fhat), [0.0]
    nf = float(np.sqrt(np.sum(fhat * fhat)))
    p = np.zeros_like(fhat) if p0 is None else np.where(lev.mask, p0, 0.0)
    hist = [relres(p, fhat, lev, nf)]
    while hist[-1] > tol and len(hist) <= max_cycles:
        p = vcycle(hier, p, fhat)
        hist.append(relres(p, fhat, lev, nf))
    return project(p, lev.mask), hist


def fp32_levels(hier: Hierarchy):
    return [lev.astype(np.float32) for lev in hier.levels]


def fp32_density_level(rho, lev: Level) -> Level:
    """The finest FP32 grid formed from the density in single precision: rho32 = fl32(rho)
    on active cells (+inf elsewhere), beta32 = 2 / (rho32_L + rho32_R) in float32 (0 on
    faces touching an inactive cell and on the bottom wall).  This is the operator of
    FP32 cycles that work from the density rather than rounding the FP64 coefficients."""
    r = np.where(lev.mask, np.asarray(rho, np.float64), np.inf).astype(np.float32)
    two = np.float32(2.0)
    bx = two / (r + np.roll(r, 1, axis=2))
    by = two / (r + np.roll(r, 1, axis=1))
    bz = np.zeros_like(r)
    bz[1:] = two / (r[1:] + r[:-1])
    return Level(bx, by, bz, lev.mask.copy(), lev.h)


def fp32_levels_from_rho(hier: Hierarchy, rho) -> list:
    """The FP32 hierarchy of cycles that work from the density on the finest grid:
    the finest grid from fl32(rho) (fp32_density_level), every coarser grid the FP64
    coarse coefficients rounded to nearest (they exist only as face products)."""
    return [fp32_density_level(rho, hier.fine)] + [lev.astype(np.float32) for lev in hier.levels[1:]]


def solve_mixed(hier: Hierarchy, f, p0=None, tol: float = 1e-10, max_steps: int = 100, lv32=None):
    """FP64 iterative refinement with one FP32 V-cycle per step (coarsest solve FP64).

    lv32: the FP32 hierarchy of the cycles; by default the FP64 coefficients of every
    grid rounded to nearest (fp32_levels), or fp32_levels_from_rho for cycles whose
    finest operator is formed from the density in single precision."""
    lev = hier.fine
    lv32 = fp32_levels(hier) if lv32 is None else lv32
    fhat = project(np.asarray(f, np.float64), lev.mask)
    nf = float(np.sqrt(np.sum(fhat * fhat)))
    p = np.zeros_like(fhat) if p0 is None else np.where(lev.mask, p0, 0.0)
    r = residual(p, fhat, lev)
    hist = [float(np.sqrt(np.sum(r * r))) / nf]
    while hist[-1] > tol and len(hist) <= max_steps:
        r32 = r.astype(np.float32)
        e32 = vcycle(hier, np.zeros_like(r32), r32, lv32)
        p = p + e32.astype(np.float64)
        r = residual(p, fhat, lev)
        hist.append(float(np.sqrt(np.sum(r * r))) / nf)
    return project(p, lev.mask), hist


def contraction(hist, skip: int = 2) -> float:
    """Geometric-mean residual reduction per cycle after the first `skip` cycles."""
    h = np.asarray(hist[skip:])
    h = h[h > 0]
    if len(h) < 2:
        return float("nan")
    return float((h[-1] / h[0]) ** (1.0 / (len(h) - 1)))


def solve_fcg(hier: Hierarchy, f, p0=None, tol: float = 1e-10, max_iters: int = 100, mixed: bool = False,
              precond=None, lv32=None):
    """Flexible conjugate gradients on the negative semi-definite A, preconditioned by
    one V(2,2) cycle from a zero guess (FP32 cycle when mixed), everything else FP64.

    A multigrid cycle is a good approximate inverse except for the few modes it misses
    (a steep, non-grid-aligned 1000:1 interface makes some); a Krylov method removes
    those.  The cycle here is not a symmetric operator (8-child mean restriction is not
    the transpose of trilinear prolongation), so the search direction is orthogonalised
    against the previous one with the flexible formula (Notay's FCG(1)):
        r = P f - A p, z = V(r), d = z
        repeat: w = A d;  alpha = (d.r)/(d.w);  p += alpha d;  r -= alpha w
                z = V(r);  beta = -(z.w)/(d.w);  d = z + beta d
    With a fixed symmetric preconditioner this is preconditioned CG.  `precond`, if
    given, replaces the V-cycle (used by the tests to compare with plain CG).
    """
    lev = hier.fine
    fhat = project(np.asarray(f, np.float64), lev.mask)
    if zero_range(f, fhat, lev.mask):
        return np.zeros_like(fhat), [0.0]
    nf = float(np.sqrt(np.sum(fhat * fhat)))
    p = np.zeros_like(fhat) if p0 is None else np.where(lev.mask, p0, 0.0)
    if mixed and lv32 is None:
        lv32 = fp32_levels(hier)

    def V(r):
        if precond is not None:
            return precond(r)
        if mixed:
            r32 = r.astype(np.float32)
            return vcycle(hier, np.zeros_like(r32), r32, lv32).astype(np.float64)
        return vcycle(hier, np.zeros_like(r), r)

    r = residual(p, fhat, lev)
    hist = [float(np.sqrt(np.sum(r * r))) / nf]
    if hist[-1] <= tol:
        return project(p, lev.mask), hist
    d = V(r)
    while len(hist) <= max_iters:
        w = apply(d, lev)
        dw = float(np.sum(d * w))
        alpha = float(np.sum(d * r)) / dw
        p = p + alpha * d
        r = r - alpha * w
        hist.append(float(np.sqrt(np.sum(r * r))) / nf)
        if hist[-1] <= tol:
            break
        z = V(r)
        beta = -float(np.sum(z * w)) / dw
        d = z + beta * d
    return project(p, lev.mask), hist


def setup_density_coarsening(rho, mask, h, coarsest: int = COARSEST) -> Hierarchy:
    """The variant section 3.1 rejects: density and cut-surface areas moved to the coarse
    grids independently, and the face coefficients re-formed on every grid.

      a_0 = o_f (open face), a_{l+1} = mean of the 4 coincident fine face areas;
      rho_{l+1} = mean of rho over the active children (cell centre to cell centre);
      beta_l = a_l * 2 / (rho_L + rho_R) on every grid.
    The finest grid is identical to `setup(face_coeffs_from_rho(rho, mask), ...)`;
    only the coarse operators differ.  A coarse cell with no active child gets rho = 1
    (its faces are closed, the value is never used).
    """
    from .operator import face_coeffs_from_rho, open_faces
    m = np.asarray(mask).astype(bool)
    ox, oy, oz = open_faces(m)
    areas = Level(ox.astype(np.float64), oy.astype(np.float64), oz.astype(np.float64), m, float(h))
    areas.mask = m & (diagonal(areas) > 0)
    rho_l = np.where(areas.mask, np.asarray(rho, np.float64), 1.0)
    levels = []
    while True:
        bx, by, bz = face_coeffs_from_rho(rho_l, np.ones_like(areas.mask))
        lev = Level(areas.bx * bx, areas.by * by, areas.bz * bz, areas.mask.copy(), areas.h)
        levels.append(lev)
        if areas.N <= coarsest:
            break
        n = areas.N // 2
        act = areas.mask.reshape(n, 2, n, 2, n, 2)
        num = np.where(act, rho_l.reshape(n, 2, n, 2, n, 2), 0.0).sum(axis=(1, 3, 5))
        cnt = act.sum(axis=(1, 3, 5))
        areas = coarsen(areas)
        rho_l = np.where(cnt > 0, num / np.maximum(cnt, 1), 1.0)
    return Hierarchy(levels, pseudo_inverse(dense_operator(levels[-1])))
