"""Oracle: fractional-area cut cells with small-cell merging (FP64, numpy).

TEST INFRASTRUCTURE ONLY.  Nothing in the solver library imports or calls this.

Paper section 2.2 (enforcement of body boundary conditions): the body is a signed
distance function psi (positive in the fluid, negative in the body); cells the hull
cuts are treated by finite volumes with the fraction of each face that lies in the
fluid (the method of fractional areas, eq. (integral2) with the no-flux condition
on the body part of the cell surface); a cell whose fluid volume is under a quarter
of the cell is merged with a neighbour, in the direction of the steepest gradient of
psi.  The paper defers the formulas to a cited reference, so this oracle fixes one
reading, the same one the HIP kernels implement:

  * psi is given at cell corners (arrays [k][j][i], k = 0..N, x and y periodic).  On a
    face it is the bilinear interpolant of the face's 4 corners, in a cell the
    trilinear interpolant of the cell's 8 corners.
  * The open-area fraction of a face is the fraction of S x S midpoint samples where
    psi > 0; the fluid volume fraction of a cell is the fraction of S^3 midpoint
    samples.  A sample's value is summed corner by corner in a fixed order with the
    weights first (they are exact dyadic numbers), so that both implementations take
    every sign decision on the same bits.  The bottom-wall faces are closed.
  * Merging: a cell with 0 < V < 1/4 goes to the face neighbour along the largest
    component of the gradient of the trilinear psi at the cell centre (ties: x, then
    y, then z), on the side where psi grows, provided that neighbour exists (z walls)
    and has V >= 1/4.  Otherwise the cell stays as a small cut cell.
  * The merged control volume keeps the target's pressure.  In the 7-point operator
    the donor becomes inactive.  A face between two donors that merge side by side
    (the same direction, into targets that are face neighbours) adds its open area to
    the face between the targets; any other face of a donor (towards a kept cell, or
    away from its target towards the body) would couple cells that are not face
    neighbours and is dropped.  The donor's source is added to the target's, and
    after the solve the donor takes the target's pressure.
  * beta_f = area_f * 2 / (rho_L + rho_R) on faces between two kept cells, else 0.
"""
from __future__ import annotations

import numpy as np

from .operator import Level

MERGE_FRACTION = 0.25


def _offsets(S: int) -> np.ndarray:
    return (np.arange(S) + 0.5) / S


def corner(psi: np.ndarray, a: int, b: int, c: int) -> np.ndarray:
    """psi at corner (i+a, j+b, k+c) of every cell (i, j, k), shape (N, N, N)."""
    N = psi.shape[1]
    return np.roll(np.roll(psi[c:c + N], -b, axis=1), -a, axis=2)


def _face_fraction(c00, c10, c01, c11, S):
    """Fraction of S x S samples of the bilinear interpolant that are > 0 (c_uv is
    the corner at u, v in {0, 1})."""
    t = _offsets(S)
    count = np.zeros(c00.shape, dtype=np.int64)
    for v in t:
        for u in t:
            w00, w10, w01, w11 = (1.0 - u) * (1.0 - v), u * (1.0 - v), (1.0 - u) * v, u * v
            val = ((w00 * c00 + w10 * c10) + w01 * c01) + w11 * c11
            count += val > 0.0
    return count / float(S * S)


def face_fractions(psi: np.ndarray, S: int = 8):
    """Open-area fractions (ax, ay, az) of the low faces of every cell.

    ax[k, j, i] is the face x = i h (corners (i, j..j+1, k..k+1)), parametrised by
    (u, v) = (y, z); ay by (x, z); az by (x, y).  az[0] = 0 (bottom wall)."""
    p = lambda a, b, c: corner(psi, a, b, c)
    ax = _face_fraction(p(0, 0, 0), p(0, 1, 0), p(0, 0, 1), p(0, 1, 1), S)
    ay = _face_fraction(p(0, 0, 0), p(1, 0, 0), p(0, 0, 1), p(1, 0, 1), S)
    az = _face_fraction(p(0, 0, 0), p(1, 0, 0), p(0, 1, 0), p(1, 1, 0), S)
    az[0] = 0.0
    return ax, ay, az


def volume_fractions(psi: np.ndarray, S: int = 8) -> np.ndarray:
    """Fluid volume fraction of every cell: S^3 samples of the trilinear interpolant."""
    t = _offsets(S)
    cs = [corner(psi, a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)]   # x fastest
    count = np.zeros(cs[0].shape, dtype=np.int64)
    for w in t:
        for v in t:
            for u in t:
                wts = [(u if a else 1.0 - u) * (v if b else 1.0 - v) * (w if c else 1.0 - w)
                       for c in (0, 1) for b in (0, 1) for a in (0, 1)]
                val = wts[0] * cs[0]
                for q in range(1, 8):
                    val = val + wts[q] * cs[q]
                count += val > 0.0
    return count / float(S ** 3)


def centre_gradient(psi: np.ndarray):
    """Gradient of the trilinear psi at each cell centre, up to the factor 1/h: the
    mean of the 4 corner differences along each axis."""
    p = lambda a, b, c: corner(psi, a, b, c)
    gx = (((p(1, 0, 0) - p(0, 0, 0)) + (p(1, 1, 0) - p(0, 1, 0))) + (p(1, 0, 1) - p(0, 0, 1))) + (p(1, 1, 1) - p(0, 1, 1))
    gy = (((p(0, 1, 0) - p(0, 0, 0)) + (p(1, 1, 0) - p(1, 0, 0))) + (p(0, 1, 1) - p(0, 0, 1))) + (p(1, 1, 1) - p(1, 0, 1))
    gz = (((p(0, 0, 1) - p(0, 0, 0)) + (p(1, 0, 1) - p(1, 0, 0))) + (p(0, 1, 1) - p(0, 1, 0))) + (p(1, 1, 1) - p(1, 1, 0))
    return gx * 0.25, gy * 0.25, gz * 0.25


def merge_targets(psi: np.ndarray, vol: np.ndarray) -> np.ndarray:
    """Flat index of the cell each small cell merges into, -1 where none."""
    N = vol.shape[0]
    gx, gy, gz = centre_gradient(psi)
    out = np.full(vol.shape, -1, dtype=np.int64)
    for k in range(N):
        for j in range(N):
            for i in range(N):
                V = vol[k, j, i]
                if not (0.0 < V < MERGE_FRACTION):
                    continue
                g = (abs(gx[k, j, i]), abs(gy[k, j, i]), abs(gz[k, j, i]))
                d = 0 if (g[0] >= g[1] and g[0] >= g[2]) else (1 if g[1] >= g[2] else 2)
                s = 1 if (gx, gy, gz)[d][k, j, i] > 0.0 else -1
                ti, tj, tk = i, j, k
                if d == 0:
                    ti = (i + s) % N
                elif d == 1:
                    tj = (j + s) % N
                else:
                    tk = k + s
                    if tk < 0 or tk >= N:
                        continue
                if vol[tk, tj, ti] < MERGE_FRACTION:
                    continue
                out[k, j, i] = (tk * N + tj) * N + ti
    return out


def _shift(a: np.ndarray, axis: int, step: int, fill):
    """b[c] = a[c + step e_axis] (x, y periodic; z out of range -> fill)."""
    if axis < 2:
        return np.roll(a, -step, axis=2 - axis)
    b = np.full_like(a, fill)
    if step > 0:
        b[:-step] = a[step:]
    else:
        b[-step:] = a[:step]
    return b


def _donor_from(merge_to: np.ndarray, axis: int, step: int) -> np.ndarray:
    """True where the neighbour c + step e_axis merges into c."""
    N = merge_to.shape[0]
    idx = np.arange(N ** 3, dtype=np.int64).reshape(N, N, N)
    return _shift(merge_to, axis, step, -1) == idx


# donor scan order of every gather: (x, -1), (x, +1), (y, -1), (y, +1), (z, -1), (z, +1)
DONOR_ORDER = [(m, s) for m in range(3) for s in (-1, 1)]


def merged_areas(ax, ay, az, merge_to):
    """Face areas after merging (low-face storage).

    A face of the grid separates the control volumes that own its two cells (a donor
    is owned by its target).  The face between c - e_l and c keeps its own area and
    gains the area of every face between two donors that merge side by side into
    those two cells: d = c + s e_m into c and d - e_l into c - e_l (m != l), added in
    DONOR_ORDER.  Every other donor face (towards a kept cell, or away from the
    target) separates volumes that are not face neighbours and is dropped."""
    a = (ax, ay, az)
    out = []
    for l in range(3):
        acc = a[l].copy()
        for m, s in DONOR_ORDER:
            if m == l:
                continue
            pair = _donor_from(merge_to, m, s) & _shift(_donor_from(merge_to, m, s), l, -1, False)
            acc = acc + np.where(pair, _shift(a[l], m, s, 0.0), 0.0)
        if l == 2:
            acc[0] = 0.0
        out.append(acc)
    return out


def cut_coeffs(rho, ax, ay, az, vol, merge_to, h: float) -> Level:
    """The merged cut-cell operator: face coefficients (low-face storage) and mask."""
    kept = (vol > 0.0) & (merge_to < 0)
    areas = merged_areas(ax, ay, az, merge_to)
    out = []
    for l, a in enumerate(areas):
        lo_kept = _shift(kept, l, -1, False)
        lo_rho = _shift(rho, l, -1, 1.0)
        beta = np.where(kept & lo_kept, a * (2.0 / (rho + lo_rho)), 0.0)
        if l == 2:
            beta[0] = 0.0
        out.append(beta)
    return Level(out[0], out[1], out[2], kept, h)


def merge_rhs(f: np.ndarray, merge_to: np.ndarray) -> np.ndarray:
    """Source of each merged control volume on its target (donors added in
    DONOR_ORDER); donors get 0."""
    g = f.copy()
    for m, s in DONOR_ORDER:
        g = g + np.where(_donor_from(merge_to, m, s), _shift(f, m, s, 0.0), 0.0)
    return np.where(merge_to >= 0, 0.0, g)


def merge_fill(p: np.ndarray, merge_to: np.ndarray) -> np.ndarray:
    """After the solve each donor takes its target's pressure."""
    q = p.copy()
    donors = np.flatnonzero(merge_to >= 0)
    q.flat[donors] = p.flat[merge_to.flat[donors]]
    return q
