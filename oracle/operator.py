"""Oracle: the discrete variable-coefficient Poisson operator (FP64, numpy).

TEST INFRASTRUCTURE ONLY.  Nothing in the solver library imports or calls this.

The operator is the finite-volume form of the pressure Poisson equation
div((1/rho) grad P) = Sigma (paper section 2, eq. (pois)), integrated over each cell
as in eq. (integral2): the flux through a face is (face coefficient) x (pressure
difference across the face) / h, and the face coefficient is the product of
1/rho and the open area of the face, formed on the finest grid (section 3.1).

Discretisation read from the paper (it gives none itself):
  * uniform cell-centred grid, N cells per side, h = 1/N, arrays [k, j, i];
  * periodic in x and y, walls (homogeneous Neumann, zero face coefficient) in z;
  * face coefficient beta_f = o_f * 2 / (rho_L + rho_R): 1/rho at the face taken
    as the inverse of the mean of the two cell densities, o_f = 1 when both cells
    are fluid and 0 when the face touches the body or is a z wall;
  * (A p)_c = m_c h^-2 sum_{faces f of c} beta_f (p_neighbour - p_c), keeping the
    paper's sign (A is negative semi-definite).
Face storage ("low faces"): bx[k,j,i] couples (i-1 mod N, j, k) with (i, j, k),
by likewise in j, bz[k,j,i] couples (i, j, k-1) with (i, j, k); bz[0] is the bottom
wall and the top wall is implicit.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


@dataclasses.dataclass
class Level:
    """One grid of the hierarchy: face coefficients, fluid mask and spacing."""
    bx: np.ndarray
    by: np.ndarray
    bz: np.ndarray
    mask: np.ndarray   # bool, True = active (fluid) cell
    h: float

    @property
    def N(self) -> int:
        return self.bx.shape[0]

    def astype(self, dtype) -> "Level":
        return Level(self.bx.astype(dtype), self.by.astype(dtype), self.bz.astype(dtype),
                     self.mask.copy(), self.h)


def open_faces(mask):
    """o_f on the low faces of every cell: both neighbours fluid; z walls closed."""
    m = np.asarray(mask).astype(bool)
    ox = m & np.roll(m, 1, axis=2)
    oy = m & np.roll(m, 1, axis=1)
    oz = np.zeros_like(m)
    oz[1:] = m[1:] & m[:-1]
    return ox, oy, oz


def face_coeffs_from_rho(rho, mask):
    """beta_f = o_f * 2/(rho_L + rho_R): 1/rho times open area on each face (sec. 3.1)."""
    ox, oy, oz = open_faces(mask)
    bx = np.where(ox, 2.0 / (rho + np.roll(rho, 1, axis=2)), 0.0)
    by = np.where(oy, 2.0 / (rho + np.roll(rho, 1, axis=1)), 0.0)
    bz = np.zeros_like(rho)
    bz[1:] = np.where(oz[1:], 2.0 / (rho[1:] + rho[:-1]), 0.0)
    return bx, by, bz


def close_faces(bx, by, bz, mask):
    """Zero the coefficients of faces that touch a body cell and of the bottom wall."""
    ox, oy, oz = open_faces(mask)
    return np.where(ox, bx, 0.0), np.where(oy, by, 0.0), np.where(oz, bz, 0.0)


def diagonal(lev: Level) -> np.ndarray:
    """D_c = sum of the six face coefficients of cell c (walls and body faces are 0)."""
    bz_hi = np.zeros_like(lev.bz)
    bz_hi[:-1] = lev.bz[1:]
    return (lev.bx + np.roll(lev.bx, -1, axis=2) + lev.by + np.roll(lev.by, -1, axis=1)
            + lev.bz + bz_hi)


def neighbour_sum(p, lev: Level):
    """S_c = sum_f beta_f p_neighbour(f), over the six faces of each cell."""
    s = (lev.bx * np.roll(p, 1, axis=2) + np.roll(lev.bx, -1, axis=2) * np.roll(p, -1, axis=2)
         + lev.by * np.roll(p, 1, axis=1) + np.roll(lev.by, -1, axis=1) * np.roll(p, -1, axis=1))
    sz = np.zeros_like(p)
    sz[1:] += lev.bz[1:] * p[:-1]       # face below, neighbour k-1
    sz[:-1] += lev.bz[1:] * p[1:]       # face above, neighbour k+1
    return s + sz


def apply(p, lev: Level):
    """(A p)_c = m_c h^-2 sum_f beta_f (p_nb - p_c), via face fluxes F = beta (p_hi - p_lo)."""
    Fx = lev.bx * (p - np.roll(p, 1, axis=2))          # low x face of each cell
    Fy = lev.by * (p - np.roll(p, 1, axis=1))
    Fz = np.zeros_like(p)
    Fz[1:] = lev.bz[1:] * (p[1:] - p[:-1])
    Fz_hi = np.zeros_like(p)
    Fz_hi[:-1] = Fz[1:]
    div = (np.roll(Fx, -1, axis=2) - Fx) + (np.roll(Fy, -1, axis=1) - Fy) + (Fz_hi - Fz)
    return np.where(lev.mask, div / (lev.h * lev.h), 0.0).astype(p.dtype, copy=False)


def face_list(lev: Level):
    """All faces as (cell_lo, cell_hi, beta) flat-index triples, walls excluded."""
    N = lev.N
    idx = np.arange(N ** 3).reshape(N, N, N)
    lo = [np.roll(idx, 1, axis=2), np.roll(idx, 1, axis=1), idx[:-1]]
    hi = [idx, idx, idx[1:]]
    beta = [lev.bx, lev.by, lev.bz[1:]]
    L = np.concatenate([a.ravel() for a in lo])
    R = np.concatenate([a.ravel() for a in hi])
    B = np.concatenate([a.ravel() for a in beta])
    return L, R, B


def assemble(lev: Level) -> sp.csr_matrix:
    """Sparse matrix of A built face by face (independent of `apply`)."""
    n = lev.N ** 3
    L, R, B = face_list(lev)
    keep = B != 0
    L, R, B = L[keep], R[keep], B[keep] / (lev.h * lev.h)
    rows = np.concatenate([L, R, L, R])
    cols = np.concatenate([R, L, L, R])
    vals = np.concatenate([B, B, -B, -B])
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    m = lev.mask.ravel().astype(np.float64)
    return sp.diags(m) @ A


def components(lev: Level) -> int:
    """Number of connected components of the active cells over open faces."""
    n = lev.N ** 3
    L, R, B = face_list(lev)
    keep = B != 0
    G = sp.coo_matrix((np.ones(keep.sum()), (L[keep], R[keep])), shape=(n, n))
    act = lev.mask.ravel()
    ncomp, lab = connected_components(G, directed=False)
    return len(np.unique(lab[act]))


def project(f, mask):
    """P f = m (f - mean over active cells of f): the compatible part of f."""
    m = np.asarray(mask).astype(bool)
    return np.where(m, f - f[m].mean(), 0.0)
