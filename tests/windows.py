"""Small windows of a large grid, for checking sampled outputs with the oracle.

One red-black sweep changes a cell from values at most two cells away (two sweeps: four),
a residual from
values one cell away, and an 8-child restriction or a trilinear prolongation from one
coarse cell around the parent.  So the oracle can recompute a sampled output of a
1024^3 pass on an 8^3 window around the sample, with the window's own (wrong) edges
two or more cells away from the sample.  Only indexing lives here: windows are cut out
of the caller's arrays (x and y wrap, z is clipped to the grid so the real walls are
kept) and the oracle does all of the arithmetic.
"""
from __future__ import annotations

import numpy as np

W = 8   # window side (even: the red-black colouring of the window is the grid's)


def origin(N: int, k: int, j: int, i: int, w: int = W):
    """(k0, j0, i0) of the window holding (k, j, i) three or four cells from its low
    edges: z clipped to [0, N - w], x and y periodic, and k0 + j0 + i0 even so that the
    window's colour (a + b + c) mod 2 is the grid's."""
    k0 = min(max(k - w // 2 + 1, 0), N - w)
    j0 = (j - w // 2 + 1) % N
    i0 = (i - w // 2 + 1) % N
    if (k0 + j0 + i0) % 2:
        i0 = (i0 - 1) % N
    return k0, j0, i0


def cut(a, o, w: int = W):
    """a[k0:k0+w, j0:j0+w (mod N), i0:i0+w (mod N)] as a numpy array (a may be a numpy
    array or a CUDA tensor; only the window is copied)."""
    k0, j0, i0 = o
    N = a.shape[-1]
    jj = (j0 + np.arange(w)) % N
    ii = (i0 + np.arange(w)) % N
    if hasattr(a, "cpu"):
        import torch
        t = a[k0:k0 + w].index_select(-2, torch.as_tensor(jj, device=a.device))
        t = t.index_select(-1, torch.as_tensor(ii, device=a.device))
        return t.cpu().numpy()
    return np.asarray(a[k0:k0 + w][:, jj][:, :, ii])


def local(o, N: int, k: int, j: int, i: int):
    """Index of grid cell (k, j, i) of an N^3 grid inside the window with origin o."""
    k0, j0, i0 = o
    return k - k0, (j - j0) % N, (i - i0) % N


def gather(t, cells):
    """t[k, j, i] for a list of cells, from a CUDA tensor (one small copy)."""
    import torch
    idx = torch.as_tensor(np.asarray(cells, dtype=np.int64).T, device=t.device)
    return t[idx[0], idx[1], idx[2]].cpu().numpy()


# ---------------------------------------------------------------- oracle values at sampled cells

def _level(rho, mask, h):
    from oracle.operator import Level, diagonal, face_coeffs_from_rho
    m = np.asarray(mask).astype(bool)
    lev = Level(*face_coeffs_from_rho(np.asarray(rho, np.float64), m), m, h)
    lev.mask = m & (diagonal(lev) > 0)
    return lev


def sweep_at(rho, mask, p, f, h, cell, order, sweeps=1):
    """The oracle's value at `cell` after one red-black sweep (order 0: red then black)
    of the whole grid, from an 8^3 window, or after two sweeps from a 12^3 window (each
    sweep reaches two cells further); returns (value, scale of the window)."""
    from oracle import multigrid as omg
    N = rho.shape[-1]
    w = 4 * sweeps + 4
    o = origin(N, *cell, w=w)
    lev = _level(cut(rho, o, w), cut(mask, o, w), h)
    pw = cut(p, o, w)
    out = omg.smooth(pw, cut(f, o, w), lev, sweeps, (omg.RED, omg.BLACK) if order == 0 else (omg.BLACK, omg.RED))
    return out[local(o, N, *cell)], max(np.abs(out).max(), np.abs(pw).max())


def residual_restrict_at(rho, mask, p, f, h, coarse_cell):
    """The oracle's 8-child mean of r = f - A p at a coarse cell, from a 4^3 window of
    coarse cells (8^3 fine cells); returns (value, scale)."""
    from oracle import multigrid as omg
    N = rho.shape[-1]
    n = N // 2
    oc = origin(n, *coarse_cell, w=4)
    of = (2 * oc[0], 2 * oc[1], 2 * oc[2])
    lev = _level(cut(rho, of), cut(mask, of), h)
    out = omg.restrict(omg.residual(cut(p, of), cut(f, of), lev))
    return out[local(oc, n, *coarse_cell)], max(np.abs(out).max(), 1e-300)


def prolong_add_at(rho, mask, p, e, h, cell):
    """The oracle's p + m trilinear(e) at a fine cell, from the 4^3 coarse cells around
    its parent and their 8^3 children; returns (value, scale)."""
    from oracle import multigrid as omg
    N = rho.shape[-1]
    n = N // 2
    oc = origin(n, cell[0] // 2, cell[1] // 2, cell[2] // 2, w=4)
    of = (2 * oc[0], 2 * oc[1], 2 * oc[2])
    lev = _level(cut(rho, of), cut(mask, of), h)
    out = omg.prolong_add(cut(p, of), cut(e, oc, w=4), lev)
    return out[local(of, N, *cell)], max(np.abs(out).max(), 1e-300)
