"""Cut-cell coefficients for an immersed body (thin binding over the C ABI).

The body is a level set psi at the cell corners, shape (N+1, N, N) ([k][j][i], corner
(i h, j h, k h), positive in the fluid).  `cut_cells` returns the open-area fraction of
every face, the fluid fraction of every cell and the merge map of cells under a
quarter full; `cut_coeffs` turns them and the density into the face coefficients and
mask that `MG` takes; `merge_rhs` / `merge_fill` move sources onto merged cells before
the solve and pressures back after it.  Every step runs in the HIP library.
"""
from __future__ import annotations

import torch

from . import _lib
from .solver import _check, _ptr, _stream


def _n(psi: torch.Tensor) -> int:
    n = psi.shape[-1]
    if tuple(psi.shape) != (n + 1, n, n):
        raise ValueError(f"psi must have shape (N+1, N, N), got {tuple(psi.shape)}")
    return n


def cut_cells(psi: torch.Tensor, samples: int = 8):
    """(ax, ay, az, vol, merge_to): open-area fractions of the low faces, fluid
    fractions, and the flat index each small cell merges into (-1 if none)."""
    n = _n(psi)
    shape = (n, n, n)
    ax, ay, az, vol = (torch.empty(shape, dtype=torch.float64, device=psi.device) for _ in range(4))
    merge_to = torch.empty(shape, dtype=torch.int32, device=psi.device)
    _check(_lib.load().mg_cut_cells(_ptr(psi, torch.float64), _lib.dims3(n), int(samples), _ptr(ax), _ptr(ay),
                                    _ptr(az), _ptr(vol), _ptr(merge_to), _stream(psi.device)), "mg_cut_cells")
    return ax, ay, az, vol, merge_to


def cut_coeffs(rho: torch.Tensor, ax, ay, az, vol, merge_to):
    """(bx, by, bz, mask) of the merged cut-cell operator."""
    n = rho.shape[-1]
    bx, by, bz = (torch.empty_like(rho) for _ in range(3))
    mask = torch.empty(rho.shape, dtype=torch.uint8, device=rho.device)
    _check(_lib.load().mg_cut_coeffs(_ptr(rho, torch.float64), *(_ptr(t, torch.float64) for t in (ax, ay, az, vol)),
                                     _ptr(merge_to, torch.int32), _lib.dims3(n), _ptr(bx), _ptr(by), _ptr(bz),
                                     _ptr(mask), _stream(rho.device)), "mg_cut_coeffs")
    return bx, by, bz, mask


def merge_rhs(merge_to: torch.Tensor, f: torch.Tensor) -> torch.Tensor:
    """f with each donor's source added onto its target (0 on donors)."""
    n = f.shape[-1]
    g = torch.empty_like(f)
    _check(_lib.load().mg_merge_rhs(_ptr(merge_to, torch.int32), _ptr(f, torch.float64), _ptr(g), _lib.dims3(n),
                                    _stream(f.device)), "mg_merge_rhs")
    return g


def merge_fill(merge_to: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    """p on each donor = p on its target, in place."""
    n = p.shape[-1]
    _check(_lib.load().mg_merge_fill(_ptr(merge_to, torch.int32), _ptr(p, torch.float64), _lib.dims3(n),
                                     _stream(p.device)), "mg_merge_fill")
    return p


__all__ = ["cut_cells", "cut_coeffs", "merge_rhs", "merge_fill"]
