"""The oracle's relative residual of a solution on grids too large for one array pass.

||P f - A p|| / ||P f|| over the active cells, with the oracle's operator
(oracle.operator: face coefficients 2/(rho_L + rho_R) on open faces, fluid cells with
no open face inactive, f projected to zero active mean), evaluated on slabs of z-planes:
each slab is extended by one plane below and above so every face of its own planes is
formed exactly as on the whole grid.  Host-side FP64 numpy; slabs run in a thread pool
(numpy releases the interpreter lock inside its array operations).
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle.operator import Level, apply, diagonal, face_coeffs_from_rho


def _slab_level(rho, mask, k0, k1, h):
    """The oracle's level for planes [a, b) = [k0 - 1, k1 + 1] clipped to the grid."""
    N = rho.shape[0]
    a, b = max(k0 - 1, 0), min(k1 + 1, N)
    m = np.asarray(mask[a:b]).astype(bool)
    bx, by, bz = face_coeffs_from_rho(np.asarray(rho[a:b], np.float64), m)
    lev = Level(bx, by, bz, m, h)
    lev.mask = m & (diagonal(lev) > 0)
    return lev, a


def slab_relres(rho, mask, f, p, h, slab: int = 32, workers: int | None = None) -> float:
    N = rho.shape[0]
    bounds = [(k, min(k + slab, N)) for k in range(0, N, slab)]
    workers = workers or min(8, os.cpu_count() or 1)
    active = np.empty(rho.shape, dtype=bool)

    def pass1(kk):
        k0, k1 = kk
        lev, a = _slab_level(rho, mask, k0, k1, h)
        act = lev.mask[k0 - a:k1 - a]
        active[k0:k1] = act
        fs = np.asarray(f[k0:k1], np.float64)
        return float(np.sum(fs, where=act)), int(np.count_nonzero(act))

    with ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(pass1, bounds))
    mean = sum(s for s, _ in parts) / sum(c for _, c in parts)

    def pass2(kk):
        k0, k1 = kk
        lev, a = _slab_level(rho, mask, k0, k1, h)
        b = a + lev.mask.shape[0]
        Ap = apply(np.asarray(p[a:b], np.float64), lev)[k0 - a:k1 - a]
        act = active[k0:k1]
        fh = np.where(act, np.asarray(f[k0:k1], np.float64) - mean, 0.0)
        r = np.where(act, fh - Ap, 0.0)
        return float(np.sum(r * r)), float(np.sum(fh * fh))

    with ThreadPoolExecutor(workers) as ex:
        parts = list(ex.map(pass2, bounds))
    return float(np.sqrt(sum(r for r, _ in parts)) / np.sqrt(sum(g for _, g in parts)))
