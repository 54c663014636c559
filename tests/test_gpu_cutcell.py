"""Cut cells on the GPU against the oracle (section 2.2, fractional areas and merging).

Fractions, volume fractions and the merge map are integer sample counts decided on
the same bits on both sides: compared exactly.  Face coefficients: within 1e-15 of
max (the face product's reciprocal may differ from numpy's quotient by an ulp).
Source and pressure moves: exact.  The merged cut-cell operator is then solved on
the GPU and compared with the oracle's sparse direct solve (relative L2 <= 1e-9).
"""
import numpy as np
import pytest
import torch

import fields
from oracle import cutcell as cc
from oracle import exact
from oracle import multigrid as omg
from oracle.operator import project
from tests.gpu_helpers import dev, host, maxrel, relerr

pytestmark = pytest.mark.gpu


def sphere_psi(N, r=0.3):
    g = np.arange(N) / N
    gz = np.arange(N + 1) / N
    return np.sqrt((g[None, None, :] - 0.5) ** 2 + (g[None, :, None] - 0.47) ** 2 + (gz[:, None, None] - 0.52) ** 2) - r


CASES = [("wavy", 32, 8), ("wavy", 64, 8), ("sphere", 32, 4), ("sphere", 32, 16), ("wavy", 16, 2)]


@pytest.mark.parametrize("body,N,S", CASES)
def test_fractions_and_merge_map_exact(body, N, S):
    from paper_1410_2240_amd.cutcell import cut_cells
    print(f"cut cells {body} N={N} S={S}", flush=True)
    psi = fields.wavy_cut(N)[1] if body == "wavy" else sphere_psi(N)
    ax, ay, az, vol, mt = (host(t) for t in cut_cells(dev(psi), S))
    want = cc.face_fractions(psi, S)
    for g, w in zip((ax, ay, az), want):
        assert np.array_equal(g, w)
    wvol = cc.volume_fractions(psi, S)
    assert np.array_equal(vol, wvol)
    wmt = cc.merge_targets(psi, wvol)
    assert np.array_equal(mt.astype(np.int64), wmt)
    assert (wmt >= 0).any() or body == "wavy" and N == 16


@pytest.mark.parametrize("N", [32, 64])
def test_coefficients_and_moves_match_oracle(N):
    from paper_1410_2240_amd.cutcell import cut_cells, cut_coeffs, merge_fill, merge_rhs
    print(f"cut coefficients N={N}", flush=True)
    rho, psi = fields.wavy_cut(N)
    geo = cut_cells(dev(psi), 8)
    bx, by, bz, mask = (host(t) for t in cut_coeffs(dev(rho), *geo))
    # the oracle's geometry from psi itself (not from the GPU's fractions and map)
    ax, ay, az = cc.face_fractions(psi, 8)
    vol = cc.volume_fractions(psi, 8)
    mt = cc.merge_targets(psi, vol)
    lev = cc.cut_coeffs(rho, ax, ay, az, vol, mt, 1.0 / N)
    assert np.array_equal(mask.astype(bool), lev.mask)
    for g, w in ((bx, lev.bx), (by, lev.by), (bz, lev.bz)):
        assert maxrel(g, w) <= 1e-15
    g = np.random.default_rng(11)
    f = g.standard_normal((N, N, N))
    assert np.array_equal(host(merge_rhs(geo[4], dev(f))), cc.merge_rhs(f, mt))
    p = g.standard_normal((N, N, N))
    assert np.array_equal(host(merge_fill(geo[4], dev(p))), cc.merge_fill(p, mt))


@pytest.mark.parametrize("krylov", [False, True])
def test_cut_cell_solve_matches_sparse_direct(krylov):
    """Solve the merged cut-cell system of the wavy field with the ellipsoid at 32^3."""
    from paper_1410_2240_amd import MG
    from paper_1410_2240_amd.cutcell import cut_cells, cut_coeffs, merge_fill, merge_rhs
    N = 32
    print(f"cut-cell solve krylov={krylov}", flush=True)
    rho, psi = fields.wavy_cut(N)
    geo = cut_cells(dev(psi), 8)
    bx, by, bz, mask = cut_coeffs(dev(rho), *geo)
    mg = MG(bx, by, bz, mask, krylov=krylov)
    g = np.random.default_rng(12)
    f0 = g.standard_normal((N, N, N))
    f = merge_rhs(geo[4], dev(f0))
    p, hist, st = mg.solve(f, tol=1e-12, max_cycles=200)
    merge_fill(geo[4], p)
    # the oracle's merged system from psi itself
    ax, ay, az = cc.face_fractions(psi, 8)
    vol = cc.volume_fractions(psi, 8)
    mt = cc.merge_targets(psi, vol)
    lev = cc.cut_coeffs(rho, ax, ay, az, vol, mt, 1.0 / N)
    lev = omg.setup(lev.bx, lev.by, lev.bz, lev.mask, lev.h).fine   # drops cells without an open face
    fo = cc.merge_rhs(f0, mt)
    want = cc.merge_fill(exact.solve_sparse(lev, project(fo, lev.mask)), mt)
    live = vol > 0
    assert relerr(np.where(live, host(p), 0.0), np.where(live, want, 0.0)) <= 1e-9
