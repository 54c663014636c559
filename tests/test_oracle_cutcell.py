"""Pins of the cut-cell oracle (fractional areas, volume fractions, merging).

Closed forms: planes that cut cells exactly between sample rows give fractions of
exactly 0, 1/2, 1/8 or 1; a tilted plane against the exact area of a polygon clipped
from the unit square; a sphere against its volume and its cross-sections.  The
merge is pinned on a layer of small cells whose target, merged areas, source and
pressure are known in closed form.
"""
import math

import numpy as np
import pytest

from oracle import cutcell as cc
from oracle import exact
from oracle.operator import apply, project

S = 8


def corners(N, fn):
    """psi at the corners (i h, j h, k h), k = 0..N."""
    g = np.arange(N) / N
    gz = np.arange(N + 1) / N
    return fn(g[None, None, :], g[None, :, None], gz[:, None, None]) + np.zeros((N + 1, N, N))


@pytest.mark.parametrize("sign", [1, -1])
def test_horizontal_plane_closed_form(sign):
    """psi = +-(z - z0) with z0 on a cell mid-plane: the cut layer is exactly half open."""
    N, k0 = 8, 3
    z0 = (k0 + 0.5) / N
    psi = corners(N, lambda x, y, z: sign * (z - z0))
    ax, ay, az = cc.face_fractions(psi, S)
    vol = cc.volume_fractions(psi, S)
    k = np.arange(N)[:, None, None] + np.zeros((N, N, N))
    fluid_above = sign > 0
    want_side = np.where(k == k0, 0.5, np.where((k > k0) == fluid_above, 1.0, 0.0))
    assert np.array_equal(ax, want_side) and np.array_equal(ay, want_side)
    assert np.array_equal(vol, want_side)
    want_z = np.where((k >= k0 + 1) == fluid_above, 1.0, 0.0)
    want_z[0] = 0.0   # bottom wall
    assert np.array_equal(az, want_z)


def test_periodic_slab_in_x():
    """A body slab |x - 1/2| < 5/(2N): the two cut columns are half open, the x faces
    inside the slab closed, and y faces follow the columns."""
    N = 16
    w = 2.5 / N
    psi = corners(N, lambda x, y, z: np.abs(x - 0.5) - w)
    ax, ay, az = cc.face_fractions(psi, S)
    vol = cc.volume_fractions(psi, S)
    i = np.arange(N)
    xc = (i + 0.5) / N
    col = np.where(np.abs(np.abs(xc - 0.5) - w) < 1e-12, 0.5, (np.abs(xc - 0.5) > w).astype(float))
    assert np.array_equal(vol, np.broadcast_to(col, vol.shape))
    assert np.array_equal(ay, np.broadcast_to(col, ay.shape))
    xf = i / N
    face = (np.abs(xf - 0.5) > w).astype(float)
    assert np.array_equal(ax, np.broadcast_to(face, ax.shape))


def clipped_area(c00, c10, c01, c11):
    """Exact area of {bilinear > 0} on the unit square when the corner values come
    from a linear function (polygon clipping)."""
    pts = [(0, 0, c00), (1, 0, c10), (1, 1, c11), (0, 1, c01)]
    poly = []
    for a, b in zip(pts, pts[1:] + pts[:1]):
        if a[2] > 0:
            poly.append(a[:2])
        if (a[2] > 0) != (b[2] > 0):
            t = a[2] / (a[2] - b[2])
            poly.append((a[0] + t * (b[0] - a[0]), a[1] + t * (b[1] - a[1])))
    if len(poly) < 3:
        return 0.0
    return 0.5 * abs(sum(p[0] * q[1] - q[0] * p[1] for p, q in zip(poly, poly[1:] + poly[:1])))


def test_tilted_plane_against_polygon_area():
    """Midpoint sampling of a face cut by a tilted plane converges to the exact clipped
    area: within 2/S for S = 64 on every face of a 4^3 block."""
    N, Sf = 4, 64
    n = np.array([0.37, -0.61, 0.70])
    psi = corners(N, lambda x, y, z: n[0] * (x - 0.41) + n[1] * (y - 0.57) + n[2] * (z - 0.46))
    # keep the plane away from the periodic seam: only interior faces are compared
    ax, ay, az = cc.face_fractions(psi, Sf)
    for k in range(N):
        for j in range(N - 1):
            for i in range(N - 1):
                P = lambda a, b, c: psi[k + c, j + b, i + a]
                want_x = clipped_area(P(0, 0, 0), P(0, 1, 0), P(0, 0, 1), P(0, 1, 1))
                want_y = clipped_area(P(0, 0, 0), P(1, 0, 0), P(0, 0, 1), P(1, 0, 1))
                assert abs(ax[k, j, i] - want_x) <= 2.0 / Sf
                assert abs(ay[k, j, i] - want_y) <= 2.0 / Sf
                if k > 0:
                    want_z = clipped_area(P(0, 0, 0), P(1, 0, 0), P(0, 1, 0), P(1, 1, 0))
                    assert abs(az[k, j, i] - want_z) <= 2.0 / Sf


def test_sphere_volume_and_cross_sections():
    """A sphere of radius 0.3: total fluid volume 1 - 4 pi r^3 / 3 and, on each plane
    x = i h, open area 1 - pi (r^2 - (x - 1/2)^2), to the interpolation error of the
    trilinear level set (O(h^2) over the surface: 2e-3 at 32^3)."""
    N, r = 32, 0.3
    psi = corners(N, lambda x, y, z: np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2) - r)
    vol = cc.volume_fractions(psi, S)
    assert abs(vol.sum() / N ** 3 - (1.0 - 4.0 * math.pi * r ** 3 / 3.0)) <= 2e-3
    ax, _, _ = cc.face_fractions(psi, S)
    for i in range(N):
        x = i / N
        want = 1.0 - math.pi * max(r * r - (x - 0.5) ** 2, 0.0)
        assert abs(ax[:, :, i].sum() / N ** 2 - want) <= 2e-3


@pytest.mark.parametrize("fluid_above", [True, False])
def test_merge_layer_closed_form(fluid_above):
    """A plane 1/8 of a cell from the top (or bottom) of layer k0: every cell of that
    layer has V = 1/8 and merges into its neighbour across the plane-parallel face
    towards the fluid; merged side faces carry 1 + 1/8 of their area."""
    N, k0 = 8, 3
    if fluid_above:
        z0 = (k0 + 7 / 8) / N
        psi = corners(N, lambda x, y, z: z - z0)
        tk = k0 + 1
    else:
        z0 = (k0 + 1 / 8) / N
        psi = corners(N, lambda x, y, z: z0 - z)
        tk = k0 - 1
    ax, ay, az = cc.face_fractions(psi, S)
    vol = cc.volume_fractions(psi, S)
    assert np.all(vol[k0] == 1 / 8)
    mt = cc.merge_targets(psi, vol)
    idx = np.arange(N ** 3).reshape(N, N, N)
    assert np.array_equal(mt[k0], idx[tk])
    assert np.all(np.delete(mt, k0, axis=0) == -1)
    rho = np.ones((N, N, N))
    lev = cc.cut_coeffs(rho, ax, ay, az, vol, mt, 1.0 / N)
    assert not lev.mask[k0].any() and lev.mask[tk].all()
    assert np.all(lev.bx[tk] == 1.125) and np.all(lev.by[tk] == 1.125)
    assert np.all(lev.bz[max(k0, tk)] == 0.0)   # the face between donor and target
    g = np.random.default_rng(3)
    f = g.standard_normal((N, N, N))
    fm = cc.merge_rhs(f, mt)
    assert np.all(fm[k0] == 0.0) and np.array_equal(fm[tk], f[tk] + f[k0])
    p = g.standard_normal((N, N, N))
    assert np.array_equal(cc.merge_fill(p, mt)[k0], p[tk])


def test_merge_direction_prefers_x_on_ties_and_respects_walls():
    """Equal |grad psi| in x and y picks x; a target beyond a z wall means no merge."""
    N = 8
    psi = corners(N, lambda x, y, z: (x - 0.5) + (y - 0.5) - 0.1 + 0.0 * z)
    gx, gy, gz = cc.centre_gradient(psi)
    vol = cc.volume_fractions(psi, S)
    mt = cc.merge_targets(psi, vol)
    small = (vol > 0) & (vol < 0.25)
    interior = small.copy()
    interior[:, :, [0, N - 1]] = False
    interior[:, [0, N - 1], :] = False
    cells = list(zip(*np.nonzero(interior)))
    assert cells
    for k, j, i in cells:
        assert abs(gx[k, j, i]) == abs(gy[k, j, i]) and gx[k, j, i] > 0
        assert mt[k, j, i] == (k * N + j) * N + (i + 1) or vol[k, j, (i + 1) % N] < 0.25
    psi = corners(N, lambda x, y, z: 0.125 / N - z)   # fluid only in the lowest 1/8 of layer 0
    vol = cc.volume_fractions(psi, S)
    assert np.all(vol[0] == 1 / 8) and np.all(vol[1:] == 0)
    assert np.all(cc.merge_targets(psi, vol) == -1)   # its target would lie beyond the wall


def test_merged_operator_is_symmetric_and_solvable():
    """The merged cut-cell operator of the wavy field at 16^3 is a symmetric 7-point
    operator with fractional coefficients; the sparse direct solve satisfies A p = P f."""
    import fields
    N = 16
    rho, psi = fields.wavy_cut(N)
    ax, ay, az = cc.face_fractions(psi, S)
    vol = cc.volume_fractions(psi, S)
    mt = cc.merge_targets(psi, vol)
    lev = cc.cut_coeffs(rho, ax, ay, az, vol, mt, 1.0 / N)
    assert np.any((ax > 0) & (ax < 1) & (lev.bx > 0)) and np.any(mt >= 0)
    g = np.random.default_rng(4)
    u, v = g.standard_normal((2, N, N, N))
    m = lev.mask
    u, v = np.where(m, u, 0.0), np.where(m, v, 0.0)
    assert abs(np.sum(u * apply(v, lev)) - np.sum(v * apply(u, lev))) <= 1e-9 * np.sum(np.abs(u * apply(v, lev)))
    f = project(cc.merge_rhs(g.standard_normal((N, N, N)), mt), m)
    p = exact.solve_sparse(lev, f)
    r = np.where(m, project(f, m) - apply(p, lev), 0.0)
    assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(f)
