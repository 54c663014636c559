"""Pins for oracle.operator: closed forms, identities and an independent assembly."""
import numpy as np
import pytest

from oracle.multigrid import dense_operator
from oracle.operator import (Level, apply, assemble, diagonal, face_coeffs_from_rho, face_list,
                             neighbour_sum, open_faces, project)
from tests.oracle_helpers import random_level


def cell_centres(N):
    c = (np.arange(N) + 0.5) / N
    return np.meshgrid(c, c, c, indexing="ij")  # z, y, x


@pytest.mark.parametrize("N", [8, 16])
@pytest.mark.parametrize("modes", [(1, 2, 3), (3, 1, 0), (0, 0, 1), (2, 0, 5), (4, 4, 7)])
def test_eigenfunctions_anisotropic(N, modes):
    """cos(2 pi a x) cos(2 pi b y) cos(pi c z) is an exact eigenvector of the
    constant-coefficient operator with periodic x, y and walls in z.  Distinct
    constants per axis catch any swap of axes or of face arrays."""
    a, b, c = modes
    z, y, x = cell_centres(N)
    betas = (0.7, 1.9, 3.1)   # x, y, z
    bx = np.full((N, N, N), betas[0])
    by = np.full((N, N, N), betas[1])
    bz = np.full((N, N, N), betas[2])
    bz[0] = 0.0
    lev = Level(bx, by, bz, np.ones((N, N, N), bool), 1.0 / N)
    for phase in (np.cos, np.sin):
        p = phase(2 * np.pi * a * x) * np.cos(2 * np.pi * b * y) * np.cos(np.pi * c * z)
        lam = -(4.0 * N * N) * (betas[0] * np.sin(np.pi * a / N) ** 2
                                + betas[1] * np.sin(np.pi * b / N) ** 2
                                + betas[2] * np.sin(np.pi * c / (2 * N)) ** 2)
        Ap = apply(p, lev)
        scale = max(abs(lam), 1.0)   # |p| <= 1; a vanishing Nyquist cosine is still checked
        assert np.abs(Ap - lam * p).max() <= 1e-12 * scale


def test_constant_in_null_space_and_compatibility():
    lev = random_level(8, 1, body=True, contrast=1000.0)
    N = lev.N
    ones = np.ones((N, N, N))
    assert np.abs(apply(ones, lev)).max() < 1e-9
    g = np.random.default_rng(2)
    for _ in range(3):
        p = g.standard_normal((N, N, N))
        # column sums of A vanish: the range of A has zero total
        assert abs(apply(p, lev).sum()) < 1e-9 * np.abs(apply(p, lev)).sum()


def test_symmetry_and_energy():
    lev = random_level(8, 3, body=True, contrast=100.0)
    N = lev.N
    g = np.random.default_rng(4)
    u = g.standard_normal((N, N, N))
    v = g.standard_normal((N, N, N))
    uAv = np.sum(u * apply(v, lev))
    vAu = np.sum(v * apply(u, lev))
    assert abs(uAv - vAu) <= 1e-12 * abs(uAv)
    # energy over faces: v.Av = -h^-2 sum_f beta_f (v_R - v_L)^2
    L, R, B = face_list(lev)
    vf = v.ravel()
    energy = -np.sum(B * (vf[R] - vf[L]) ** 2) / lev.h ** 2
    assert abs(np.sum(v * apply(v, lev)) - energy) <= 1e-12 * abs(energy)
    assert energy < 0


def test_dense_from_apply_matches_face_assembly():
    lev = random_level(4, 5, body=True, contrast=10.0)
    A1 = dense_operator(lev)
    A2 = assemble(lev).toarray()
    assert np.abs(A1 - A2).max() <= 1e-12 * np.abs(A2).max()
    assert np.abs(A1 - A1.T).max() <= 1e-12 * np.abs(A1).max()


def test_body_cells_decoupled():
    lev = random_level(8, 6, body=True)
    N = lev.N
    p = np.random.default_rng(7).standard_normal((N, N, N))
    Ap = apply(p, lev)
    assert np.all(Ap[~lev.mask] == 0)
    q = p.copy()
    q[~lev.mask] = 123.0          # body values never reach a fluid cell
    assert np.array_equal(apply(q, lev), Ap)


def test_diagonal_and_neighbour_sum_rebuild_operator():
    lev = random_level(8, 8, body=True, contrast=50.0)
    p = np.random.default_rng(9).standard_normal(lev.bx.shape)
    Ap = (neighbour_sum(p, lev) - diagonal(lev) * p) / lev.h ** 2
    assert np.abs(np.where(lev.mask, Ap, 0) - apply(p, lev)).max() <= 1e-12 * np.abs(Ap).max()


def test_face_coefficients_from_density():
    N = 8
    g = np.random.default_rng(10)
    rho = g.uniform(1e-3, 1.0, (N, N, N))
    mask = np.ones((N, N, N), np.uint8)
    mask[2:4, 3:5, 1:6] = 0
    bx, by, bz = face_coeffs_from_rho(rho, mask)
    ox, oy, oz = open_faces(mask)
    # equal densities give 1/rho; the face value depends symmetrically on both sides
    rc = np.full((N, N, N), 0.25)
    cx, cy, cz = face_coeffs_from_rho(rc, np.ones_like(mask))
    assert np.allclose(cx, 4.0) and np.allclose(cy, 4.0) and np.allclose(cz[1:], 4.0)
    assert np.all(cz[0] == 0)
    flipped = face_coeffs_from_rho(rho[:, :, ::-1].copy(), mask[:, :, ::-1].copy())[0]
    # reflecting x maps the low face of i to the low face of N-i (mod N)
    assert np.allclose(np.roll(flipped[:, :, ::-1], 1, axis=2), bx)
    assert np.all(bx[~ox] == 0) and np.all(by[~oy] == 0) and np.all(bz[~oz] == 0)
    # water/air face: 2/(1 + 0.001), between 1 (water) and 1000 (air)
    w = face_coeffs_from_rho(np.array([[[1.0, 1e-3]]]).repeat(2, 0).repeat(2, 1)[:, :, :2], np.ones((2, 2, 2), np.uint8))[0]
    assert 1.0 < w[0, 0, 1] < 1000.0


def test_interface_face_is_inverse_of_mean_density():
    """Reading C3: a face between water (rho = 1) and air (rho = 1e-3) takes 1/rho of the
    mean density, 2/(1 + 1e-3) ~ 1.998, close to the water value: the heavy fluid limits
    the flux.  The rejected reading (mean of 1/rho) would give (1 + 1000)/2 = 500.5.  A
    z column water below air puts the interface on a z face; x and y faces stay inside one
    fluid (1 and 1000)."""
    N = 4
    rho = np.ones((N, N, N))
    rho[N // 2:] = 1e-3
    bx, by, bz = face_coeffs_from_rho(rho, np.ones((N, N, N), np.uint8))
    want = 2.0 / (1.0 + 1e-3)
    assert np.all(bz[N // 2] == want)
    assert abs(bz[N // 2, 0, 0] - 500.5) > 400.0
    assert np.all(bz[1:N // 2] == 1.0) and np.allclose(bz[N // 2 + 1:], 1e3, rtol=1e-15, atol=0)
    assert np.all(bz[0] == 0.0)
    assert np.all(bx[:N // 2] == 1.0) and np.allclose(bx[N // 2:], 1e3, rtol=1e-15, atol=0)
    assert np.array_equal(bx, by)


def test_projection_removes_active_mean():
    mask = np.ones((4, 4, 4), bool)
    mask[0, 0, :2] = False
    f = np.random.default_rng(11).standard_normal((4, 4, 4)) + 3.0
    pf = project(f, mask)
    assert abs(pf[mask].sum()) < 1e-12 and np.all(pf[~mask] == 0)


def test_slab_residual_equals_whole_grid_residual():
    """The slab-by-slab residual used at 1024^3 equals the whole-array one (64^3 crest
    field with the body, a random p, slabs of 8 planes and a ragged last slab)."""
    import fields
    from oracle.multigrid import setup
    from oracle.operator import face_coeffs_from_rho, project
    from tests.slab_residual import slab_relres
    N = 64
    inp = fields.make("c5", N)
    H = setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    p = np.random.default_rng(9).standard_normal((N, N, N)) * 1e-3
    p = np.where(H.fine.mask, p, 0.0)
    fh = project(inp.f, H.fine.mask)
    r = np.where(H.fine.mask, fh - apply(p, H.fine), 0.0)
    want = float(np.linalg.norm(r) / np.linalg.norm(fh))
    for slab in (8, 24):
        got = slab_relres(inp.rho, inp.mask, inp.f, p, inp.h, slab=slab, workers=3)
        assert abs(got - want) <= 1e-12 * want, (slab, got, want)
