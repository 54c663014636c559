"""Pins for oracle.projection: divergence and projection against the operator."""
import numpy as np

import fields
from oracle import exact, projection
from oracle.multigrid import setup
from oracle.operator import apply, face_coeffs_from_rho, project as fproject
from tests.oracle_helpers import random_level


def face_field(N, seed):
    g = np.random.default_rng(seed)
    return tuple(g.standard_normal((N, N, N)) for _ in range(3))


def test_divergence_of_scaled_gradient_is_the_operator():
    """div(project(0, p)) = -dt A p for any p: the divergence and the face gradient
    compose to the pinned operator (signs, faces and walls must all agree)."""
    lev = random_level(8, 120, body=True, contrast=1000.0)
    p = np.random.default_rng(121).standard_normal(lev.bx.shape)
    zero = tuple(np.zeros_like(p) for _ in range(3))
    dt = 0.37
    U = projection.project(zero, p, lev, dt)
    got = projection.divergence(U, lev, dt=1.0)
    assert np.abs(got + dt * apply(p, lev)).max() <= 1e-12 * np.abs(dt * apply(p, lev)).max()


def test_divergence_telescopes_and_kills_constants():
    lev = random_level(8, 122, body=True)
    U = face_field(8, 123)
    f = projection.divergence(U, lev)
    assert abs(f[lev.mask].sum()) <= 1e-11 * np.abs(f).sum()
    const = tuple(np.full((8, 8, 8), c) for c in (1.5, -2.0, 0.0))   # no z flow (walls)
    lev_open = random_level(8, 124, body=False)
    assert np.abs(projection.divergence(const, lev_open)).max() < 1e-12


def test_projection_makes_the_field_divergence_free():
    """One Runge-Kutta stage: f = div(U + dt R)/dt, exact solve, projection -> div = 0."""
    inp = fields.wavy_body(16)
    H = setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    U, R = face_field(16, 125), face_field(16, 126)
    dt = 0.01
    f = projection.divergence(U, H.fine, dt, R)
    p = exact.solve_sparse(H.fine, f)
    Un = projection.project(U, p, H.fine, dt, R)
    d = projection.divergence(Un, H.fine)
    assert np.abs(d).max() <= 1e-9 * np.abs(f).max() * dt
    # closed faces carry no velocity
    from oracle.operator import open_faces
    ox, oy, oz = open_faces(H.fine.mask)
    assert np.all(Un[0][~ox] == 0) and np.all(Un[2][~oz] == 0)
    # the source is compatible
    assert abs(fproject(f, H.fine.mask).sum() - f.sum()) < 1e-9 * np.abs(f).sum()


def test_projection_is_idempotent():
    """Projecting a projected field changes nothing: its divergence is zero, so the next
    solve gives p = 0 (reading C21) and the projection returns the field as it is, the
    closed faces still 0.  Wavy interface with the body at 16^3, exact solves."""
    from oracle.multigrid import solve
    inp = fields.wavy_body(16)
    H = setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    U, R = face_field(16, 127), face_field(16, 128)
    dt = 0.01

    def projected(V, R):
        f = projection.divergence(V, H.fine, dt, R)
        p = exact.solve_sparse(H.fine, f)
        return projection.project(V, p, H.fine, dt, R)

    U1 = projected(U, R)
    f1 = projection.divergence(U1, H.fine, 1.0)
    scale = max(np.abs(u).max() for u in U1)
    p1, hist = solve(H, f1, tol=1e-12)
    # what is left of the divergence is rounding: its solution is rounding-sized too
    assert np.abs(p1).max() * np.abs(H.fine.bx).max() / H.fine.h <= 1e-9 * scale
    U2 = projection.project(U1, p1, H.fine, 1.0)
    for a, b in zip(U2, U1):
        assert np.abs(a - b).max() <= 1e-9 * scale
    # the projection of a field with no divergence and no forcing is the field itself
    U3 = projection.project(U1, np.zeros_like(p1), H.fine, dt)
    for a, b in zip(U3, U1):
        assert np.array_equal(a, b)
