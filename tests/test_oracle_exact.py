"""Pins for oracle.exact: the three direct solvers against each other and the operator."""
import numpy as np
import pytest

import fields
from oracle import exact
from oracle.multigrid import setup
from oracle.operator import Level, apply, components, face_coeffs_from_rho, project
from tests.oracle_helpers import random_level, relerr


def check_solution(lev, f, p, tol):
    m = lev.mask
    r = project(f, m) - apply(p, lev)
    assert np.linalg.norm(r) <= tol * np.linalg.norm(project(f, m))
    assert abs(p[m].sum()) <= 1e-12 * np.abs(p).sum()
    assert np.all(p[~m] == 0) or np.abs(p[~m]).max() < 1e-14 * np.abs(p).max()


@pytest.mark.parametrize("N,seed", [(4, 70), (8, 71)])
def test_dense_and_sparse_agree_with_body(N, seed):
    lev = random_level(N, seed, body=True, contrast=1000.0)
    assert components(lev) == 1
    f = np.random.default_rng(seed).standard_normal((N, N, N))
    pd = exact.solve_dense(lev, f)
    ps = exact.solve_sparse(lev, f)
    check_solution(lev, f, pd, 1e-11)
    assert relerr(ps, pd) < 1e-11


def test_fft_matches_dense_at_contrast_1000():
    N = 8
    inp = fields.flat(N, 2.0)
    lev = setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h).fine
    pd = exact.solve_dense(lev, inp.f)
    pf = exact.solve_fft_z(lev, inp.f)
    assert relerr(pf, pd) < 1e-12


def test_fft_anisotropic_profiles_match_sparse():
    """Different z profiles for bx and by (and a random bz) catch a swapped axis."""
    N = 8
    g = np.random.default_rng(72)
    bxk, byk, bzk = g.uniform(0.5, 2.0, N), g.uniform(1e-3, 1.0, N), g.uniform(0.1, 5.0, N)
    bzk[0] = 0
    bcast = lambda v: np.broadcast_to(v[:, None, None], (N, N, N)).copy()
    lev = Level(bcast(bxk), bcast(byk), bcast(bzk), np.ones((N, N, N), bool), 1.0 / N)
    f = g.standard_normal((N, N, N))
    assert relerr(exact.solve_fft_z(lev, f), exact.solve_sparse(lev, f)) < 1e-12


def test_fft_residual_at_64():
    inp = fields.flat(64, 1.0)
    lev = setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h).fine
    p = exact.solve_fft_z(lev, inp.f)
    check_solution(lev, inp.f, p, 1e-12)


def test_fft_rejects_body_and_xy_variation():
    lev = random_level(4, 73, body=True)
    with pytest.raises(ValueError):
        exact.solve_fft_z(lev, np.zeros((4, 4, 4)))


def test_configs_have_one_fluid_component():
    for name in ("c1", "c2", "c5"):
        inp = fields.make(name, 32)
        lev = setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h).fine
        assert components(lev) == 1, name
