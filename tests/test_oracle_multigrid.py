"""Pins for oracle.multigrid: smoother, transfers, coarsening, coarse solve, cycles."""
import numpy as np
import pytest

from oracle import exact
from oracle.multigrid import (BLACK, RED, colour_mask, coarse_solve, coarsen, contraction,
                              dense_operator, prolong, prolong_add, pseudo_inverse, rbgs_half,
                              residual, restrict, setup, solve, solve_mixed, vcycle)
from oracle.operator import Level, apply, diagonal, face_coeffs_from_rho, project
from tests.oracle_helpers import random_hierarchy, random_level, relerr


# ------------------------------------------------------------------ smoother

@pytest.mark.parametrize("colour", [RED, BLACK])
def test_half_sweep_solves_its_colour(colour):
    """After a half-sweep every updated cell satisfies its own equation exactly,
    and cells of the other colour are untouched."""
    lev = random_level(8, 20, body=True, contrast=1000.0)
    N = lev.N
    g = np.random.default_rng(21)
    p = np.where(lev.mask, g.standard_normal((N, N, N)), 0.0)
    f = project(g.standard_normal((N, N, N)), lev.mask)
    q = rbgs_half(p, f, lev, colour)
    sel = colour_mask(N, colour) & lev.mask
    r = f - apply(q, lev)
    scale = np.abs(f).max() + np.abs(apply(p, lev)).max()
    assert np.abs(r[sel]).max() <= 1e-12 * scale
    assert np.array_equal(q[~sel], p[~sel])
    # red = (i + j + k) even
    assert colour_mask(4, RED)[0, 0, 0] and not colour_mask(4, RED)[0, 0, 1]


def test_half_sweeps_decrease_energy():
    """Gauss-Seidel minimises the energy functional one cell at a time, so with f = 0
    every half-sweep lowers E(e) = -e.Ae (A is negative semi-definite)."""
    lev = random_level(8, 22, body=True, contrast=1000.0)
    e = np.where(lev.mask, np.random.default_rng(23).standard_normal(lev.bx.shape), 0.0)
    zero = np.zeros_like(e)
    energy = -np.sum(e * apply(e, lev))
    for colour in (RED, BLACK, RED, BLACK):
        e = rbgs_half(e, zero, lev, colour)
        new = -np.sum(e * apply(e, lev))
        assert new < energy
        energy = new


# ------------------------------------------------------------------ transfers

def test_restriction_of_cosines():
    """Mean of two children of cos(theta (i+1/2)) is cos(theta/2) cos(2 theta (I+1/2))."""
    N = 16
    i = np.arange(N)
    I = np.arange(N // 2)
    for a, b, c in [(1, 2, 3), (3, 0, 1), (5, 7, 2)]:
        th = [2 * np.pi * a / N, 2 * np.pi * b / N, np.pi * c / N]   # x, y, z
        fine = (np.cos(th[2] * (i + 0.5))[:, None, None] * np.cos(th[1] * (i + 0.5))[None, :, None]
                * np.cos(th[0] * (i + 0.5))[None, None, :])
        coarse = (np.cos(2 * th[2] * (I + 0.5))[:, None, None] * np.cos(2 * th[1] * (I + 0.5))[None, :, None]
                  * np.cos(2 * th[0] * (I + 0.5))[None, None, :])
        factor = np.cos(th[0] / 2) * np.cos(th[1] / 2) * np.cos(th[2] / 2)
        assert np.abs(restrict(fine) - factor * coarse).max() < 1e-14


def test_restriction_conserves_sum():
    r = np.random.default_rng(30).standard_normal((8, 8, 8))
    assert abs(8 * restrict(r).sum() - r.sum()) < 1e-12


def test_prolongation_constants_and_linears():
    n = 8
    e = np.full((n, n, n), 2.5)
    assert np.allclose(prolong(e), 2.5, rtol=0, atol=1e-15)
    # trilinear interpolation is exact on trilinear functions away from wrap and walls
    Xc = (np.arange(n) + 0.5) * 2.0          # coarse centres in fine-cell units
    Xf = np.arange(2 * n) + 0.5
    Kc, Jc, Ic = np.meshgrid(Xc, Xc, Xc, indexing="ij")
    Kf, Jf, If = np.meshgrid(Xf, Xf, Xf, indexing="ij")
    fun = lambda z, y, x: 1.0 + 0.3 * x - 0.7 * y + 0.2 * z + 0.05 * x * y - 0.02 * y * z + 0.01 * x * y * z
    P = prolong(fun(Kc, Jc, Ic))
    inner = (slice(1, -1),) * 3
    assert np.abs(P[inner] - fun(Kf, Jf, If)[inner]).max() < 1e-12


def test_prolongation_wrap_and_walls():
    g = np.random.default_rng(31)
    e = g.standard_normal((4, 4, 4))
    P = prolong(e)
    # periodic x, y: shifting the coarse field by one cell shifts the fine field by two
    assert np.allclose(prolong(np.roll(e, 1, axis=2)), np.roll(P, 2, axis=2), atol=1e-15)
    assert np.allclose(prolong(np.roll(e, 1, axis=1)), np.roll(P, 2, axis=1), atol=1e-15)
    # mirror symmetry in every axis
    for ax in range(3):
        assert np.allclose(prolong(np.flip(e, ax)), np.flip(P, ax), atol=1e-15)
    # z walls: the outermost fine planes interpolate only in x, y from their parent plane
    ez = np.broadcast_to(np.arange(4.0)[:, None, None] ** 2, (4, 4, 4)).copy()
    Pz = prolong(ez)
    assert np.allclose(Pz[0], 0.0) and np.allclose(Pz[-1], 9.0)
    assert np.allclose(Pz[1], 0.75 * 0 + 0.25 * 1) and np.allclose(Pz[2], 0.75 * 1 + 0.25 * 0)


def test_prolong_add_skips_body():
    lev = random_level(8, 32, body=True)
    e = np.ones((4, 4, 4))
    p = np.zeros((8, 8, 8))
    q = prolong_add(p, e, lev)
    assert np.all(q[~lev.mask] == 0) and np.allclose(q[lev.mask], 1.0)


# ------------------------------------------------------------------ coarsening

def inject(e):
    return np.repeat(np.repeat(np.repeat(e, 2, 0), 2, 1), 2, 2)


@pytest.mark.parametrize("seed,body", [(40, False), (41, True), (42, True)])
def test_coarse_operator_is_half_galerkin_with_piecewise_constant_transfers(seed, body):
    """A_c e = 1/2 R A P0 e with P0 = injection to the 8 children and R = their mean:
    the coarse face sums the fluxes of its 4 fine faces, at twice the spacing."""
    lev = random_level(8, seed, body=body, contrast=1000.0)
    c = coarsen(lev)
    g = np.random.default_rng(seed + 100)
    for _ in range(3):
        e = g.standard_normal((4, 4, 4))
        lhs = apply(e, c)
        rhs = 0.5 * restrict(apply(inject(e), lev))
        assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


def test_coarsening_structure():
    N = 16
    lev = random_level(N, 43, body=True)
    c = coarsen(lev)
    assert c.h == 2 * lev.h and c.N == N // 2
    assert np.all(c.bz[0] == 0)
    any_child = lev.mask.reshape(8, 2, 8, 2, 8, 2).any(axis=(1, 3, 5))
    assert np.array_equal(c.mask, any_child & (diagonal(c) > 0))
    # constant coefficients stay constant
    b = np.full((N, N, N), 3.0)
    bz = b.copy()
    bz[0] = 0
    cc = coarsen(Level(b, b, bz, np.ones((N, N, N), bool), 1.0 / N))
    assert np.all(cc.bx == 3.0) and np.all(cc.bz[1:] == 3.0)


def test_flat_interface_stays_a_face_on_every_level():
    """z-only density with the interface at z = 1/2: every level keeps x, y
    coefficients constant per plane, and the mid-plane face keeps the fine value."""
    N = 32
    from fields import density_from_phi, flat_phi_column
    rho = np.broadcast_to(density_from_phi(flat_phi_column(N, 2.0))[:, None, None], (N, N, N)).copy()
    m = np.ones((N, N, N), np.uint8)
    H = setup(*face_coeffs_from_rho(rho, m), m, 1.0 / N)
    mid = H.fine.bz[N // 2, 0, 0]
    for lev in H.levels:
        assert np.all(lev.bx == lev.bx[:, :1, :1])
        assert lev.bz[lev.N // 2, 0, 0] == pytest.approx(mid, rel=1e-15)


# ------------------------------------------------------------------ coarse solve

def test_coarse_pseudo_inverse_matches_library_pinv():
    H = random_hierarchy(8, 50, body=True, contrast=1000.0)
    c = H.levels[-1]
    A = dense_operator(c)
    assert np.abs(H.coarse_pinv - np.linalg.pinv(A, rcond=1e-12)).max() <= 1e-9 * np.abs(H.coarse_pinv).max()
    assert np.abs(A @ H.coarse_pinv @ A - A).max() <= 1e-10 * np.abs(A).max()
    f = project(np.random.default_rng(51).standard_normal((4, 4, 4)), c.mask)
    e = coarse_solve(H, f)
    assert np.abs(apply(e, c) - f).max() <= 1e-10 * np.abs(f).max()
    assert abs(e[c.mask].sum()) < 1e-10 * np.abs(e).sum()


def test_pseudo_inverse_handles_isolated_null_vectors():
    A = np.diag([0.0, -2.0, -3.0])
    A[1, 2] = A[2, 1] = 1.0
    P = pseudo_inverse(A)
    assert np.allclose(P, np.linalg.pinv(A))


# ------------------------------------------------------------------ cycles and solves

def c1_like(N, smear=2.0):
    import fields
    inp = fields.flat(N, smear)
    return setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h), inp


def test_solve_reaches_fft_solution():
    H, inp = c1_like(32)
    p, hist = solve(H, inp.f, tol=1e-12, max_cycles=60)
    assert hist[-1] <= 1e-12
    assert relerr(p, exact.solve_fft_z(H.fine, inp.f)) < 1e-9
    assert contraction(hist) < 0.3


def test_solve_with_body_reaches_sparse_direct_solution():
    import fields
    inp = fields.wavy_body(32)
    H = setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    assert np.any(~H.fine.mask)
    p, hist = solve(H, inp.f, tol=1e-12, max_cycles=100)
    assert hist[-1] <= 1e-12
    assert relerr(p, exact.solve_sparse(H.fine, inp.f)) < 1e-9
    assert np.all(p[~H.fine.mask] == 0)
    assert abs(p[H.fine.mask].mean()) < 1e-14 * np.abs(p).max()


def test_warm_start_and_initial_history():
    H, inp = c1_like(16)
    p, hist = solve(H, inp.f, tol=1e-12)
    assert hist[0] == 1.0
    p2, hist2 = solve(H, inp.f, p0=p, tol=1e-12)
    assert len(hist2) == 1 and hist2[0] <= 1e-12


def test_mixed_refinement_reaches_fp64_solution():
    H, inp = c1_like(32, smear=1.0)
    pm, hm = solve_mixed(H, inp.f, tol=1e-12, max_steps=60)
    assert hm[-1] <= 1e-12
    assert relerr(pm, exact.solve_fft_z(H.fine, inp.f)) < 1e-9


def test_fp32_cycle_is_single_precision():
    H, inp = c1_like(16)
    from oracle.multigrid import fp32_levels
    lv = fp32_levels(H)
    assert lv[0].bx.dtype == np.float32
    r32 = project(inp.f, H.fine.mask).astype(np.float32)
    e = vcycle(H, np.zeros_like(r32), r32, lv)
    assert e.dtype == np.float32


def test_cycles_do_not_grow_with_grid():
    """The one multigrid claim of the paper: convergence does not degrade as the
    grid grows.  Cycles to 1e-10 for the flat-interface field at 16^3 .. 64^3."""
    counts = []
    for N in (16, 32, 64):
        H, inp = c1_like(N)
        _, hist = solve(H, inp.f, tol=1e-10, max_cycles=60)
        counts.append(len(hist) - 1)
    assert max(counts) - min(counts) <= 3, counts


def test_residual_zero_in_body():
    lev = random_level(8, 60, body=True)
    g = np.random.default_rng(61)
    r = residual(g.standard_normal((8, 8, 8)), project(g.standard_normal((8, 8, 8)), lev.mask), lev)
    assert np.all(r[~lev.mask] == 0)


# ------------------------------------------------------------------ flexible CG

def test_fcg_with_identity_preconditioner_is_plain_cg():
    """With a fixed symmetric preconditioner FCG(1) is preconditioned CG: with B = I its
    iterates equal scipy's conjugate gradients on the SPD matrix -A (same start, same
    right-hand side), iteration by iteration."""
    import scipy.sparse.linalg as spla
    from oracle.operator import assemble
    from oracle.multigrid import solve_fcg
    H = random_hierarchy(8, 90, body=True, contrast=100.0)
    lev = H.fine
    f = project(np.random.default_rng(91).standard_normal(lev.bx.shape), lev.mask)
    M = -assemble(lev)
    iters = []
    spla.cg(M, -f.ravel(), x0=np.zeros(f.size), rtol=1e-30, maxiter=6,
            callback=lambda xk: iters.append(xk.copy()))
    for k in (1, 3, 6):
        # hist index k after k iterations; FCG's p is gauge-projected at the end
        pk, hist = solve_fcg(H, f, tol=1e-300, max_iters=k, precond=lambda r: -r)
        want = project(iters[k - 1].reshape(f.shape), lev.mask)
        assert relerr(pk, want) <= 1e-10, k


def test_fcg_exact_preconditioner_converges_in_one_step():
    from oracle.multigrid import solve_fcg
    H = random_hierarchy(8, 92, body=True, contrast=1000.0)
    lev = H.fine
    f = project(np.random.default_rng(93).standard_normal(lev.bx.shape), lev.mask)
    A = dense_operator(lev)
    Ap = np.linalg.pinv(A, rcond=1e-12)
    p, hist = solve_fcg(H, f, tol=1e-12, max_iters=5, precond=lambda r: (Ap @ r.ravel()).reshape(r.shape))
    assert len(hist) == 2 and hist[-1] <= 1e-12


@pytest.mark.parametrize("mixed", [False, True])
def test_fcg_vcycle_reaches_exact_solution_in_fewer_iterations(mixed):
    import fields
    from oracle.multigrid import solve_fcg
    inp = fields.stokes_crest(32)
    H = setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    p, hist = solve_fcg(H, inp.f, tol=1e-12, max_iters=60, mixed=mixed)
    assert hist[-1] <= 1e-12
    assert relerr(p, exact.solve_sparse(H.fine, inp.f)) < 1e-9
    _, mg_hist = solve(H, inp.f, tol=1e-12, max_cycles=200)
    assert len(hist) < len(mg_hist)


# ------------------------------------------------------------------ coarsening ablation

def test_density_coarsening_same_fine_grid_and_constant_case():
    import fields
    from oracle.multigrid import setup_density_coarsening
    inp = fields.wavy_body(16)
    Hf = setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    Hd = setup_density_coarsening(inp.rho, inp.mask, inp.h)
    for a, b in ((Hf.fine.bx, Hd.fine.bx), (Hf.fine.by, Hd.fine.by), (Hf.fine.bz, Hd.fine.bz)):
        assert np.array_equal(a, b)
    assert all(np.array_equal(a.mask, b.mask) for a, b in zip(Hf.levels, Hd.levels))
    # constant density: both ways of coarsening give the same operators
    rho = np.full((16, 16, 16), 0.25)
    Hf = setup(*face_coeffs_from_rho(rho, inp.mask), inp.mask, inp.h)
    Hd = setup_density_coarsening(rho, inp.mask, inp.h)
    for a, b in zip(Hf.levels, Hd.levels):
        assert np.allclose(a.bx, b.bx, rtol=1e-15) and np.allclose(a.bz, b.bz, rtol=1e-15)


def test_density_coarsening_smooths_a_sharp_interface():
    """Two planes of water (rho 1) under two of air (1e-3): after one coarsening the
    face-product grid keeps 1/rho on the air plane's x faces, while averaging density
    first gives 2/(1 + 1e-3) on the interface plane - the interface is smeared."""
    N = 8
    rho = np.ones((N, N, N))
    rho[1:] = 1e-3          # water at k = 0; air above (the coarse cell K=0 straddles)
    m = np.ones((N, N, N), np.uint8)
    from oracle.multigrid import setup_density_coarsening
    Hf = setup(*face_coeffs_from_rho(rho, m), m, 1.0 / N)
    Hd = setup_density_coarsening(rho, m, 1.0 / N)
    # coarse K = 0 holds fine planes k = 0 (water) and k = 1 (air)
    assert Hf.levels[1].bx[0, 0, 0] == pytest.approx(0.5 * (1.0 + 1e3))
    assert Hd.levels[1].bx[0, 0, 0] == pytest.approx(1.0 / (0.5 * (1.0 + 1e-3)))


def test_fp32_density_level_is_the_rounded_operator_within_float_ulps():
    """The single-precision operator formed from the density: within 2 float32 ulps of
    round-to-nearest of the FP64 coefficients on open faces, exactly 0 on every face the
    FP64 setup closes (body, dropped cells, bottom wall)."""
    import fields
    from oracle.multigrid import fp32_density_level, setup
    from oracle.operator import face_coeffs_from_rho
    inp = fields.make("c2", 32)
    H = setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    lev = H.levels[0]
    l32 = fp32_density_level(inp.rho, lev)
    for b32, b64 in ((l32.bx, lev.bx), (l32.by, lev.by), (l32.bz, lev.bz)):
        assert b32.dtype == np.float32
        assert np.array_equal(b32 == 0, b64 == 0)
        ref = b64.astype(np.float32)
        ulp = np.spacing(np.maximum(ref, np.float32(1e-30)))
        assert np.max(np.abs(b32.astype(np.float64) - ref) / ulp) <= 2.0


def test_rhs_without_range_component_gives_zero():
    """Reading C21: f = 0 and a constant f project to zero (to rounding), so both
    solvers return p = 0 with the history [0] whatever the guess; an ordinary right-hand
    side is unaffected (history starts at 1 from p = 0)."""
    import oracle.multigrid as omg
    H = random_hierarchy(16, 41, body=True, contrast=1000.0)
    g = np.random.default_rng(42)
    guess = g.standard_normal((16, 16, 16))
    for f in (np.zeros((16, 16, 16)), np.full((16, 16, 16), 0.1)):
        assert omg.zero_range(f, project(f, H.fine.mask), H.fine.mask)
        for solver in (omg.solve, omg.solve_fcg):
            p, hist = solver(H, f, p0=guess)
            assert hist == [0.0] and not p.any()
    f = g.standard_normal((16, 16, 16))
    assert not omg.zero_range(f, project(f, H.fine.mask), H.fine.mask)
    _, hist = omg.solve(H, f, tol=1e-8)
    assert hist[0] == 1.0 and hist[-1] <= 1e-8


def test_mixed_refinement_on_density_form_fp32_operator():
    """Mixed refinement whose FP32 finest operator is formed from fl32(rho), as the
    cycles of a hierarchy set up from the density do on grids swept in one pass: it
    reaches the exact FP64 solution (FFT + Thomas) all the same, because the FP64
    residual decides convergence; its rate stays close to that of the rounded-beta
    cycles (the two FP32 operators differ by two float32 ulps at most)."""
    from oracle.multigrid import fp32_levels_from_rho
    H, inp = c1_like(32, smear=1.0)
    lv = fp32_levels_from_rho(H, inp.rho)
    assert lv[0].bx.dtype == np.float32 and len(lv) == len(H.levels)
    for a, b in zip(lv[1:], H.levels[1:]):
        assert np.array_equal(a.bx, b.bx.astype(np.float32))
    pm, hm = solve_mixed(H, inp.f, tol=1e-12, max_steps=60, lv32=lv)
    assert hm[-1] <= 1e-12
    assert relerr(pm, exact.solve_fft_z(H.fine, inp.f)) < 1e-9
    _, hr = solve_mixed(H, inp.f, tol=1e-12, max_steps=60)
    assert abs(len(hm) - len(hr)) <= 1
