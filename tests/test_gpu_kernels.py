"""Per-kernel parity of the HIP library against the oracle (element by element).

FP64 kernels: max |gpu - oracle| <= 1e-13 max |oracle| (the two differ only in the
order of additions and in fused multiply-adds).  FP32 kernels: against the oracle
run in numpy float32, <= 2e-5 max |oracle| (a few float32 ulps of the largest term).
Sizes span several thread blocks and, at 48^3-free power-of-two grids, the periodic
wrap and both z walls.
"""
import numpy as np
import pytest
import torch

from oracle import multigrid as omg
from oracle.operator import apply as oapply
from oracle.operator import face_coeffs_from_rho as orho
from oracle.operator import project
from tests.gpu_helpers import dev, host, maxrel, raw_problem

pytestmark = pytest.mark.gpu

TOL64 = 1e-13
TOL32 = 2e-5


@pytest.fixture(scope="module")
def problem():
    from paper_1410_2240_amd import MG
    N = 32
    bx, by, bz, mask = raw_problem(N, 1234, body=True, contrast=1000.0)
    H = omg.setup(bx, by, bz, mask, 1.0 / N)
    mg = MG(dev(bx), dev(by), dev(bz), dev(mask), mixed=True)
    return N, H, mg


def test_coeffs_from_rho_matches_oracle():
    from paper_1410_2240_amd import coeffs_from_rho
    import fields
    inp = fields.make("c2", 32)
    got = coeffs_from_rho(dev(inp.rho), dev(inp.mask))
    for g, want in zip(got, orho(inp.rho, inp.mask)):
        assert maxrel(host(g), want) <= 1e-15


def test_hierarchy_matches_oracle(problem):
    N, H, mg = problem
    assert mg.levels == len(H.levels)
    for l, lev in enumerate(H.levels):
        n, h = mg.level_info(l)
        assert n == lev.N and h == pytest.approx(lev.h, rel=1e-15)
        bx, by, bz, m = (host(t) for t in mg.level_coeffs(l))
        assert np.array_equal(m.astype(bool), lev.mask), l
        for g, want in ((bx, lev.bx), (by, lev.by), (bz, lev.bz)):
            assert maxrel(g, want) <= 1e-15, l


def test_apply_matches_oracle(problem):
    N, H, mg = problem
    p = np.random.default_rng(1).standard_normal((N, N, N))
    got = host(mg.apply(dev(p)))
    assert maxrel(got, oapply(p, H.fine)) <= TOL64


@pytest.mark.parametrize("level", [0, 1])
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("sweeps", [1, 2])
def test_smooth_fp64(problem, level, order, sweeps):
    N, H, mg = problem
    lev = H.levels[level]
    g = np.random.default_rng(10 + level)
    p = np.where(lev.mask, g.standard_normal(lev.bx.shape), 0.0)
    f = project(g.standard_normal(lev.bx.shape), lev.mask)
    want = omg.smooth(p, f, lev, sweeps, (omg.RED, omg.BLACK) if order == 0 else (omg.BLACK, omg.RED))
    got = host(mg.smooth(level, dev(p), dev(f), sweeps, order))
    assert maxrel(got, want) <= TOL64


@pytest.mark.parametrize("level", [0, 2])
def test_residual_restrict_fp64(problem, level):
    N, H, mg = problem
    lev = H.levels[level]
    g = np.random.default_rng(20 + level)
    p = np.where(lev.mask, g.standard_normal(lev.bx.shape), 0.0)
    f = project(g.standard_normal(lev.bx.shape), lev.mask)
    want = omg.restrict(omg.residual(p, f, lev))
    got = host(mg.residual_restrict(level, dev(p), dev(f)))
    assert maxrel(got, want) <= TOL64


@pytest.mark.parametrize("level", [0, 1, 2])
def test_prolong_add_fp64(problem, level):
    N, H, mg = problem
    lev = H.levels[level]
    n = lev.N // 2
    g = np.random.default_rng(30 + level)
    e = g.standard_normal((n, n, n))
    p = np.where(lev.mask, g.standard_normal(lev.bx.shape), 0.0)
    want = omg.prolong_add(p, e, lev)
    got = host(mg.prolong_add(level, dev(e), dev(p)))
    assert maxrel(got, want) <= TOL64


def test_coarse_solve_fp64(problem):
    N, H, mg = problem
    f = np.random.default_rng(40).standard_normal((4, 4, 4))
    want = omg.coarse_solve(H, f)
    got = host(mg.coarse_solve(dev(f)))
    # two eigen-solvers of the same 64 x 64 matrix: agreement limited by its conditioning
    lam = np.abs(np.linalg.eigvalsh(omg.dense_operator(H.levels[-1])))
    kappa = lam.max() / lam[lam > 1e-12 * lam.max()].min()
    assert maxrel(got, want) <= max(TOL64, 1e-15 * kappa)


def test_vcycle_fp64(problem):
    N, H, mg = problem
    lev = H.fine
    g = np.random.default_rng(50)
    p = np.where(lev.mask, g.standard_normal(lev.bx.shape), 0.0)
    f = project(g.standard_normal(lev.bx.shape), lev.mask)
    want = omg.vcycle(H, p, f)
    got = host(mg.vcycle(dev(p), dev(f)))
    assert maxrel(got, want) <= 1e-11


# ---------------------------------------------------------------- FP32 components

def f32(x):
    return np.asarray(x, np.float32)


@pytest.mark.parametrize("level", [0, 1])
def test_smooth_fp32(problem, level):
    N, H, mg = problem
    lev32 = omg.fp32_levels(H)[level]
    g = np.random.default_rng(60 + level)
    p = f32(np.where(lev32.mask, g.standard_normal(lev32.bx.shape), 0.0))
    f = f32(project(g.standard_normal(lev32.bx.shape), lev32.mask))
    want = omg.smooth(p, f, lev32, 2, (omg.RED, omg.BLACK))
    got = host(mg.smooth(level, dev(p), dev(f), 2, 0))
    assert got.dtype == np.float32
    assert maxrel(got, want) <= TOL32


def test_residual_restrict_and_prolong_fp32(problem):
    N, H, mg = problem
    lev32 = omg.fp32_levels(H)[0]
    g = np.random.default_rng(70)
    p = f32(np.where(lev32.mask, g.standard_normal(lev32.bx.shape), 0.0))
    f = f32(project(g.standard_normal(lev32.bx.shape), lev32.mask))
    want = omg.restrict(omg.residual(p, f, lev32))
    assert maxrel(host(mg.residual_restrict(0, dev(p), dev(f))), want) <= TOL32
    e = f32(g.standard_normal((N // 2,) * 3))
    want = omg.prolong_add(p, e, lev32)
    assert maxrel(host(mg.prolong_add(0, dev(e), dev(p))), want) <= TOL32


def test_vcycle_fp32_with_fp64_coarse(problem):
    N, H, mg = problem
    lv32 = omg.fp32_levels(H)
    g = np.random.default_rng(80)
    r = f32(project(g.standard_normal((N, N, N)), H.fine.mask))
    want = omg.vcycle(H, np.zeros_like(r), r, lv32)
    got = host(mg.vcycle(dev(np.zeros_like(r)), dev(r)))
    assert maxrel(got, want) <= 1e-4


def test_fp32_rejected_on_fp64_context():
    from paper_1410_2240_amd import MG, MGError
    N = 8
    bx, by, bz, mask = raw_problem(N, 5, body=False)
    mg = MG(dev(bx), dev(by), dev(bz), dev(mask))
    with pytest.raises(MGError):
        mg.smooth(0, dev(np.zeros((N, N, N), np.float32)), dev(np.zeros((N, N, N), np.float32)))


def test_coeff_grad_matches_oracle(problem):
    from oracle import adjoint
    N, H, mg = problem
    g = np.random.default_rng(90)
    mu = np.stack([np.where(H.fine.mask, g.standard_normal((N, N, N)), 0.0) for _ in range(3)])
    p = np.stack([np.where(H.fine.mask, g.standard_normal((N, N, N)), 0.0) for _ in range(3)])
    grho, faces = mg.coeff_grad(dev(mu), dev(p), faces=True)
    want_faces = adjoint.face_gradient(mu, p, H.fine)
    for got, want in zip(faces, want_faces):
        assert maxrel(host(got), want) <= TOL64
    assert maxrel(host(grho), adjoint.density_gradient(want_faces, H.fine)) <= TOL64


# ---------------------------------------------------------------- one-pass fused sweep

@pytest.fixture(scope="module")
def problem128():
    from paper_1410_2240_amd import MG
    N = 128
    bx, by, bz, mask = raw_problem(N, 4321, body=True, contrast=1000.0)
    H = omg.setup(bx, by, bz, mask, 1.0 / N)
    mg = MG(dev(bx), dev(by), dev(bz), dev(mask), mixed=True)
    return N, H, mg


@pytest.mark.parametrize("level", [0, 1])
@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("sweeps", [1, 2])
def test_fused_sweep_fp64(problem128, level, order, sweeps):
    """Grids of 64^3 and up run one red-black sweep per pass (128^3: tiles, z-chunks,
    halos; the 64^3 grid below it, from face arrays: 8^3 blocks with a 2-cell halo, one
    workgroup each): the result must equal the two half-sweeps of the oracle."""
    N, H, mg = problem128
    lev = H.levels[level]
    g = np.random.default_rng(100 + level)
    p = np.where(lev.mask, g.standard_normal(lev.bx.shape), 0.0)
    f = project(g.standard_normal(lev.bx.shape), lev.mask)
    want = omg.smooth(p, f, lev, sweeps, (omg.RED, omg.BLACK) if order == 0 else (omg.BLACK, omg.RED))
    got = host(mg.smooth(level, dev(p), dev(f), sweeps, order))
    assert maxrel(got, want) <= TOL64


def test_block_sweep_vcycle_64_matches_oracle(problem128):
    """A V-cycle from the 64^3 grid of the 128^3 hierarchy down: on the 64^3 and 32^3
    grids the block sweeps, the second pre-smoothing sweep also restricting its
    residual and the first post-smoothing sweep adding the prolongated correction
    first; against the oracle's cycle on the same grids."""
    from oracle.multigrid import Hierarchy
    from paper_1410_2240_amd import MG
    N, H, _ = problem128
    lev = H.levels[1]
    sub = Hierarchy(levels=H.levels[1:], coarse_pinv=H.coarse_pinv)
    mg = MG(dev(lev.bx), dev(lev.by), dev(lev.bz), dev(lev.mask.astype(np.uint8)), h=lev.h)
    g = np.random.default_rng(120)
    p = np.where(lev.mask, g.standard_normal(lev.bx.shape), 0.0)
    f = project(g.standard_normal(lev.bx.shape), lev.mask)
    want = omg.vcycle(sub, p, f)
    got = host(mg.vcycle(dev(p), dev(f)))
    assert maxrel(got, want) <= 1e-11


@pytest.mark.parametrize("level", [0, 1])
@pytest.mark.parametrize("order", [0, 1])
def test_fused_sweep_fp32(problem128, level, order):
    """FP32 sweeps of the 128^3 grid (one-pass, z-marching) and of the 64^3 grid below it
    (block sweeps) against the oracle in float32."""
    N, H, mg = problem128
    lev32 = omg.fp32_levels(H)[level]
    g = np.random.default_rng(110 + level)
    p = f32(np.where(lev32.mask, g.standard_normal(lev32.bx.shape), 0.0))
    f = f32(project(g.standard_normal(lev32.bx.shape), lev32.mask))
    want = omg.smooth(p, f, lev32, 2, (omg.RED, omg.BLACK) if order == 0 else (omg.BLACK, omg.RED))
    got = host(mg.smooth(level, dev(p), dev(f), 2, order))
    assert maxrel(got, want) <= TOL32


@pytest.mark.slow
def test_fused_sweep_512_whole_columns_matches_oracle():
    """From 512^3 up each workgroup sweeps its tile's whole z column in one chunk, with
    no chunk boundary: one FP64 density-form sweep of the bench field (wavy interface +
    body) at 512^3 against the oracle's two half-sweeps, every element."""
    import fields
    from oracle.operator import Level, diagonal
    from paper_1410_2240_amd import MG
    N = 512
    inp = fields.make("c2", N)
    print("512^3 sweep: oracle", flush=True)
    lev = Level(*orho(inp.rho, inp.mask), inp.mask.astype(bool), inp.h)
    lev.mask = lev.mask & (diagonal(lev) > 0)
    g = np.random.default_rng(512)
    p = np.where(lev.mask, g.standard_normal((N, N, N)), 0.0)
    f = g.standard_normal((N, N, N))
    want = omg.smooth(p, f, lev, 1, (omg.RED, omg.BLACK))
    del lev
    print("512^3 sweep: GPU", flush=True)
    mg = MG.from_rho(dev(inp.rho), dev(inp.mask))
    got = host(mg.smooth(0, dev(p), dev(f), 1, 0))
    assert maxrel(got, want) <= TOL64
