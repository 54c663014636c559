"""Parity at the sizes the bench runs, in the launch configurations it times.

256^3 bench field (wavy interface + ellipsoid, density form on the finest grid):
every element of one FP64 sweep (the one-pass kernel, 128 x 16 tiles, 32-plane
z-chunks, so with chunk seams) and of two (the two-sweep pass, 32 x 32 tiles, 64-plane
chunks), of the residual + restriction, of the prolongation and of the whole
coarsened hierarchy against the oracle; FP64 kernels to <= 1e-13 max |oracle| (the
two differ in the order of additions and in fused multiply-adds), coefficients to
<= 1e-15.  Solutions at 128^3 and 256^3 against the oracle's multigrid solve of the
same field, relative L2 error <= 1e-9.

1024^3 Stokes crest + body (the headline workload; whole-column z-chunks): sampled
outputs of one sweep, of two sweeps in one two-sweep launch, of the residual +
restriction and of the prolongation, each recomputed by the oracle on an 8^3 window
around the sample (12^3 for two sweeps; tests/windows.py; the window rule is pinned
against whole-grid oracle passes in tests/test_windows.py).
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import fields
from oracle import multigrid as omg
from oracle.operator import face_coeffs_from_rho, project
from tests import windows as win
from tests.gpu_helpers import dev, host, maxrel, relerr

pytestmark = pytest.mark.gpu

TOL64 = 1e-13


def seeded(N, field, scale=1.0):
    """N(0, 1) per cell, drawn slab by slab from default_rng([1410, field, k])."""
    out = np.empty((N, N, N))

    def fill(k0, k1):
        for k in range(k0, k1):
            out[k] = np.random.default_rng([1410, field, k]).standard_normal((N, N)) * scale

    W = min(16, os.cpu_count() or 1)
    step = -(-N // W)
    with ThreadPoolExecutor(W) as ex:
        list(ex.map(lambda k0: fill(k0, min(N, k0 + step)), range(0, N, step)))
    return out


# ---------------------------------------------------------------- 256^3, every element

@pytest.fixture(scope="module")
def bench256():
    from paper_1410_2240_amd import MG
    N = 256
    print("256^3 c2: inputs and oracle hierarchy", flush=True)
    inp = fields.make("c2", N)
    H = omg.setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    mg = MG.from_rho(dev(inp.rho), dev(inp.mask))
    return inp, H, mg


def test_hierarchy_256_matches_oracle(bench256):
    inp, H, mg = bench256
    assert mg.levels == len(H.levels) == 7
    for l, lev in enumerate(H.levels):
        print(f"256^3 c2: level {l} coefficients", flush=True)
        bx, by, bz, m = (host(t) for t in mg.level_coeffs(l))
        assert np.array_equal(m.astype(bool), lev.mask), l
        for g, want in ((bx, lev.bx), (by, lev.by), (bz, lev.bz)):
            assert maxrel(g, want) <= 1e-15, l


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("sweeps", [1, 2])
def test_sweep_256_matches_oracle(bench256, order, sweeps):
    """The finest grid's FP64 density-form smoother in both its launches: one sweep is
    the one-pass kernel (128 x 16 tiles, 32-plane z-chunks, eight chunk seams per
    column), two sweeps are one launch of the two-sweep pass that every V-cycle runs
    (32 x 32 tiles, 64-plane chunks); both orders."""
    inp, H, mg = bench256
    lev = H.fine
    g = np.random.default_rng(2560 + 2 * order + sweeps)
    p = np.where(lev.mask, g.standard_normal(lev.bx.shape), 0.0)
    f = project(inp.f, lev.mask)
    print(f"256^3 c2: sweep order={order} sweeps={sweeps}: oracle", flush=True)
    want = omg.smooth(p, f, lev, sweeps, (omg.RED, omg.BLACK) if order == 0 else (omg.BLACK, omg.RED))
    print(f"256^3 c2: sweep order={order} sweeps={sweeps}: GPU", flush=True)
    got = host(mg.smooth(0, dev(p), dev(f), sweeps, order))
    assert maxrel(got, want) <= TOL64


def test_residual_restrict_256_matches_oracle(bench256):
    inp, H, mg = bench256
    lev = H.fine
    g = np.random.default_rng(2570)
    p = np.where(lev.mask, g.standard_normal(lev.bx.shape), 0.0)
    f = project(inp.f, lev.mask)
    print("256^3 c2: residual + restriction", flush=True)
    want = omg.restrict(omg.residual(p, f, lev))
    got = host(mg.residual_restrict(0, dev(p), dev(f)))
    assert maxrel(got, want) <= TOL64


@pytest.mark.parametrize("level", [0, 1])
def test_prolong_add_256_matches_oracle(bench256, level):
    inp, H, mg = bench256
    lev = H.levels[level]
    n = lev.N // 2
    g = np.random.default_rng(2580 + level)
    e = g.standard_normal((n, n, n))
    p = np.where(lev.mask, g.standard_normal(lev.bx.shape), 0.0)
    print(f"256^3 c2: prolongation level {level}", flush=True)
    want = omg.prolong_add(p, e, lev)
    got = host(mg.prolong_add(level, dev(e), dev(p)))
    assert maxrel(got, want) <= TOL64


# ---------------------------------------------------------------- solutions of the bench field

def solution_case(N):
    from paper_1410_2240_amd import MG
    print(f"{N}^3 c2: oracle flexible-CG solve to 1e-12", flush=True)
    inp = fields.make("c2", N)
    H = omg.setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    want, hist = omg.solve_fcg(H, inp.f, tol=1e-12, max_iters=80)
    assert hist[-1] <= 1e-12
    del H
    for mixed in (False, True):
        for krylov in (False, True):
            print(f"{N}^3 c2: GPU mixed={mixed} krylov={krylov}", flush=True)
            mg = MG.from_rho(dev(inp.rho), dev(inp.mask), mixed=mixed, krylov=krylov)
            p, h, st = mg.solve(dev(inp.f), tol=1e-12, max_cycles=200)
            err = relerr(host(p), want)
            print(f"{N}^3 c2: mixed={mixed} krylov={krylov} cycles={st['cycles']} p error {err:.2e}", flush=True)
            assert err <= 1e-9, (mixed, krylov, err, h[-1])
            del mg, p
            torch.cuda.empty_cache()


def test_bench_field_128_solution_matches_oracle():
    """FP64 and mixed, V-cycles and flexible CG, all to 1e-12, against the oracle's
    multigrid (flexible CG) solution of the same field to 1e-12."""
    solution_case(128)


@pytest.mark.slow
def test_bench_field_256_solution_matches_oracle():
    """The bench field at its full size (256^3): p against the oracle's solution."""
    solution_case(256)


# ---------------------------------------------------------------- mixed precision: the FP32 operator the GPU runs

def test_mixed_history_and_fp32_cycle_follow_the_density_form_oracle():
    """On a 64^3 hierarchy set up from rho the FP32 cycles form their finest faces from
    fl32(rho) (reading C14): one FP32 V-cycle against the oracle's cycle on that FP32
    hierarchy (element by element, FP32 arithmetic on both sides), and the refinement
    history step by step against the oracle's mixed refinement on it."""
    from paper_1410_2240_amd import MG
    N = 64
    inp = fields.make("c2", N)
    H = omg.setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    lv32 = omg.fp32_levels_from_rho(H, inp.rho)
    mg = MG.from_rho(dev(inp.rho), dev(inp.mask), mixed=True)
    r32 = project(inp.f, H.fine.mask).astype(np.float32)
    want = omg.vcycle(H, np.zeros_like(r32), r32, lv32)
    got = host(mg.vcycle(dev(np.zeros_like(r32)), dev(r32)))
    assert got.dtype == np.float32
    assert maxrel(got, want) <= 1e-4
    _, hist_o = omg.solve_mixed(H, inp.f, tol=1e-12, max_steps=100, lv32=lv32)
    _, hist_g, st = mg.solve(dev(inp.f), tol=1e-12, max_cycles=100)
    assert abs(len(hist_g) - len(hist_o)) <= 1, (len(hist_g), len(hist_o))
    for a, b in zip(hist_g, hist_o):
        if b > 1e-10:   # above the FP64 rounding of the residual itself
            assert abs(a - b) <= 1e-3 * b, (a, b)


# ---------------------------------------------------------------- 1024^3, sampled outputs

@pytest.fixture(scope="module")
def crest1024():
    from paper_1410_2240_amd import MG
    N = 1024
    print("1024^3 c5: generating the inputs", flush=True)
    inp = fields.make("c5", N)
    p = seeded(N, 7)
    p[inp.mask == 0] = 0.0
    rho, mask = dev(inp.rho), dev(inp.mask)
    print("1024^3 c5: hierarchy", flush=True)
    mg = MG.from_rho(rho, mask)
    return inp, p, rho, mask, mg


def sample_cells(inp, rng, count=160):
    """Random cells, plus cells at tile edges (x = 0, 127, 128 mod 128; y = 0, 15, 16 mod
    16), at both z walls, next to the body and on the interface."""
    N = inp.N
    cells = [tuple(int(v) for v in rng.integers(0, N, 3)) for _ in range(count)]
    for k in (0, 1, N - 2, N - 1):
        cells.append((k, int(rng.integers(0, N)), int(rng.integers(0, N))))
    for i in (0, 127, 128, N - 1):
        cells.append((int(rng.integers(0, N)), int(rng.integers(0, N)), i))
    for j in (0, 15, 16, N - 1):
        cells.append((int(rng.integers(0, N)), j, int(rng.integers(0, N))))
    body = np.argwhere(inp.mask[N // 2 - 40:N // 2 + 40] == 0)
    for b in body[rng.integers(0, len(body), 16)]:
        cells.append((int(b[0]) + N // 2 - 40, int(b[1]), (int(b[2]) + 1) % N))   # next to the body in x
    # the interface: where rho changes fastest along z in the column at a random (j, i)
    for _ in range(16):
        j, i = (int(v) for v in rng.integers(0, N, 2))
        col = inp.rho[:, j, i]
        k = int(np.argmax(np.abs(np.diff(col))))
        cells.append((k, j, i))
    return cells


@pytest.mark.slow
@pytest.mark.parametrize("order", [0, 1])
def test_sweep_1024_sampled_outputs_match_oracle(crest1024, order):
    """One FP64 density-form sweep of the headline grid (whole-column chunks)."""
    inp, p, rho, mask, mg = crest1024
    print(f"1024^3 c5: sweep order={order}: GPU", flush=True)
    out = mg.smooth(0, dev(p), dev(inp.f), 1, order)
    cells = sample_cells(inp, np.random.default_rng(10240 + order))
    got = win.gather(out, cells)
    del out
    torch.cuda.empty_cache()
    print(f"1024^3 c5: sweep order={order}: oracle on {len(cells)} windows", flush=True)
    for c, gv in zip(cells, got):
        wv, scale = win.sweep_at(inp.rho, inp.mask, p, inp.f, inp.h, c, order)
        assert abs(gv - wv) <= TOL64 * scale, (c, gv, wv)


@pytest.mark.slow
@pytest.mark.parametrize("order", [0, 1])
def test_two_sweeps_1024_sampled_outputs_match_oracle(crest1024, order):
    """Two FP64 density-form sweeps of the headline grid in one launch of the two-sweep
    pass (32 x 32 tiles, whole-column chunks, the launch the bench times), each sample
    recomputed by the oracle's two sweeps on a 12^3 window."""
    inp, p, rho, mask, mg = crest1024
    print(f"1024^3 c5: two sweeps order={order}: GPU", flush=True)
    out = mg.smooth(0, dev(p), dev(inp.f), 2, order)
    cells = sample_cells(inp, np.random.default_rng(10260 + order))
    got = win.gather(out, cells)
    del out
    torch.cuda.empty_cache()
    print(f"1024^3 c5: two sweeps order={order}: oracle on {len(cells)} windows", flush=True)
    for c, gv in zip(cells, got):
        wv, scale = win.sweep_at(inp.rho, inp.mask, p, inp.f, inp.h, c, order, sweeps=2)
        assert abs(gv - wv) <= TOL64 * scale, (c, gv, wv)


@pytest.mark.slow
def test_residual_restrict_1024_sampled_outputs_match_oracle(crest1024):
    inp, p, rho, mask, mg = crest1024
    print("1024^3 c5: residual + restriction: GPU", flush=True)
    fc = mg.residual_restrict(0, dev(p), dev(inp.f))
    coarse = [(k // 2, j // 2, i // 2) for k, j, i in sample_cells(inp, np.random.default_rng(10250))]
    got = win.gather(fc, coarse)
    del fc
    torch.cuda.empty_cache()
    print(f"1024^3 c5: residual + restriction: oracle on {len(coarse)} windows", flush=True)
    for c, gv in zip(coarse, got):
        wv, scale = win.residual_restrict_at(inp.rho, inp.mask, p, inp.f, inp.h, c)
        assert abs(gv - wv) <= TOL64 * scale, (c, gv, wv)


@pytest.mark.slow
def test_prolong_add_1024_sampled_outputs_match_oracle(crest1024):
    inp, p, rho, mask, mg = crest1024
    e = seeded(inp.N // 2, 8)
    print("1024^3 c5: prolongation: GPU", flush=True)
    out = mg.prolong_add(0, dev(e), dev(p))
    cells = sample_cells(inp, np.random.default_rng(10260))
    got = win.gather(out, cells)
    del out
    torch.cuda.empty_cache()
    print(f"1024^3 c5: prolongation: oracle on {len(cells)} windows", flush=True)
    for c, gv in zip(cells, got):
        wv, scale = win.prolong_add_at(inp.rho, inp.mask, p, e, inp.h, c)
        assert abs(gv - wv) <= TOL64 * scale, (c, gv, wv)
