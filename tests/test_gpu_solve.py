"""Solve parity: GPU solutions against the oracle's exact solutions and multigrid.

Bar: relative L2 error on p <= 1e-9 (FP64, and mixed precision after convergence).
Parity runs solve to 1e-12 so that the error bound (condition number x residual)
sits well below the bar; the bench workloads at full size are checked through the
oracle's own residual of the GPU solution, which holds at any size.
"""
import numpy as np
import pytest
import torch

import fields
from oracle import exact
from oracle import multigrid as omg
from oracle.operator import apply as oapply
from oracle.operator import project
from tests.gpu_helpers import dev, host, mg_from_inputs, relerr, workload

pytestmark = pytest.mark.gpu


def oracle_relres(inp, H, p):
    fh = project(inp.f, H.fine.mask)
    r = np.where(H.fine.mask, fh - oapply(p, H.fine), 0.0)
    return float(np.linalg.norm(r) / np.linalg.norm(fh))


@pytest.mark.parametrize("mixed", [False, True])
def test_flat_32_matches_fft_exact(mixed):
    inp, H = workload("c1", 32)
    mg = mg_from_inputs(inp, mixed)
    p, hist, st = mg.solve(dev(inp.f), tol=1e-12, max_cycles=60)
    pe = exact.solve_fft_z(H.fine, inp.f)
    assert relerr(host(p), pe) <= 1e-9
    assert hist[-1] <= 1e-12 and st["status"] == 0
    # FP64 history follows the oracle's multigrid cycle by cycle
    if not mixed:
        _, ohist = omg.solve(H, inp.f, tol=1e-12, max_cycles=60)
        assert len(hist) == len(ohist)
        for a, b in zip(hist, ohist):
            # cycle-by-cycle agreement down to the rounding floor of the residual norm
            assert abs(a - b) <= 1e-6 * b + 1e-15


def test_dense_cross_check_8():
    inp, H = workload("c1", 8)
    mg = mg_from_inputs(inp)
    p, hist, _ = mg.solve(dev(inp.f), tol=1e-13, max_cycles=80)
    assert relerr(host(p), exact.solve_dense(H.fine, inp.f)) <= 1e-9


def test_constant_density_eigenfunction():
    """rho = 1 everywhere: f = lambda * cos mode (a,b,c) = (1,2,3) gives p = that mode."""
    N = 32
    c = (np.arange(N) + 0.5) / N
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    mode = np.cos(2 * np.pi * x) * np.cos(4 * np.pi * y) * np.cos(3 * np.pi * z)
    lam = -(4.0 * N * N) * (np.sin(np.pi / N) ** 2 + np.sin(2 * np.pi / N) ** 2 + np.sin(3 * np.pi / (2 * N)) ** 2)
    rho = np.ones((N, N, N))
    mask = np.ones((N, N, N), np.uint8)
    from paper_1410_2240_amd import MG
    mg = MG.from_rho(dev(rho), dev(mask))
    p, _, _ = mg.solve(dev(lam * mode), tol=1e-13, max_cycles=60)
    assert relerr(host(p), mode) <= 1e-9


@pytest.mark.parametrize("mixed", [False, True])
def test_wavy_body_32_matches_sparse_direct(mixed):
    inp, H = workload("c2", 32)
    mg = mg_from_inputs(inp, mixed)
    p, hist, st = mg.solve(dev(inp.f), tol=1e-12, max_cycles=100)
    pe = exact.solve_sparse(H.fine, inp.f)
    got = host(p)
    assert relerr(got, pe) <= 1e-9
    assert np.all(got[inp.mask == 0] == 0)
    assert abs(got[inp.mask == 1].mean()) <= 1e-12 * np.abs(got).max()


@pytest.mark.parametrize("name,N", [("c2", 64), ("c5", 64), ("c3", 64)])
def test_workloads_64_match_oracle_multigrid(name, N):
    inp, H = workload(name, N)
    want, _ = omg.solve(H, inp.f, tol=1e-12, max_cycles=100)
    for mixed in (False, True):
        mg = mg_from_inputs(inp, mixed)
        p, hist, _ = mg.solve(dev(inp.f), tol=1e-12, max_cycles=100)
        assert relerr(host(p), want) <= 1e-9, (name, mixed)


def test_flat_128_mixed_matches_fft():
    inp, H = workload("c3", 128)
    pe = exact.solve_fft_z(H.fine, inp.f)
    for mixed in (False, True):
        p, hist, st = mg_from_inputs(inp, mixed).solve(dev(inp.f), tol=1e-12, max_cycles=100)
        assert relerr(host(p), pe) <= 1e-9, mixed


def test_flat_512_fp64_and_mixed_match_fft_exact():
    """The 512^3 mixed-precision workload at its full size (1-cell smear, density ratio
    1000): FP64 V-cycles and FP32 cycles inside FP64 refinement, and flexible CG with
    either cycle, all to 1e-12, against the oracle's exact FFT + Thomas solution (the
    sweeps march whole z columns at this size)."""
    import fields as F
    from oracle.operator import Level, face_coeffs_from_rho
    from paper_1410_2240_amd import MG
    inp = F.make("c3", 512)
    print("512^3 c3: oracle FFT solve", flush=True)
    lev = Level(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask.astype(bool), inp.h)
    pe = exact.solve_fft_z(lev, inp.f)
    del lev
    for mixed in (False, True):
        for krylov in (False, True):
            print(f"512^3 c3: GPU solve mixed={mixed} krylov={krylov}", flush=True)
            mg = MG.from_rho(dev(inp.rho), dev(inp.mask), mixed=mixed, krylov=krylov)
            p, hist, st = mg.solve(dev(inp.f), tol=1e-12, max_cycles=100)
            assert relerr(host(p), pe) <= 1e-9, (mixed, krylov, hist[-1])
            del p, mg
            torch.cuda.empty_cache()


def test_bench_workload_256_residual_by_oracle():
    """The benchmarked 256^3 wavy-interface + body workload, solved as the benchmark
    does (FP64 and mixed, tol 1e-10): the oracle recomputes the residual in FP64."""
    inp, H = workload("c2", 256)
    for mixed in (False, True):
        p, hist, st = mg_from_inputs(inp, mixed).solve(dev(inp.f), tol=1e-10, max_cycles=100)
        rr = oracle_relres(inp, H, host(p))
        assert rr <= 1.05e-10, (mixed, rr, hist[-3:])
        assert abs(rr - hist[-1]) <= 1e-3 * hist[-1] + 1e-14


@pytest.mark.slow
def test_crest_1024_full_size_fcg_residual_by_oracle():
    """The 1024^3 Stokes-crest + body workload at its full size, as it is timed: flexible
    CG with FP64 and with mixed-precision cycles, both to 1e-10.  The oracle recomputes
    each solution's residual in FP64, slab by slab (no oracle solve fits at this size);
    the mixed solution is compared with the GPU's own FP64 one."""
    from paper_1410_2240_amd import MG
    from tests.slab_residual import slab_relres
    print("1024^3 c5: generating the inputs", flush=True)
    inp = fields.make("c5", 1024)
    rho, mask, f = dev(inp.rho), dev(inp.mask), dev(inp.f)
    sols = {}
    for mixed in (False, True):
        print(f"1024^3 c5: GPU flexible CG mixed={mixed}", flush=True)
        mg = MG.from_rho(rho, mask, mixed=mixed, krylov=True)
        p, hist, st = mg.solve(f, tol=1e-10, max_cycles=200)
        assert st["status"] == 0 and hist[-1] <= 1e-10, (mixed, st, hist[-3:])
        del mg
        ph = host(p)
        del p
        torch.cuda.empty_cache()
        print(f"1024^3 c5: oracle residual mixed={mixed}", flush=True)
        rr = slab_relres(inp.rho, inp.mask, inp.f, ph, inp.h)
        print(f"1024^3 c5: mixed={mixed} steps={len(hist) - 1} gpu {hist[-1]:.3e} oracle {rr:.3e}", flush=True)
        assert rr <= 1.05e-10, (mixed, rr, hist[-3:])
        assert abs(rr - hist[-1]) <= 1e-3 * hist[-1] + 1e-14
        sols[mixed] = ph
    d = relerr(sols[True], sols[False])
    print(f"1024^3 c5: mixed vs FP64 solution {d:.3e}", flush=True)
    assert d <= 1e-9


def test_repeatable_bitwise():
    inp, _ = workload("c2", 32)
    mg = mg_from_inputs(inp)
    a, ha, _ = mg.solve(dev(inp.f), tol=1e-12)
    b, hb, _ = mg.solve(dev(inp.f), tol=1e-12)
    assert torch.equal(a, b) and ha == hb


def test_batch_and_warm_start():
    inp, H = workload("c1", 32)
    mg = mg_from_inputs(inp)
    fb = fields.batch_rhs(inp.mask, 3)
    p, hists, st = mg.solve(dev(fb), tol=1e-12)
    for b in range(3):
        assert relerr(host(p[b]), exact.solve_fft_z(H.fine, fb[b])) <= 1e-9
    assert len(hists) == 3 and st["cycles"] == sum(len(h) - 1 for h in hists)
    p2, h2, _ = mg.solve(dev(fb[0]), p=p[0].clone(), tol=1e-12)
    assert len(h2) == 1   # already converged


def test_mixed_batch_and_warm_start_64():
    """Mixed refinement on a 64^3 density-form grid, where each step's FP64 update is
    formed inside the next residual pass and the iterate alternates between the caller's
    p and the solver's second buffer: a batch of three right-hand sides against the
    exact solutions, solves that end in either buffer, and warm starts."""
    from paper_1410_2240_amd import MG
    inp, H = workload("c1", 64)
    mg = MG.from_rho(dev(inp.rho), dev(inp.mask), mixed=True)
    fb = fields.batch_rhs(inp.mask, 3)
    p, hists, st = mg.solve(dev(fb), tol=1e-12)
    for b in range(3):
        assert relerr(host(p[b]), exact.solve_fft_z(H.fine, fb[b])) <= 1e-9
    steps = {len(h) - 1 for h in hists}
    # from a rough warm start, an odd and an even number of steps
    for tol in (1e-6, 1e-7, 1e-8):
        q, hq, _ = mg.solve(dev(fb[0]), tol=tol)
        steps.add(len(hq) - 1)
        w, hw, _ = mg.solve(dev(fb[0]), p=q.clone(), tol=1e-12)
        assert relerr(host(w), exact.solve_fft_z(H.fine, fb[0])) <= 1e-9
        assert len(hw) < len(hists[0])
    assert any(s % 2 for s in steps) and any(s % 2 == 0 for s in steps), steps


@pytest.mark.parametrize("N,mixed,krylov,lanes", [(64, False, False, 2), (64, True, False, 2), (64, False, True, 3),
                                                  (64, True, True, 2), (32, False, False, 1), (128, False, False, 3),
                                                  (256, False, True, 2)])
def test_lanes_give_the_one_by_one_results(N, mixed, krylov, lanes):
    """A batch solved on 1 + lanes concurrent streams: every item's solution and history
    bit for bit those of the one-at-a-time loop (five items, so lanes get unequal
    shares), the solutions within the bar of the exact ones, and the caller's stream
    ordered after the lanes (the comparison below runs on it without a sync)."""
    from paper_1410_2240_amd import MG
    inp, H = workload("c1", N)
    fb = fields.batch_rhs(inp.mask, 5)
    one = MG.from_rho(dev(inp.rho), dev(inp.mask), mixed=mixed, krylov=krylov)
    par = MG.from_rho(dev(inp.rho), dev(inp.mask), mixed=mixed, krylov=krylov, lanes=lanes)
    p1, h1, s1 = one.solve(dev(fb), tol=1e-12)
    pl, hl, sl = par.solve(dev(fb), tol=1e-12)
    assert torch.equal(p1, pl)
    assert h1 == hl and s1["cycles"] == sl["cycles"] and s1["status"] == sl["status"] == 0
    for b in (0, 4):
        assert relerr(host(pl[b]), exact.solve_fft_z(H.fine, fb[b])) <= 1e-9
    # a second batch on the same lanes, and a single item (no lane used)
    p2, h2, _ = par.solve(dev(fb[:2]), tol=1e-12)
    assert torch.equal(p2, p1[:2]) and h2 == h1[:2]
    p3, h3, _ = par.solve(dev(fb[3]), tol=1e-12)
    assert torch.equal(p3, p1[3]) and h3 == h1[3]


def test_lanes_follow_the_callers_stream():
    """On a side stream: the right-hand sides are produced there just before the call,
    and the solutions are consumed there just after it, with no synchronisation in
    between.  Lanes must start after the first and finish before the second."""
    from paper_1410_2240_amd import MG
    inp, _ = workload("c1", 64)
    fb = dev(fields.batch_rhs(inp.mask, 4))
    ref, _, _ = MG.from_rho(dev(inp.rho), dev(inp.mask)).solve(fb, tol=1e-12)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        par = MG.from_rho(dev(inp.rho), dev(inp.mask), lanes=3)
        for _ in range(2):
            f = torch.empty_like(fb)
            f.copy_(fb * 2.0)            # queued on the side stream just before the solve
            p, _, st = par.solve(f, tol=1e-12)
            q = p * 0.5                  # queued on the side stream just after it
    torch.cuda.synchronize()
    assert st["status"] == 0
    assert torch.equal(q, ref)   # scaling by 2 is exact in every step of the solve


def test_lanes_report_statuses_in_batch_order():
    """Items that stop early on lanes: the same statuses, histories and first message as
    the one-at-a-time loop; argument errors before any work; lanes added once only."""
    from paper_1410_2240_amd import MG, MGError
    from paper_1410_2240_amd import _lib
    inp, _ = workload("c1", 64)
    fb = fields.batch_rhs(inp.mask, 4)
    bad = fb.copy()
    bad[2, 3, 3, 3] = np.nan
    one = MG.from_rho(dev(inp.rho), dev(inp.mask))
    par = MG.from_rho(dev(inp.rho), dev(inp.mask), lanes=3)
    for f, code in ((fb, _lib.MG_ENOCONV), (bad, _lib.MG_EBREAKDOWN)):
        maxc = 2 if code == _lib.MG_ENOCONV else 100
        r1 = one.solve(dev(f), tol=1e-12, max_cycles=maxc, raise_on_fail=False)
        m1 = _lib.last_error()
        rl = par.solve(dev(f), tol=1e-12, max_cycles=maxc, raise_on_fail=False)
        ml = _lib.last_error()
        assert r1[2]["status"] == rl[2]["status"] == code
        assert r1[1] == rl[1] and torch.equal(r1[0], rl[0])
        assert ml and m1 == ml
    # a zero right-hand side among others: p = 0 and the history [0] for it alone
    zf = fb.copy()
    zf[1] = 0.0
    pz, hz, sz = par.solve(dev(zf), tol=1e-12)
    p1, h1, _ = one.solve(dev(zf), tol=1e-12)
    assert sz["status"] == 0 and hz[1] == [0.0] and not host(pz[1]).any()
    assert torch.equal(pz, p1) and hz == h1
    with pytest.raises(MGError) as ei:
        par.solve(dev(fb), tol=-1.0)
    assert ei.value.code == _lib.MG_EINVAL
    lib = _lib.load()
    assert lib.mg_add_lanes(par._ctx, _ptr_of(par.lane_workspace), par.lane_workspace.numel(), 1) == _lib.MG_EINVAL
    assert "already" in _lib.last_error()
    per = lib.mg_lane_workspace_size(_lib.dims3(64), 0)
    small = torch.empty(per, dtype=torch.uint8, device="cuda")
    assert lib.mg_add_lanes(one._ctx, _ptr_of(small), per, 2) == _lib.MG_EWORKSPACE
    assert lib.mg_add_lanes(one._ctx, _ptr_of(small), per, 0) == _lib.MG_EINVAL
    assert lib.mg_add_lanes(one._ctx, _ptr_of(small), per, _lib.MG_MAX_LANES + 1) == _lib.MG_EINVAL
    # the failed calls left the context without lanes: a batch still solves one by one
    p, h, st = one.solve(dev(fb[:2]), tol=1e-12)
    assert st["status"] == 0


def _ptr_of(t):
    import ctypes
    return ctypes.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ error paths

def test_errors_reported():
    from paper_1410_2240_amd import MG, MGError
    from paper_1410_2240_amd._lib import MG_EBREAKDOWN, MG_EINVAL, MG_ENOCONV
    inp, H = workload("c1", 16)
    mg = mg_from_inputs(inp)
    p, hist, st = mg.solve(dev(inp.f), tol=1e-12, max_cycles=1, raise_on_fail=False)
    assert st["status"] == MG_ENOCONV and len(hist) == 2
    bad = inp.f.copy()
    bad[3, 3, 3] = np.nan
    _, _, st = mg.solve(dev(bad), raise_on_fail=False)
    assert st["status"] == MG_EBREAKDOWN
    with pytest.raises(MGError) as ei:
        mg.solve(dev(inp.f), tol=-1.0)
    assert ei.value.code == MG_EINVAL
    neg = np.ones((16, 16, 16))
    neg[1, 2, 3] = -1.0
    with pytest.raises(MGError):
        MG(dev(neg), dev(np.ones((16,) * 3)), dev(np.ones((16,) * 3)), dev(np.ones((16,) * 3, np.uint8)))
    with pytest.raises(ValueError):
        MG(dev(np.ones((12,) * 3)), dev(np.ones((12,) * 3)), dev(np.ones((12,) * 3)), dev(np.ones((12,) * 3, np.uint8)))


@pytest.mark.parametrize("mixed,krylov", [(False, False), (True, False), (False, True)])
def test_degenerate_right_hand_sides(mixed, krylov):
    """f = 0 and a constant f (whose projection is 0): the solution is p = 0 whatever the
    guess, with the history [0] and no cycle; 64^3, so both finest-grid paths apply."""
    from paper_1410_2240_amd import MG
    inp, _ = workload("c5", 64)
    mg = MG.from_rho(dev(inp.rho), dev(inp.mask), mixed=mixed, krylov=krylov)
    guess = dev(np.random.default_rng(5).standard_normal(inp.f.shape))
    for f in (np.zeros_like(inp.f), np.full_like(inp.f, 3.5)):
        p, hist, st = mg.solve(dev(f), p=guess.clone(), tol=1e-10)
        assert st["status"] == 0 and st["cycles"] == 0 and hist == [0.0]
        assert not host(p).any()


def test_no_fluid_rejected_at_setup():
    """A grid with no fluid cell (all body), or one whose only fluid cell has no open
    face, has no equation: setup reports MG_EINVAL."""
    from paper_1410_2240_amd import MG, MGError
    from paper_1410_2240_amd._lib import MG_EINVAL
    N = 16
    rho = dev(np.ones((N, N, N)))
    for mask in (np.zeros((N, N, N), np.uint8), np.eye(1, N ** 3, 77, dtype=np.uint8).reshape(N, N, N)):
        with pytest.raises(MGError) as ei:
            MG.from_rho(rho, dev(mask))
        assert ei.value.code == MG_EINVAL


def test_incompatible_rhs_mean_removed():
    inp, H = workload("c2", 32)
    mg = mg_from_inputs(inp)
    shifted = np.where(inp.mask == 1, inp.f + 7.5, 0.0)
    p, hist, st = mg.solve(dev(shifted), tol=1e-12)
    assert st["removed_mean"] == pytest.approx(7.5, rel=1e-9)
    assert relerr(host(p), exact.solve_sparse(H.fine, inp.f)) <= 1e-9


def test_isolated_fluid_cell_dropped():
    """A fluid cell enclosed by body cells has no equation: it is reported and kept at 0."""
    from paper_1410_2240_amd import MG
    N = 16
    rho = np.ones((N, N, N))
    mask = np.ones((N, N, N), np.uint8)
    mask[4:9, 4:9, 4:9] = 0
    mask[6, 6, 6] = 1
    mg = MG.from_rho(dev(rho), dev(mask))
    f = fields.divergence_rhs(mask)
    p, hist, st = mg.solve(dev(f), tol=1e-12)
    assert st["dropped_cells"] == 1 and host(p)[6, 6, 6] == 0.0


# ------------------------------------------------------------------ flexible CG outer iteration

@pytest.mark.parametrize("mixed", [False, True])
def test_fcg_matches_exact_solutions(mixed):
    from paper_1410_2240_amd import MG
    for name, N, exact_solve in (("c1", 32, exact.solve_fft_z), ("c2", 32, exact.solve_sparse)):
        inp, H = workload(name, N)
        mg = MG.from_rho(dev(inp.rho), dev(inp.mask), mixed=mixed, krylov=True)
        p, hist, st = mg.solve(dev(inp.f), tol=1e-12, max_cycles=60)
        assert hist[-1] <= 1e-12 and st["status"] == 0
        assert relerr(host(p), exact_solve(H.fine, inp.f)) <= 1e-9, (name, mixed)


def test_fcg_history_follows_oracle():
    from paper_1410_2240_amd import MG
    inp, H = workload("c5", 32)
    mg = MG.from_rho(dev(inp.rho), dev(inp.mask), krylov=True)
    p, hist, st = mg.solve(dev(inp.f), tol=1e-12, max_cycles=60)
    _, ohist = omg.solve_fcg(H, inp.f, tol=1e-12, max_iters=60)
    # rounding differences grow slowly along a CG recurrence
    for a, b in list(zip(hist, ohist))[:8]:
        assert abs(a - b) <= 1e-6 * b + 1e-15


@pytest.mark.parametrize("mixed", [False, True])
def test_fcg_beats_vcycles_on_crest_64(mixed):
    from paper_1410_2240_amd import MG
    inp, H = workload("c5", 64)
    want, _ = omg.solve(H, inp.f, tol=1e-12, max_cycles=200)
    mg = MG.from_rho(dev(inp.rho), dev(inp.mask), mixed=mixed, krylov=True)
    p, hist, st = mg.solve(dev(inp.f), tol=1e-12, max_cycles=100)
    assert relerr(host(p), want) <= 1e-9
    _, mg_hist, _ = mg_from_inputs(inp, mixed).solve(dev(inp.f), tol=1e-12, max_cycles=200)
    assert len(hist) < len(mg_hist) / 2


def test_crest_256_fcg_residual_by_oracle():
    """The steep-crest field where V-cycles alone converge slowly: flexible CG to 1e-10,
    FP64 and mixed, residual recomputed by the oracle."""
    from paper_1410_2240_amd import MG
    inp, H = workload("c5", 256)
    for mixed in (False, True):
        mg = MG.from_rho(dev(inp.rho), dev(inp.mask), mixed=mixed, krylov=True)
        p, hist, st = mg.solve(dev(inp.f), tol=1e-10, max_cycles=100)
        rr = oracle_relres(inp, H, host(p))
        assert rr <= 1.05e-10, (mixed, rr, len(hist))


# ------------------------------------------------------------------ coarsening ablation

def test_setup_from_rho_equals_setup_from_face_arrays():
    from paper_1410_2240_amd import MG, coeffs_from_rho
    inp, H = workload("c2", 32)
    a = MG.from_rho(dev(inp.rho), dev(inp.mask))
    b = MG(*coeffs_from_rho(dev(inp.rho), dev(inp.mask)), dev(inp.mask))
    for l in range(a.levels):
        for x, y in zip(a.level_coeffs(l), b.level_coeffs(l)):
            assert torch.equal(x, y)


def test_density_coarsening_hierarchy_matches_oracle():
    from paper_1410_2240_amd import MG
    from tests.gpu_helpers import maxrel
    inp, _ = workload("c2", 32)
    Hd = omg.setup_density_coarsening(inp.rho, inp.mask, inp.h)
    mg = MG.from_rho(dev(inp.rho), dev(inp.mask), coarsening="density")
    for l, lev in enumerate(Hd.levels):
        bx, by, bz, m = (host(t) for t in mg.level_coeffs(l))
        assert np.array_equal(m.astype(bool), lev.mask), l
        for g, want in ((bx, lev.bx), (by, lev.by), (bz, lev.bz)):
            assert maxrel(g, want) <= 1e-15, l


@pytest.mark.parametrize("name", ["c2", "c5"])
def test_face_product_coarsening_beats_density_coarsening(name):
    """Section 3.1: moving (1/rho) x area to the coarse grids as one unit converges
    better than moving density cell centre to cell centre, which smears the interface.
    Plain V-cycles with density coarsening diverge at density ratio 1000; as a
    flexible-CG preconditioner they need far more steps.  Both reach the same answer."""
    from paper_1410_2240_amd import MG
    from paper_1410_2240_amd._lib import MG_EBREAKDOWN, MG_ENOCONV
    inp, H = workload(name, 64)
    face = MG.from_rho(dev(inp.rho), dev(inp.mask), krylov=True)
    dens = MG.from_rho(dev(inp.rho), dev(inp.mask), krylov=True, coarsening="density")
    pf, hf, _ = face.solve(dev(inp.f), tol=1e-10, max_cycles=200)
    pd, hd, _ = dens.solve(dev(inp.f), tol=1e-10, max_cycles=200)
    assert len(hd) > 1.5 * len(hf), (len(hf), len(hd))
    assert relerr(host(pd), host(pf)) <= 1e-8
    plain = MG.from_rho(dev(inp.rho), dev(inp.mask), coarsening="density")
    _, hp, st = plain.solve(dev(inp.f), tol=1e-10, max_cycles=40, raise_on_fail=False)
    assert st["status"] in (MG_EBREAKDOWN, MG_ENOCONV) and hp[-1] > 1e-6


# ------------------------------------------------------------------ Runge-Kutta stage around the solve

def test_divergence_and_projection_match_oracle():
    from oracle import projection
    from paper_1410_2240_amd import MG
    from tests.gpu_helpers import maxrel
    inp, H = workload("c2", 32)
    g = np.random.default_rng(140)
    U = tuple(g.standard_normal((32, 32, 32)) for _ in range(3))
    R = tuple(g.standard_normal((32, 32, 32)) for _ in range(3))
    p = np.where(H.fine.mask, g.standard_normal((32, 32, 32)), 0.0)
    mg = MG.from_rho(dev(inp.rho), dev(inp.mask))
    dt = 0.02
    for r in (None, R):
        f = host(mg.divergence(tuple(dev(a) for a in U), None if r is None else tuple(dev(a) for a in r), dt))
        assert maxrel(f, projection.divergence(U, H.fine, dt, r)) <= 1e-13
        ud = tuple(dev(a) for a in U)
        mg.project(ud, dev(p), None if r is None else tuple(dev(a) for a in r), dt)
        for got, want in zip(ud, projection.project(U, p, H.fine, dt, r)):
            assert maxrel(host(got), want) <= 1e-13


def test_runge_kutta_stage_leaves_no_divergence_256():
    """f = div(U + dt R)/dt, flexible-CG solve to 1e-12, projection: the new face
    velocity is discretely divergence-free at the bench size (oracle-free property)."""
    from paper_1410_2240_amd import MG
    inp, _ = workload("c2", 256)
    mg = MG.from_rho(dev(inp.rho), dev(inp.mask), krylov=True)
    g = torch.Generator(device="cuda").manual_seed(7)
    U = tuple(torch.randn((256, 256, 256), dtype=torch.float64, device="cuda", generator=g) for _ in range(3))
    R = tuple(torch.randn((256, 256, 256), dtype=torch.float64, device="cuda", generator=g) for _ in range(3))
    dt = 1e-3
    f = mg.divergence(U, R, dt)
    p, hist, st = mg.solve(f, tol=1e-12, max_cycles=60)
    mg.project(U, p, R, dt)
    d = mg.divergence(U, None, 1.0)
    assert float(d.abs().max()) <= 1e-9 * float(f.abs().max()) * dt * 10


@pytest.mark.parametrize("N,mixed", [(16, False), (64, False), (64, True)])
def test_fcg_on_a_workspace_of_nan_patterns(N, mixed):
    """The first flexible-CG direction is z itself: no buffer is read before the solve
    writes it.  A workspace filled with 0xFF bytes (NaN bit patterns in every double)
    before mg_setup_from_rho gives the same bits as one filled with zeros.  Called
    through the C ABI with workspaces the test fills (16^3 runs the grid-stride
    passes, 64^3 the z-marching ones)."""
    import ctypes
    from paper_1410_2240_amd import _lib
    lib = _lib.load()
    inp, _ = workload("c2", N)
    rho, mask, f = dev(inp.rho), dev(inp.mask), dev(inp.f)
    flags = _lib.MG_KRYLOV | (_lib.MG_MIXED if mixed else 0)
    size = lib.mg_workspace_size(_lib.dims3(N), flags)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    out = []
    for fill in (0, 0xFF):
        ws = torch.full((size,), fill, dtype=torch.uint8, device="cuda")
        ctx = ctypes.c_void_p()
        assert lib.mg_setup_from_rho(ctypes.byref(ctx), ctypes.c_void_p(ws.data_ptr()), size,
                                     ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(mask.data_ptr()),
                                     _lib.dims3(N), 1.0 / N, flags, stream) == 0
        p = torch.zeros_like(f)
        hist = np.zeros(101)
        nh = (ctypes.c_int * 1)()
        rc = lib.mg_solve(ctx, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(p.data_ptr()), 1, 1e-10, 100,
                          hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nh, None)
        lib.mg_destroy(ctx)
        assert rc == 0, (fill, rc, _lib.last_error())
        out.append((host(p), hist[:nh[0]].copy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("krylov", [False, True])
def test_from_rho_workspace_gives_the_same_bits(krylov):
    """MG_FROM_RHO leaves the FP32 face arrays of the finest grid out of a mixed
    workspace (the FP32 cycles form those faces from the density), and gives flexible CG
    a third direction, with which it updates p every second step.  A mixed solve on a
    workspace sized and set up with the flag, filled with NaN bit patterns, equals bit
    for bit the solve on a workspace sized without it (128^3: one-pass sweeps and the
    z-marching passes on the FP32 density copy; both outer iterations)."""
    import ctypes
    from paper_1410_2240_amd import _lib
    lib = _lib.load()
    N = 128
    inp, _ = workload("c2", N)
    rho, mask, f = dev(inp.rho), dev(inp.mask), dev(inp.f)
    base = _lib.MG_MIXED | (_lib.MG_KRYLOV if krylov else 0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    sizes = [lib.mg_workspace_size(_lib.dims3(N), fl) for fl in (base, base | _lib.MG_FROM_RHO)]
    assert sizes[0] - sizes[1] >= 3 * N ** 3 * 4 - (N ** 3 * 8 if krylov else 0)
    out = []
    for flags, size in zip((base, base | _lib.MG_FROM_RHO), sizes):
        ws = torch.full((size,), 0xFF, dtype=torch.uint8, device="cuda")
        ctx = ctypes.c_void_p()
        assert lib.mg_setup_from_rho(ctypes.byref(ctx), ctypes.c_void_p(ws.data_ptr()), size,
                                     ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(mask.data_ptr()),
                                     _lib.dims3(N), 1.0 / N, flags, stream) == 0, _lib.last_error()
        p = torch.zeros_like(f)
        hist = np.zeros(101)
        nh = (ctypes.c_int * 1)()
        rc = lib.mg_solve(ctx, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(p.data_ptr()), 1, 1e-10, 100,
                          hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nh, None)
        lib.mg_destroy(ctx)
        assert rc == 0, (flags, rc, _lib.last_error())
        out.append((host(p), hist[:nh[0]].copy()))
        del ws
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_fp64_fcg_from_rho_workspace_gives_the_same_bits():
    """FP64 flexible CG at 256^3 on a workspace laid out with MG_FROM_RHO (a second
    residual and a third direction: the residual update inside the preconditioner's
    first pass, p updated every second step) against one without (their own passes,
    p every step), NaN bit patterns in both: the same solution bit for bit, on solves
    that end after an odd and after an even number of steps.  The residual norms of the
    history are summed in another order (per workgroup of the two-sweep pass), so they
    agree to rounding and give the same number of steps."""
    import ctypes
    from paper_1410_2240_amd import _lib
    lib = _lib.load()
    N = 256
    inp, _ = workload("c2", N)
    rho, mask, f = dev(inp.rho), dev(inp.mask), dev(inp.f)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    steps = set()
    for tol in (1e-10, 1e-6):
        out = []
        for flags in (_lib.MG_KRYLOV, _lib.MG_KRYLOV | _lib.MG_FROM_RHO):
            size = lib.mg_workspace_size(_lib.dims3(N), flags)
            ws = torch.full((size,), 0xFF, dtype=torch.uint8, device="cuda")
            ctx = ctypes.c_void_p()
            assert lib.mg_setup_from_rho(ctypes.byref(ctx), ctypes.c_void_p(ws.data_ptr()), size,
                                         ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(mask.data_ptr()),
                                         _lib.dims3(N), 1.0 / N, flags, stream) == 0, _lib.last_error()
            p = torch.zeros_like(f)
            hist = np.zeros(101)
            nh = (ctypes.c_int * 1)()
            rc = lib.mg_solve(ctx, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(p.data_ptr()), 1, tol, 100,
                              hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nh, None)
            lib.mg_destroy(ctx)
            assert rc == 0, (flags, rc, _lib.last_error())
            out.append((host(p), hist[:nh[0]].copy()))
            del ws
        steps.add(len(out[0][1]) - 1)
        print(f"256^3 FP64 FCG to {tol:g}: {len(out[0][1]) - 1} steps", flush=True)
        assert np.array_equal(out[0][0], out[1][0])
        assert len(out[0][1]) == len(out[1][1])
        assert np.allclose(out[0][1], out[1][1], rtol=1e-12, atol=0)
    assert {s % 2 for s in steps} == {0, 1}, steps
