"""Benchmark of the multigrid pressure-projection solve on one MI355X.

One step = one pressure projection as the flow solver runs it at every Runge-Kutta
stage: face products from the new density (on the device), hierarchy setup, and an
FP64 solve from p = 0 to a relative residual of 1e-10.  The default workload is the
largest one that fits one GPU, the 1024^3 Stokes-crest field with the immersed
ellipsoid (density ratio 1000; 1.07e9 cells), inputs resident in HBM before timing
starts.  Its outer iteration is flexible CG with one V(2,2) cycle per step: plain
V(2,2) cycling stalls near 2e-9 on this field (reported beside it).  The mixed-precision
projection (FP32 cycles), the 512^3 and 256^3 workloads and the other legs of the path
are extra keys of the same line.

Prints one JSON line.  value = grid points x V-cycles / second over the timed steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic scalars moved per finest cell by one V(2,2) cycle.  A grid with the face
# arrays: 4 sweeps x 6 (p, f, bx, by, bz read, p written) + residual-and-restrict 5.125
# + prolongation 2.125 = 31.25, and each coarser grid 1/8 of the one above.  The finest
# grid of a hierarchy built from rho reads one density instead of three face arrays, in
# FP64 and in the FP32 cycle alike: 4 x 4 + 3.125 + 2.125 = 21.25, plus 31.25 / 7 for
# the coarser grids.
VCYCLE_SCALARS_ONE = 21.25 + 31.25 / 7
# On grids of 256^3 and up the finest grid sweeps two at a time, FP64 and FP32 alike (p,
# f and the density read once, p written once per pair): 2 x 4 + 3.125 + 2.125 = 13.25
VCYCLE_SCALARS_TWO = 13.25 + 31.25 / 7
# the same count with three face arrays on the finest grid too (31.25 x 8 / 7)
VCYCLE_SCALARS_FACE = 31.25 * 8 / 7

METRIC = "grid-pts/s per V-cycle + time-to-1e-10 residual (FP64 vs mixed), % HBM peak"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c5",
                    help="c1..c5 (default c5: 1024^3 Stokes crest + body, the largest single-GPU workload)")
    ap.add_argument("--n", type=int, default=None, help="override the grid size")
    ap.add_argument("--outer", choices=("auto", "vcycle", "fcg"), default="auto",
                    help="outer iteration of the timed projection (auto: flexible CG on c5, V-cycles otherwise)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--max-cycles", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-legs", action="store_true",
                    help="leave out the 512^3 / 256^3 workloads and the 256^3 / 128^3 legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 512 MiB device copy (HBM counter calibration) and exit")
    ap.add_argument("--oracle-timing", action="store_true",
                    help="only time the CPU oracle on this host (multigrid 32^3..256^3, FFT+Thomas 512^3) and exit")
    ap.add_argument("--level-breakdown", action="store_true",
                    help="only time each grid's share of a V(2,2) cycle on the bench field and exit")
    ap.add_argument("--coarsening-sweep", action="store_true",
                    help="only compare the two coarsenings of section 3.1 on the wavy field from 32^3 to 1024^3 "
                         "(cycles and contraction factor of plain V-cycles, flexible-CG steps) and exit")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def solve_timer(rho, mask, f, tol, max_cycles):
    """Returns timed(mixed, krylov, steps, warmup): the mean time of `steps` projections
    (setup from rho + solve from p = 0), with the last context, solution and history."""
    import torch
    from paper_1410_2240_amd import MG

    def projection(mixed, krylov):
        mg = MG.from_rho(rho, mask, mixed=mixed, krylov=krylov)
        p, hist, st = mg.solve(f, tol=tol, max_cycles=max_cycles, raise_on_fail=False)
        return mg, p, hist, st

    def timed(mixed, krylov, steps, warmup):
        for _ in range(warmup):
            projection(mixed, krylov)
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        cycles = 0
        mg = p = None
        for _ in range(steps):
            del mg, p   # one hierarchy at a time: the previous step's is freed first
            mg, p, hist, st = projection(mixed, krylov)
            cycles += st["cycles"]
        stop.record()
        torch.cuda.synchronize()
        return {"ms": start.elapsed_time(stop) / steps, "cycles": cycles / steps, "status": st["status"],
                "final_relres": hist[-1], "mg": mg, "p": p, "hist": hist}

    return timed


def public(r):
    return {k: v for k, v in r.items() if k not in ("mg", "p", "hist")}


def vcycle_ms(mg, f, mask, dtype):
    """Pure V-cycle time: 10 cycles with no residual checks, on a compatible f."""
    import torch
    fx = f if dtype == torch.float64 else ((f - f[mask.bool()].mean()) * mask).to(dtype)
    p = torch.zeros_like(fx)
    mg.vcycle(p, fx)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(10):
        mg.vcycle(p, fx)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / 10


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.oracle_timing:
        print(json.dumps(oracle_timing()))
        return
    if args.coarsening_sweep:
        print(json.dumps(coarsening_sweep(args)))
        return
    if args.level_breakdown:
        print(json.dumps(level_breakdown(args)))
        return
    import numpy as np
    import torch

    if args.copy_calibration:
        # reads 512 MiB and writes 512 MiB: the scale of the FETCH_SIZE / WRITE_SIZE counters
        a = torch.ones(64 << 20, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": a.numel() * 8}))
        return

    import fields

    t_gen = time.time()
    inp = fields.make(args.config, args.n)
    N, n = inp.N, inp.n
    dev = torch.device("cuda:0")
    rho = torch.from_numpy(inp.rho).to(dev)
    mask = torch.from_numpy(inp.mask).to(dev)
    f = torch.from_numpy(inp.f).to(dev)
    t_gen = time.time() - t_gen
    log(f"inputs {inp.name} {N}^3 generated and copied in {t_gen:.1f} s")
    krylov = args.outer == "fcg" or (args.outer == "auto" and args.config == "c5")
    outer = "flexible CG (FCG(1)), one V(2,2) RBGS cycle per step" if krylov else "V(2,2) RBGS cycles"
    timed = solve_timer(rho, mask, f, args.tol, args.max_cycles)

    # ---- the timed step: FP64 projection, exactly --steps of them after --warmup
    torch.cuda.reset_peak_memory_stats()
    r64 = timed(False, krylov, args.steps, args.warmup)
    peak64 = torch.cuda.max_memory_allocated()
    log(f"fp64 projection ({outer}) {r64['ms']:.2f} ms, {r64['cycles']:.0f} cycles, status {r64['status']}, "
        f"relres {r64['final_relres']:.3e}")
    mg64 = r64["mg"]
    vc64 = vcycle_ms(mg64, f, mask, torch.float64)

    # dominant kernel: the finest-grid smoother, timed on the stream it runs on.  On grids
    # of 256^3 and up it sweeps two at a time: four sweeps are two launches p -> t -> p, as
    # in a cycle; below, two sweeps are two one-pass launches.
    two64 = N >= 256
    fz = torch.zeros_like(f)
    ps = torch.zeros_like(f)
    sweeps = 4 if two64 else 2
    mg64.smooth(0, ps, fz, sweeps, 0)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5 if N >= 1024 else 10
    a.record()
    for _ in range(reps):
        mg64.smooth(0, ps, fz, sweeps, 0)
    b.record()
    torch.cuda.synchronize()
    launch_ms = a.elapsed_time(b) / (2 * reps)
    # algorithmic bytes of one launch on the finest grid of a hierarchy built from rho: p,
    # f and the density form of the coefficients read, p written (for two sweeps or one)
    sweep_bytes = n * 8 * 4
    achieved = sweep_bytes / (launch_ms * 1e-3) / 1e9
    del fz, ps
    r64.pop("mg"), r64.pop("p")
    del mg64
    torch.cuda.empty_cache()

    # ---- the mixed-precision projection (FP32 cycles inside FP64 refinement / FCG)
    torch.cuda.reset_peak_memory_stats()
    rmx = timed(True, krylov, max(1, args.steps // 4), 1)
    peakmx = torch.cuda.max_memory_allocated()
    log(f"mixed projection ({outer}) {rmx['ms']:.2f} ms, {rmx['cycles']:.0f} steps, status {rmx['status']}, "
        f"relres {rmx['final_relres']:.3e}")
    vc32 = vcycle_ms(rmx["mg"], f, mask, torch.float32)
    # the FP32 cycles' finest-grid smoother: two red-black sweeps per pass (grids of 256^3
    # and up); four sweeps = two passes p -> t -> p, as in a cycle
    two_sweep = None
    if N >= 256:
        f32 = ((f - f[mask.bool()].mean()) * mask).float()
        p32 = torch.zeros_like(f32)
        mgx = rmx["mg"]
        mgx.smooth(0, p32, f32, 4, 0)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            mgx.smooth(0, p32, f32, 4, 0)
        b.record()
        torch.cuda.synchronize()
        pass_ms = a.elapsed_time(b) / (2 * reps)
        two_sweep = {"kernel": "rbgs_fused2 (finest grid of the FP32 cycles, density form, two red-black sweeps "
                               "per launch)", "launch_ms": pass_ms, "bytes_per_launch": n * 4 * 4,
                     "achieved_GBs": n * 4 * 4 / (pass_ms * 1e-3) / 1e9,
                     "frac": n * 4 * 4 / (pass_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "note": "ALU-bound (face coefficients formed from the density at every update); "
                             "two one-pass FP32 sweeps move twice the bytes"}
        del f32, p32, mgx
    rmx.pop("mg"), rmx.pop("p")
    torch.cuda.empty_cache()

    # ---- the other outer iteration on the same field, once each (plain V(2,2) cycling is
    # the paper's method; on the crest field it stalls and ends in MG_ENOCONV)
    other = {}
    for mixed in (False, True):
        cap = 100 if krylov else args.max_cycles
        ro = solve_timer(rho, mask, f, args.tol, cap)(mixed, not krylov, 1, 0)
        ro.pop("mg"), ro.pop("p"), ro.pop("hist")
        ro["max_cycles"] = cap
        ro["note"] = "one run, its first allocation of the workspace included"
        other["mixed" if mixed else "fp64"] = ro
        log(f"{'V-cycles' if krylov else 'flexible CG'} {'mixed' if mixed else 'fp64'}: {ro}")
        torch.cuda.empty_cache()
    r64.pop("hist"), rmx.pop("hist")
    del rho, mask, f
    torch.cuda.empty_cache()

    legs = {}
    if not args.no_legs and args.config == "c5":
        legs["c3_flat_smear1_512"] = config_leg("c3", 512, args)
        legs["c2_wavy_body_256"] = config_leg("c2", 256, args)
    if not args.no_legs:
        legs["coarsening_ablation"] = coarsening_leg(256, args)
        legs["cut_cells"] = cut_cell_leg(256, args)
        legs["differentiation"] = differentiation_leg(args)
        legs["rk2_projection"] = rk2_leg(256, args)
    traffic = recorded_traffic(inp.name, N)
    scalars = VCYCLE_SCALARS_TWO if N >= 256 else VCYCLE_SCALARS_ONE
    out = {
        "metric": METRIC,
        "value_definition": f"grid points x V-cycles / time of the FP64 projection (setup from rho + solve to "
                            f"{args.tol:g} from p = 0, outer iteration: {outer}); time_to_tol_ms gives FP64 and "
                            f"mixed, roofline and vcycle_roofline_frac the fraction of HBM peak",
        "value": n * r64["cycles"] / (r64["ms"] * 1e-3),
        "unit": "grid-pts/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r64["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": inp.name, "N": N, "cells": n, "tol": args.tol, "outer": outer,
                   "cycle": "V(2,2) RBGS", "density_ratio": 1000},
        "time_to_tol_ms": {"fp64": r64["ms"], "mixed": rmx["ms"], "mixed_speedup": r64["ms"] / rmx["ms"]},
        "cycles_to_tol": {"fp64": r64["cycles"], "mixed": rmx["cycles"]},
        "final_relres": {"fp64": r64["final_relres"], "mixed": rmx["final_relres"]},
        "status": {"fp64": r64["status"], "mixed": rmx["status"]},
        "mixed_steps_timed": max(1, args.steps // 4),
        ("plain_vcycles" if krylov else "krylov_fcg"): other,
        "peak_memory_bytes": {"fp64": peak64, "mixed": peakmx},
        "vcycle_ms": {"fp64": vc64, "fp32": vc32},
        "vcycle_pts_per_s": {"fp64": n / (vc64 * 1e-3), "fp32": n / (vc32 * 1e-3)},
        # algorithmic scalars per finest cell per V(2,2) cycle of the design that runs
        # (density form on the finest grid), and against the face-array count
        "vcycle_roofline_frac": {"fp64": scalars * 8 * n / (vc64 * 1e-3) / (HBM_PEAK_GBS * 1e9),
                                 "fp32": scalars * 4 * n / (vc32 * 1e-3) / (HBM_PEAK_GBS * 1e9),
                                 "fp64_face_array_count": VCYCLE_SCALARS_FACE * 8 * n / (vc64 * 1e-3)
                                 / (HBM_PEAK_GBS * 1e9),
                                 "fp32_face_array_count": VCYCLE_SCALARS_FACE * 4 * n / (vc32 * 1e-3)
                                 / (HBM_PEAK_GBS * 1e9)},
        "roofline": {"bound": "hbm",
                     "kernel": ("rbgs_fused2 (finest grid, FP64 density form, two red-black sweeps per launch)"
                                if two64 else "rbgs_fused (finest grid, FP64 density form, one red-black sweep)"),
                     "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "launch_ms": launch_ms, "bytes_per_launch": sweep_bytes},
        "fp32_two_sweep_pass": two_sweep,
        "input_gen_s": t_gen,
        **legs,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(inp)
    print(json.dumps(out), flush=True)


def config_leg(name, N, args):
    """Another workload at its own size: FP64 against mixed, plain V-cycles and flexible
    CG, each the mean of three projections (setup + solve to tol) after one warm-up."""
    import torch
    import fields
    t0 = time.time()
    inp = fields.make(name, N)
    rho = torch.from_numpy(inp.rho).cuda()
    mask = torch.from_numpy(inp.mask).cuda()
    f = torch.from_numpy(inp.f).cuda()
    out = {"workload": inp.name, "N": N, "input_gen_s": time.time() - t0}
    del inp
    timed = solve_timer(rho, mask, f, args.tol, args.max_cycles)
    for krylov in (False, True):
        row = {}
        for mixed in (False, True):
            r = timed(mixed, krylov, 3, 1)
            if not krylov:
                r[("fp32" if mixed else "fp64") + "_vcycle_ms"] = vcycle_ms(r["mg"], f, mask,
                                                                            torch.float32 if mixed else torch.float64)
            row["mixed" if mixed else "fp64"] = public(r)
            del r
            torch.cuda.empty_cache()
        row["mixed_speedup"] = row["fp64"]["ms"] / row["mixed"]["ms"]
        out["flexible_cg" if krylov else "vcycles"] = row
    log(f"{out['workload']}: {out}")
    del rho, mask, f
    torch.cuda.empty_cache()
    return out


def coarsening_leg(N, args):
    """Coarsening ablation (section 3.1) on the wavy interface + body field: face
    products moved as one unit against density restricted cell centre to cell centre,
    both as flexible-CG preconditioners, and the plain V-cycle with each (the paper
    reports density restriction as the slower one)."""
    import torch
    import fields
    from paper_1410_2240_amd import MG
    inp = fields.make("c2", N)
    rho = torch.from_numpy(inp.rho).cuda()
    mask = torch.from_numpy(inp.mask).cuda()
    f = torch.from_numpy(inp.f).cuda()
    abl = {"workload": f"{inp.name}_{N}"}
    for mode in ("face", "density"):
        torch.cuda.synchronize()
        t0 = time.time()
        mgk = MG.from_rho(rho, mask, krylov=True, coarsening=mode)
        p, hist, st = mgk.solve(f, tol=args.tol, max_cycles=args.max_cycles, raise_on_fail=False)
        torch.cuda.synchronize()
        abl[mode] = {"fcg_steps": st["cycles"], "fcg_status": st["status"], "fcg_ms": (time.time() - t0) * 1e3}
        del mgk, p
        mgp = MG.from_rho(rho, mask, coarsening=mode)
        _, hp, stp = mgp.solve(f, tol=args.tol, max_cycles=30, raise_on_fail=False)
        abl[mode].update({"vcycles_30_relres": hp[-1], "vcycles_status": stp["status"]})
        del mgp
        torch.cuda.empty_cache()
    log(f"coarsening ablation {abl}")
    return abl


def cut_cell_leg(N, args):
    """The same wavy field with the ellipsoid as a cut-cell body (section 2.2): time to
    build fractions, merge map and coefficients, and a flexible-CG solve to tol."""
    import torch
    import fields
    from paper_1410_2240_amd import MG
    from paper_1410_2240_amd.cutcell import cut_cells, cut_coeffs, merge_fill, merge_rhs
    rho_np, psi_np = fields.wavy_cut(N)
    rho = torch.from_numpy(rho_np).cuda()
    psi = torch.from_numpy(psi_np).cuda()
    del rho_np, psi_np
    geo = cut_cells(psi, 8)
    torch.cuda.synchronize()
    a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    a.record()
    geo = cut_cells(psi, 8)
    b.record()
    bx, by, bz, mask = cut_coeffs(rho, *geo)
    c.record()
    torch.cuda.synchronize()
    vol, merge_to = geo[3], geo[4]
    g = torch.Generator(device="cuda").manual_seed(1410)
    f = merge_rhs(merge_to, torch.randn(rho.shape, dtype=torch.float64, device="cuda", generator=g))
    torch.cuda.synchronize()
    t0 = time.time()
    mg = MG(bx, by, bz, mask, krylov=True)
    p, hist, st = mg.solve(f, tol=args.tol, max_cycles=args.max_cycles, raise_on_fail=False)
    merge_fill(merge_to, p)
    torch.cuda.synchronize()
    out = {"cut_cells_ms": a.elapsed_time(b), "cut_coeffs_ms": b.elapsed_time(c),
           "cut_cells": int(((vol > 0) & (vol < 1)).sum()), "merged_cells": int((merge_to >= 0).sum()),
           "fcg_steps": st["cycles"], "fcg_status": st["status"], "final_relres": hist[-1],
           "setup_plus_solve_ms": (time.time() - t0) * 1e3, "rhs": "P(N(0,1)) merged"}
    log(f"cut cells {out}")
    return out


def differentiation_leg(args):
    """The differentiated projection: 8 right-hand sides at 128^3 (flat interface),
    poisson_solve forward (setup + 8 solves) and the backward of L = sum w.p (8 adjoint
    solves + the coefficient gradient), one right-hand side at a time and with the
    default concurrent lanes; best of two, and whether the two give the same bits."""
    import torch
    import fields
    from paper_1410_2240_amd.autograd import DEFAULT_CONCURRENCY, poisson_solve
    N, B = 128, 8
    inp = fields.make("c4", N)
    rho = torch.from_numpy(inp.rho).cuda().requires_grad_(True)
    mask = torch.from_numpy(inp.mask).cuda()
    fb = torch.from_numpy(fields.batch_rhs(inp.mask, B)).cuda().requires_grad_(True)
    w = torch.from_numpy(fields.adjoint_weights(N, B)).cuda()
    out = {"workload": "c4_flat_128_batch8", "tol": args.tol, "concurrency": DEFAULT_CONCURRENCY}
    for prec in ("fp64", "mixed"):
        res = {}
        for lanes in (0, None):
            best_f = best_b = float("inf")
            for _ in range(2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                p = poisson_solve(fb, rho, mask, tol=args.tol, precision=prec, lanes=lanes)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                gf, grho = torch.autograd.grad((w * p).sum(), (fb, rho))
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                best_f, best_b = min(best_f, t1 - t0), min(best_b, t2 - t1)
            res["one_at_a_time" if lanes == 0 else "concurrent"] = {
                "forward_ms": best_f * 1e3, "backward_ms": best_b * 1e3, "out": (p.detach(), gf, grho)}
        a, b = res["one_at_a_time"].pop("out"), res["concurrent"].pop("out")
        res["identical"] = all(torch.equal(x, y) for x, y in zip(a, b))
        out[prec] = res
        del a, b
    torch.cuda.empty_cache()
    log(f"differentiation {out}")
    return out


def rk2_leg(N, args):
    """The pressure projection of one two-stage Runge-Kutta step (section 2.1: a
    projection after each stage, eqs. runge1 / runge2) on the bench field.  Each stage
    sets the hierarchy up from rho (the density changes every stage in the flow solver),
    forms f = div(U + dt R)/dt from the face velocities, solves, and projects; the
    second stage starts from the first stage's pressure.  Inputs (seeded): U^n = seeded
    N(0, 1) face velocities made divergence-free by one untimed projection, as after the
    previous step; R1 = N(0, 1) per face; R2 = R1 + 0.01 N(0, 1), the forcing evaluated
    again at the intermediate velocity; dt = 1e-3.  Reports the step time, each stage's
    cycles, the second stage's cycles from p = 0 for comparison, and the largest
    divergence left, relative to the largest source."""
    import torch
    from paper_1410_2240_amd import MG
    import fields
    inp = fields.make("c2", N)
    rho = torch.from_numpy(inp.rho).cuda()
    mask = torch.from_numpy(inp.mask).cuda()
    del inp
    g = torch.Generator(device="cuda").manual_seed(1410)
    shape = (N, N, N)
    def randn():
        return torch.randn(shape, dtype=torch.float64, device="cuda", generator=g)
    U = tuple(randn() for _ in range(3))
    R1 = tuple(randn() for _ in range(3))
    R2 = tuple(r + 0.01 * randn() for r in R1)
    dt = 1e-3
    prep = MG.from_rho(rho, mask)
    p0, _, _ = prep.solve(prep.divergence(U, None, 1.0), tol=1e-12, max_cycles=100)
    prep.project(U, p0, None, 1.0)
    del prep, p0
    out = {"workload": f"c2_wavy_body_{N}", "dt": dt, "tol": args.tol}
    for prec in ("fp64", "mixed"):
        mixed = prec == "mixed"
        best, res = float("inf"), None
        for _ in range(3):
            V = tuple(u.clone() for u in U)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mg1 = MG.from_rho(rho, mask, mixed=mixed)
            f1 = mg1.divergence(V, R1, dt)
            p1, h1, _ = mg1.solve(f1, tol=args.tol, max_cycles=args.max_cycles, raise_on_fail=False)
            mg1.project(V, p1, R1, dt)
            mg2 = MG.from_rho(rho, mask, mixed=mixed)
            f2 = mg2.divergence(V, R2, dt)
            p2, h2, _ = mg2.solve(f2, p=p1.clone(), tol=args.tol, max_cycles=args.max_cycles, raise_on_fail=False)
            mg2.project(V, p2, R2, dt)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            if t < best:
                best = t
                div = mg2.divergence(V, None, 1.0)
                res = {"step_ms": t * 1e3, "stage1_cycles": len(h1) - 1, "stage2_cycles_warm": len(h2) - 1,
                       "max_div_rel": float(div.abs().max()) / (float(f2.abs().max()) * dt)}
            del mg1, mg2
        mgc = MG.from_rho(rho, mask, mixed=mixed)
        _, hc, _ = mgc.solve(f2, tol=args.tol, max_cycles=args.max_cycles, raise_on_fail=False)
        res["stage2_cycles_cold"] = len(hc) - 1
        del mgc
        out[prec] = res
    torch.cuda.empty_cache()
    log(f"rk2 projection {out}")
    return out


def level_breakdown(args):
    """Where a V(2,2) cycle spends its time on the bench field: per grid of 128^3 and up,
    the four sweeps, the residual + restriction and the prolongation, each timed through
    the component entry points with HIP events (best of the mean of 20 calls); the grids
    of 64^3 and below (four block-sweep launches each, the restriction and prolongation
    fused into them, then the single-workgroup tail from 16^3 down) are the whole cycle
    minus those.  FP64 cycle, and the FP32 cycle of a mixed context."""
    import torch
    import fields
    from paper_1410_2240_amd import MG
    N = args.n or 256
    inp = fields.make(args.config, N)
    rho = torch.from_numpy(inp.rho).cuda()
    mask = torch.from_numpy(inp.mask).cuda()
    f0 = torch.from_numpy(inp.f).cuda()
    del inp

    def tm(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(3):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                fn()
            b.record()
            torch.cuda.synchronize()
            best = min(best, a.elapsed_time(b) / reps)
        return best * 1e3   # us

    out = {"workload": f"{args.config}_{N}"}
    g = torch.Generator(device="cuda").manual_seed(1410)
    for prec, mixed, dt in (("fp64", False, torch.float64), ("fp32", True, torch.float32)):
        mg = MG.from_rho(rho, mask, mixed=mixed)
        grids, above = [], 0.0
        for lv in range(mg.levels - 1):
            n_l, _ = mg.level_info(lv)
            if n_l <= 64:
                break
            p = torch.zeros((n_l,) * 3, dtype=dt, device="cuda")
            f = f0.to(dt) if lv == 0 else torch.randn((n_l,) * 3, dtype=torch.float64, device="cuda",
                                                       generator=g).to(dt)
            ec = torch.zeros((n_l // 2,) * 3, dtype=dt, device="cuda")
            sweeps = tm(lambda: mg.smooth(lv, p, f, 4, 0))   # a cycle's four sweeps, p -> t -> ... -> p
            rr = tm(lambda: mg.residual_restrict(lv, p, f))
            pro = tm(lambda: mg.prolong_add(lv, ec, p))
            grids.append({"n": n_l, "sweeps_us": sweeps, "residual_restrict_us": rr, "prolong_us": pro,
                          "total_us": sweeps + rr + pro})
            above += sweeps + rr + pro
            del p, f, ec
        pf = torch.zeros_like(f0, dtype=dt)
        ff = f0.to(dt)
        cycle = tm(lambda: mg.vcycle(pf, ff))
        out[prec] = {"cycle_us": cycle, "grids": grids, "grids_64_and_below_us": cycle - above}
        log(f"level breakdown {prec}: {out[prec]}")
        del mg, pf, ff
        torch.cuda.empty_cache()
    return out


def coarsening_sweep(args):
    """Section 3.1's claim across grid sizes: the face products coarsened as one unit
    against the density restricted cell centre to cell centre (areas apart), on the
    wavy interface + body field from 32^3 to 1024^3.  Per N and coarsening: plain
    V-cycles (at most 100) with their status, cycles and asymptotic contraction factor
    (geometric mean of the last five residual ratios), and flexible-CG steps to tol."""
    import numpy as np
    import torch
    import fields
    from paper_1410_2240_amd import MG
    out = {"workload": "c2_wavy_body", "tol": args.tol, "max_vcycles": 100, "sizes": {}}
    for N in (32, 64, 128, 256, 512, 1024):
        t0 = time.time()
        inp = fields.make("c2", N)
        rho = torch.from_numpy(inp.rho).cuda()
        mask = torch.from_numpy(inp.mask).cuda()
        f = torch.from_numpy(inp.f).cuda()
        del inp
        log(f"coarsening sweep {N}^3: inputs in {time.time() - t0:.1f} s")
        row = {}
        for mode in ("face", "density"):
            mg = MG.from_rho(rho, mask, coarsening=mode)
            _, h, st = mg.solve(f, tol=args.tol, max_cycles=100, raise_on_fail=False)
            del mg
            tail = [b / a for a, b in zip(h[:-1], h[1:]) if a > 0][-5:]
            rate = float(np.prod(tail) ** (1.0 / len(tail))) if tail else None
            torch.cuda.synchronize()
            t1 = time.time()
            mgk = MG.from_rho(rho, mask, krylov=True, coarsening=mode)
            _, hk, stk = mgk.solve(f, tol=args.tol, max_cycles=200, raise_on_fail=False)
            torch.cuda.synchronize()
            del mgk
            torch.cuda.empty_cache()
            row[mode] = {"vcycle_status": st["status"], "vcycles": st["cycles"], "vcycle_final_relres": h[-1],
                         "vcycle_rate": rate, "fcg_status": stk["status"], "fcg_steps": stk["cycles"],
                         "fcg_final_relres": hk[-1], "fcg_ms": (time.time() - t1) * 1e3}
            log(f"  {mode}: {row[mode]}")
        out["sizes"][str(N)] = row
        del rho, mask, f
        torch.cuda.empty_cache()
    return out


TRAFFIC_KERNEL = "k_rbgs_fused2<double, false, false>"


def kernel_source_hash():
    """SHA-256 over the sources the dominant kernel is compiled from and the hipcc flags:
    recorded counter traffic is valid only for the build it was taken on."""
    import hashlib
    from paper_1410_2240_amd import build as _build
    hsh = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        hsh.update(rel.encode())
        hsh.update(open(os.path.join(ROOT, rel), "rb").read())
    hsh.update(" ".join(_build.HIPCC_FLAGS).encode())
    return hsh.hexdigest()


TRAFFIC_SOURCES = ("paper_1410_2240_amd/csrc/mg_fused2.hip", "paper_1410_2240_amd/csrc/mg_buffer.h",
                   "paper_1410_2240_amd/csrc/mg_kernels.h")


def recorded_traffic(workload, N):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter
    runs (scaled FETCH_SIZE + WRITE_SIZE), or None when they were taken on another
    workload or size, or the kernel's sources or build flags have changed since."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[TRAFFIC_KERNEL]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("build_sha256") != kernel_source_hash() or rec["workload"] != workload or rec["N"] != N:
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_baseline(inp):
    """The oracle on this host's cores, on a bounded sample of the same workload.

    value: the oracle's FP64 V(2,2) cycle in grid points per second, on the same field
    recipe at the largest size whose cycle takes seconds (256^3 for the 1024^3 field: one
    oracle cycle at 1024^3 would take minutes).  Beside it, at the full size, the oracle's
    FP64 residual r = P f - A p (the part of a cycle it can run there) over a 64-plane
    slab, in grid points per second."""
    import numpy as np

    import fields
    from oracle import multigrid as omg
    from oracle.operator import Level, apply, diagonal, face_coeffs_from_rho, project
    name = next(k for k in fields.WORKLOADS if inp.name.startswith(k + "_"))
    Ns = min(inp.N, 256)
    small = inp if Ns == inp.N else fields.make(name, Ns)
    t0 = time.time()
    H = omg.setup(*face_coeffs_from_rho(small.rho, small.mask), small.mask, small.h)
    t_setup = time.time() - t0
    fh = project(small.f, H.fine.mask)
    p = np.zeros_like(fh)
    cycles = 0
    t0 = time.time()
    while cycles < 2 and time.time() - t0 < 30:
        p = omg.vcycle(H, p, fh)
        cycles += 1
    dt = (time.time() - t0) / cycles
    del H, fh, p
    out = {"value": small.n / dt, "unit": "grid-pts/s", "cores": 1, "kind": "oracle",
           "sample": f"{cycles} FP64 V(2,2) cycles of the numpy oracle on the {name} recipe at {Ns}^3 "
                     f"(setup {t_setup:.1f} s excluded); numpy elementwise kernels are single-threaded",
           "host_cpus": os.cpu_count()}
    if inp.N > Ns:
        # the residual of a random p over planes 448..511 of the full grid (faces formed
        # from the planes either side, as on the whole grid)
        k0, k1 = inp.N // 2 - 64, inp.N // 2
        t0 = time.time()
        m = inp.mask[k0 - 1:k1 + 1].astype(bool)
        lev = Level(*face_coeffs_from_rho(inp.rho[k0 - 1:k1 + 1], m), m, inp.h)
        lev.mask = m & (diagonal(lev) > 0)
        pr = np.random.default_rng(3).standard_normal(m.shape)
        r = np.where(lev.mask, inp.f[k0 - 1:k1 + 1] - apply(pr, lev), 0.0)[1:-1]
        t_res = time.time() - t0
        out["full_size_residual"] = {"pts_per_s": (k1 - k0) * inp.N * inp.N / t_res, "planes": k1 - k0,
                                     "N": inp.N, "seconds": t_res, "norm2": float(np.sum(r * r))}
    return out


def oracle_timing():
    """The CPU oracle on this host, the baseline beside the GPU numbers: FP64 multigrid
    per V(2,2) cycle and to a relative residual of 1e-10 from p = 0 on the bench field
    (wavy interface + body) at 32^3 .. 256^3, and the FFT + Thomas direct solve of the
    512^3 flat field (a different algorithm: exact, not iterative).  numpy's elementwise
    kernels and numpy.fft run on one thread."""
    import numpy as np

    import fields
    from oracle import exact
    from oracle import multigrid as omg
    from oracle.operator import Level, face_coeffs_from_rho, project
    rows = []
    for N in (32, 64, 128, 256):
        inp = fields.make("c2", N)
        t0 = time.time()
        H = omg.setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
        t_setup = time.time() - t0
        fh = project(inp.f, H.fine.mask)
        p = np.zeros_like(fh)
        reps = 2 if N >= 256 else 3
        t0 = time.time()
        for _ in range(reps):
            p = omg.vcycle(H, p, fh)
        t_cycle = (time.time() - t0) / reps
        t0 = time.time()
        _, hist = omg.solve(H, inp.f, tol=1e-10, max_cycles=100)
        t_solve = time.time() - t0
        rows.append({"N": N, "setup_s": t_setup, "vcycle_s": t_cycle, "grid_pts_per_s": inp.n / t_cycle,
                     "cycles_to_1e-10": len(hist) - 1, "solve_s": t_solve})
        log(f"oracle {N}^3: V-cycle {t_cycle:.3f} s, {len(hist) - 1} cycles to 1e-10 in {t_solve:.1f} s")
    inp = fields.make("c3", 512)
    lev = Level(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask.astype(bool), inp.h)
    t0 = time.time()
    exact.solve_fft_z(lev, inp.f)
    t_fft = time.time() - t0
    log(f"oracle 512^3 FFT + Thomas: {t_fft:.1f} s")
    return {"oracle_timing": {"host_cpus": os.cpu_count(), "threads_used": 1, "multigrid_c2": rows,
                              "fft_thomas_c3_512": {"solve_s": t_fft, "algorithm": "direct (FFT in x, y; Thomas in z)"}}}


if __name__ == "__main__":
    main()
