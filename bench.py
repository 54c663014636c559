"""Benchmark of the multigrid pressure-projection solve on one MI355X.

One step = one pressure projection as the flow solver runs it at every Runge-Kutta
stage: face products from the new density (on the device), hierarchy setup, and an
FP64 multigrid solve from p = 0 to a relative residual of 1e-10.  The workload is
the 256^3 wavy-interface field with the immersed ellipsoid body (density ratio 1000),
inputs resident in HBM before timing starts.

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
VCYCLE_SCALARS_F64 = 21.25 + 31.25 / 7
VCYCLE_SCALARS_F32 = VCYCLE_SCALARS_F64


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2", help="c1..c5 (default c2: 256^3 wavy interface + body)")
    ap.add_argument("--n", type=int, default=None, help="override the grid size")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--max-cycles", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    from paper_1410_2240_amd import MG

    t_gen = time.time()
    inp = fields.make(args.config, args.n)
    N, n = inp.N, inp.n
    dev = torch.device("cuda:0")
    rho = torch.from_numpy(inp.rho).to(dev)
    mask = torch.from_numpy(inp.mask).to(dev)
    f = torch.from_numpy(inp.f).to(dev)
    t_gen = time.time() - t_gen
    log(f"inputs {inp.name} {N}^3 generated in {t_gen:.1f} s")

    def projection(mixed, krylov=False):
        # face products from rho formed in the workspace, hierarchy, solve
        mg = MG.from_rho(rho, mask, mixed=mixed, krylov=krylov)
        p, hist, st = mg.solve(f, tol=args.tol, max_cycles=args.max_cycles, raise_on_fail=False)
        return mg, p, hist, st

    def timed(mixed, steps, warmup, krylov=False):
        for _ in range(warmup):
            projection(mixed, krylov)
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        cycles = 0
        for _ in range(steps):
            mg, p, hist, st = projection(mixed, krylov)
            cycles += st["cycles"]
        stop.record()
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / steps, cycles / steps, mg, p, hist, st["status"]

    # pure V-cycle time (10 cycles, no residual checks) in FP64 and FP32
    def vcycle_ms(mg, dtype):
        fx = f if dtype == torch.float64 else (f - f[mask.bool()].mean()).float() * mask
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

    ms64, cyc64, mg64, p64, hist64, st64 = timed(False, args.steps, args.warmup)
    log(f"fp64 projection {ms64:.2f} ms, {cyc64:.0f} cycles, status {st64}")
    vc64 = vcycle_ms(mg64, torch.float64)

    # dominant kernel: the finest-grid smoother, timed on the stream it runs on
    fz = torch.zeros_like(f)
    ps = torch.zeros_like(f)
    mg64.smooth(0, ps, fz, 2, 0)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    a.record()
    for _ in range(reps):
        mg64.smooth(0, ps, fz, 2, 0)   # two one-pass sweeps, exactly as inside the V-cycle
    b.record()
    torch.cuda.synchronize()
    launch_ms = a.elapsed_time(b) / (2 * reps)
    # algorithmic bytes of one red-black sweep on the finest grid of a hierarchy built
    # from rho: p, f and the density form of the coefficients read, p written
    half_bytes = n * 8 * 4
    achieved = half_bytes / (launch_ms * 1e-3) / 1e9
    del mg64, p64, fz, ps
    torch.cuda.empty_cache()

    msmx, cycmx, mgmx, pmx, histmx, stmx = timed(True, max(1, args.steps), 1)
    log(f"mixed projection {msmx:.2f} ms, {cycmx:.0f} steps, status {stmx}")
    vc32 = vcycle_ms(mgmx, torch.float32)
    del mgmx, pmx
    torch.cuda.empty_cache()

    # flexible CG outer iteration (one V-cycle per step), FP64 and FP32 preconditioner
    kr = {}
    for mixed in (False, True):
        ms, cyc, mgk, pk, hist, st = timed(mixed, max(1, args.steps), 1, krylov=True)
        kr["mixed" if mixed else "fp64"] = {"ms": ms, "steps": cyc, "final_relres": hist[-1], "status": st}
        log(f"fcg {'mixed' if mixed else 'fp64'} {ms:.2f} ms, {cyc:.0f} steps, status {st}")
        del mgk, pk
        torch.cuda.empty_cache()

    # coarsening ablation (section 3.1): face products moved as one unit against density
    # restricted cell centre to cell centre, both as flexible-CG preconditioners, and the
    # plain V-cycle with density coarsening (which the paper reports as slower)
    abl = {}
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
    cut = cut_cell_leg(N, args) if args.config == "c2" else None
    diff = differentiation_leg(args) if args.config == "c2" else None
    rk2 = rk2_leg(N, args) if args.config == "c2" else None
    traffic = recorded_traffic(inp.name, N)
    out = {
        "metric": "grid-pts/s per V-cycle + time-to-1e-10 residual (FP64 vs mixed), % HBM peak",
        "value_definition": "grid points x V-cycles / time of the FP64 projection (setup from rho + solve to "
                            "1e-10 from p = 0); time_to_tol_ms gives FP64 and mixed, roofline and "
                            "vcycle_roofline_frac the fraction of HBM peak",
        "value": n * cyc64 / (ms64 * 1e-3),
        "unit": "grid-pts/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms64,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": inp.name, "N": N, "cells": n, "tol": args.tol, "cycle": "V(2,2) RBGS",
                   "density_ratio": 1000},
        "time_to_tol_ms": {"fp64": ms64, "mixed": msmx, "mixed_speedup": ms64 / msmx},
        "cycles_to_tol": {"fp64": cyc64, "mixed_ir_steps": cycmx},
        "final_relres": {"fp64": hist64[-1], "mixed": histmx[-1]},
        "status": {"fp64": st64, "mixed": stmx},
        "krylov_fcg": kr,
        "coarsening_ablation": abl,
        "cut_cells": cut,
        "differentiation": diff,
        "rk2_projection": rk2,
        "vcycle_ms": {"fp64": vc64, "fp32": vc32},
        "vcycle_pts_per_s": {"fp64": n / (vc64 * 1e-3), "fp32": n / (vc32 * 1e-3)},
        # algorithmic scalars per finest cell per V(2,2) cycle: the FP64 finest grid reads
        # the density form (4 sweeps x 4 + 3.125 + 2.125), FP32 grids the face arrays
        "vcycle_roofline_frac": {"fp64": VCYCLE_SCALARS_F64 * 8 * n / (vc64 * 1e-3) / (HBM_PEAK_GBS * 1e9),
                                 "fp32": VCYCLE_SCALARS_F32 * 4 * n / (vc32 * 1e-3) / (HBM_PEAK_GBS * 1e9)},
        "roofline": {"bound": "hbm", "kernel": "rbgs_fused (finest grid, FP64 density form, one red-black sweep)",
                     "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "launch_ms": launch_ms, "bytes_per_launch": half_bytes},
        "input_gen_s": t_gen,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(inp)
    print(json.dumps(out), flush=True)


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
    """Where a V(2,2) cycle spends its time on the bench field: per grid with a coarser
    one below it (down to 32^3), the four sweeps, the residual + restriction and the
    prolongation, each timed through the component entry points with HIP events (best
    of the mean of 20 calls); the single-workgroup tail (16^3 and below) is the whole
    cycle minus those.  FP64 cycle, and the FP32 cycle of a mixed context."""
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
            if n_l <= 16:
                break
            p = torch.zeros((n_l,) * 3, dtype=dt, device="cuda")
            f = f0.to(dt) if lv == 0 else torch.randn((n_l,) * 3, dtype=torch.float64, device="cuda",
                                                       generator=g).to(dt)
            ec = torch.zeros((n_l // 2,) * 3, dtype=dt, device="cuda")
            sweeps = 2 * tm(lambda: mg.smooth(lv, p, f, 2, 0))
            rr = tm(lambda: mg.residual_restrict(lv, p, f))
            pro = tm(lambda: mg.prolong_add(lv, ec, p))
            grids.append({"n": n_l, "sweeps_us": sweeps, "residual_restrict_us": rr, "prolong_us": pro,
                          "total_us": sweeps + rr + pro})
            above += sweeps + rr + pro
            del p, f, ec
        pf = torch.zeros_like(f0, dtype=dt)
        ff = f0.to(dt)
        cycle = tm(lambda: mg.vcycle(pf, ff))
        out[prec] = {"cycle_us": cycle, "grids": grids, "tail_us": cycle - above}
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


def recorded_traffic(workload, N):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter
    runs (scaled FETCH_SIZE + WRITE_SIZE), or None when they were taken on another
    workload or the kernel source has changed since."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["k_rbgs_fused<double, 128, 16, true, false>"]
    except (OSError, KeyError, ValueError):
        return None
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"] or rec["workload"] != workload or rec["N"] != N:
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_baseline(inp):
    """The oracle's FP64 V-cycle on the same workload, timed on this host."""
    import numpy as np

    from oracle import multigrid as omg
    from oracle.operator import face_coeffs_from_rho, project
    t0 = time.time()
    H = omg.setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    t_setup = time.time() - t0
    fh = project(inp.f, H.fine.mask)
    p = np.zeros_like(fh)
    cycles = 0
    t0 = time.time()
    while cycles < 2 and time.time() - t0 < 30:
        p = omg.vcycle(H, p, fh)
        cycles += 1
    dt = (time.time() - t0) / cycles
    return {"value": inp.n / dt, "unit": "grid-pts/s", "cores": 1, "kind": "oracle",
            "sample": f"{cycles} FP64 V(2,2) cycles of the numpy oracle on the same {inp.N}^3 workload "
                      f"(setup {t_setup:.1f} s excluded); numpy elementwise kernels are single-threaded",
            "host_cpus": os.cpu_count()}


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
