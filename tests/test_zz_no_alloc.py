"""mg_solve_static, the solve for callers that cannot allocate device memory, against
mg_solve on the same hierarchies: bit for bit the same p, history and statistics, on
two calls in a row (a 64^3 hierarchy, then a smaller 32^3 one, so the second call finds
the first call's contents in the shared static scratch), for FP64, mixed and flexible
CG, with batches; the largest supported FP64 grid (128^3); and the error for a hierarchy
whose solve scratch exceeds the static array.  mg_solve on the same context afterwards
still gives its own result (the context's workspace pointers are put back)."""
import numpy as np
import pytest
import torch

import fields
from tests.gpu_helpers import dev

pytestmark = pytest.mark.gpu


def solve_both(mg, f, tol=1e-10, max_cycles=60):
    p0, h0, s0 = mg.solve(f, tol=tol, max_cycles=max_cycles)
    p1, h1, s1 = mg.solve(f, tol=tol, max_cycles=max_cycles, static_scratch=True)
    torch.cuda.synchronize()
    assert torch.equal(p0, p1)
    assert h0 == h1
    for k in ("cycles", "levels", "active_cells", "dropped_cells", "removed_mean", "final_relres", "status"):
        assert s0[k] == s1[k], k
    return p0, h0


@pytest.mark.parametrize("mixed,krylov", [(False, False), (True, False), (False, True), (True, True)])
def test_static_scratch_solve_equals_workspace_solve(mixed, krylov):
    from paper_1410_2240_amd import MG
    for N in (64, 32):   # the second call is the smaller grid
        print(f"static scratch: {N}^3 mixed={mixed} krylov={krylov}", flush=True)
        inp = fields.make("c2", N)
        mg = MG.from_rho(dev(inp.rho), dev(inp.mask), mixed=mixed, krylov=krylov)
        f = dev(inp.f)
        p, hist = solve_both(mg, f)
        assert hist[-1] <= 1e-10
        # batched right-hand sides, item after item
        fb = dev(fields.batch_rhs(inp.mask, 2))
        pb0, hb0, _ = mg.solve(fb, tol=1e-10, max_cycles=60)
        pb1, hb1, _ = mg.solve(fb, tol=1e-10, max_cycles=60, static_scratch=True)
        assert torch.equal(pb0, pb1) and hb0 == hb1
        # the workspace solve again, after the static one: unchanged
        p2, h2, _ = mg.solve(f, tol=1e-10, max_cycles=60)
        assert torch.equal(p, p2) and h2 == hist


def test_static_scratch_largest_fp64_grid():
    from paper_1410_2240_amd import MG
    print("static scratch: 128^3 FP64", flush=True)
    inp = fields.make("c4", 128)
    mg = MG.from_rho(dev(inp.rho), dev(inp.mask))
    _, hist = solve_both(mg, dev(inp.f))
    assert hist[-1] <= 1e-10


def test_static_scratch_rejects_a_larger_solve():
    from paper_1410_2240_amd import MG, MGError
    from paper_1410_2240_amd._lib import MG_EINVAL
    print("static scratch: 128^3 mixed is too large", flush=True)
    inp = fields.make("c4", 128)
    mg = MG.from_rho(dev(inp.rho), dev(inp.mask), mixed=True)
    f = dev(inp.f)
    p = torch.full_like(f, 7.0)
    with pytest.raises(MGError) as e:
        mg.solve(f, p=p, static_scratch=True)
    assert e.value.code == MG_EINVAL and "static scratch" in str(e.value)
    assert bool((p == 7.0).all())   # nothing was queued
    _, hist, st = mg.solve(f, tol=1e-10)
    assert st["status"] == 0
