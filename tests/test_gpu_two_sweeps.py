"""The two-sweep pass (two red-black sweeps per march up z, density form, grids of 256^3
and up; FP32 in 128 x 16 tiles, FP64 in 32 x 32 tiles) against the one-pass sweep and
the oracle.

Each update of the two-sweep pass does the arithmetic of the one-pass sweep on the same
neighbour values, so two sweeps in one pass must equal two one-pass sweeps bit for bit:
both orders, sweep counts 2 to 4 (pairs and a single sweep after them), at 256^3
(32-plane z-chunks, seven chunk seams per column) and 512^3 (two chunks), on the crest
field with its body (walls, body faces, dropped cells) and the wavy field; 1024^3 (whole
columns) on the headline field.  The FP32 V-cycle built on it, whose pre-smoothing of a
correction starts from a zero input without reading it, is compared element by element
with the oracle's FP32 V-cycle on the density-form FP32 operator at 256^3.
"""
import numpy as np
import pytest
import torch

import fields
from oracle import multigrid as omg
from oracle.operator import face_coeffs_from_rho, project
from tests.gpu_helpers import dev, host, maxrel

pytestmark = pytest.mark.gpu


def mixed_context(name, N):
    from paper_1410_2240_amd import MG
    inp = fields.make(name, N)
    return inp, MG.from_rho(dev(inp.rho), dev(inp.mask), mixed=True)


def random_fp32(inp, seed, dtype=torch.float32):
    g = torch.Generator(device="cuda").manual_seed(seed)
    live = dev(inp.mask).bool()
    p = torch.randn(inp.rho.shape, generator=g, device="cuda", dtype=dtype) * live
    f = torch.randn(inp.rho.shape, generator=g, device="cuda", dtype=dtype) * live
    return p, f


def one_pass_sweeps(mg, p, f, sweeps, order):
    for _ in range(sweeps):
        p = mg.smooth(0, p, f, 1, order)   # one sweep per call: the one-pass kernel
    return p


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["fp32", "fp64"])
@pytest.mark.parametrize("name,N", [("c5", 256), ("c2", 256), pytest.param("c5", 512, marks=pytest.mark.slow)])
def test_two_sweeps_equal_two_one_pass_sweeps(name, N, dtype):
    inp, mg = mixed_context(name, N)
    for order in (0, 1):
        for sweeps in (2, 3, 4):
            print(f"two-sweep pass {name} {N}^3 {dtype} order={order} sweeps={sweeps}", flush=True)
            p, f = random_fp32(inp, 10 * sweeps + order, dtype)
            got = mg.smooth(0, p.clone(), f, sweeps, order)
            want = one_pass_sweeps(mg, p.clone(), f, sweeps, order)
            assert torch.equal(got, want), (order, sweeps)


@pytest.mark.slow
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["fp32", "fp64"])
def test_two_sweeps_equal_two_one_pass_sweeps_1024(dtype):
    """The headline grid: whole-column chunks (FP32: 512 workgroups in two rounds; FP64:
    1024 in four)."""
    inp, mg = mixed_context("c5", 1024)
    for order in (0, 1):
        print(f"two-sweep pass c5 1024^3 {dtype} order={order}", flush=True)
        p, f = random_fp32(inp, 1024 + order, dtype)
        got = mg.smooth(0, p.clone(), f, 2, order)
        want = one_pass_sweeps(mg, p.clone(), f, 2, order)
        assert torch.equal(got, want), order
        del got, want, p, f
        torch.cuda.empty_cache()


def test_fp32_vcycle_256_matches_density_form_oracle():
    """One FP32 V(2,2) cycle from a zero guess (as in every refinement or flexible-CG
    step) at 256^3 against the oracle's FP32 cycle on the same FP32 operator: the finest
    grid formed from fl32(rho), the coarse grids the rounded FP64 face products, the 4^3
    solve in FP64; element by element, to a few float32 ulps of the largest value."""
    inp, mg = mixed_context("c2", 256)
    H = omg.setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    lv32 = omg.fp32_levels_from_rho(H, inp.rho)
    r32 = project(inp.f, H.fine.mask).astype(np.float32)
    print("FP32 V-cycle 256^3: oracle", flush=True)
    want = omg.vcycle(H, np.zeros_like(r32), r32, lv32)
    print("FP32 V-cycle 256^3: GPU", flush=True)
    got = host(mg.vcycle(dev(np.zeros_like(r32)), dev(r32)))
    assert got.dtype == np.float32
    assert maxrel(got, want) <= 1e-4
