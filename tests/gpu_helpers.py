"""Shared helpers of the GPU parity tests: host <-> device copies and problems."""
import numpy as np
import torch

import fields
from oracle.multigrid import setup
from oracle.operator import face_coeffs_from_rho


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def maxrel(a, b):
    """max |a - b| / max |b|"""
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def raw_problem(N, seed, body=True, contrast=1000.0):
    """Random raw face coefficients (faces NOT closed) and a box body: setup input."""
    g = np.random.default_rng(seed)
    bx, by, bz = (np.exp(g.uniform(np.log(1.0 / contrast), np.log(2.0), (N, N, N))) for _ in range(3))
    mask = np.ones((N, N, N), dtype=np.uint8)
    if body:
        a = N // 4
        mask[a:a + N // 4, a:a + N // 3, a:a + N // 2] = 0
    return bx, by, bz, mask


def workload(name, N):
    """(inputs, oracle hierarchy) for a named workload at size N."""
    inp = fields.make(name, N)
    H = setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    return inp, H


def mg_from_inputs(inp, mixed=False):
    from paper_1410_2240_amd import MG
    return MG.from_rho(dev(inp.rho), dev(inp.mask), mixed=mixed)
