"""Pin of the window rule of tests/windows.py: the oracle's value at a sampled cell from
an 8^3 window equals the whole-grid oracle's value there, for one red-black sweep in
either order (two sweeps from a 12^3 window), the residual + 8-child restriction and the trilinear prolongation, at
random cells, on both z walls, across the periodic wrap in x and y and next to the body
(32^3 Stokes-crest field with its droplets, bubbles and the ellipsoid)."""
import numpy as np
import pytest

import fields
from oracle import multigrid as omg
from oracle.operator import face_coeffs_from_rho
from tests import windows as win


@pytest.fixture(scope="module")
def crest():
    N = 32
    inp = fields.make("c5", N)
    H = omg.setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    g = np.random.default_rng(77)
    p = np.where(inp.mask == 1, g.standard_normal((N, N, N)), 0.0)
    f = g.standard_normal((N, N, N))
    e = g.standard_normal((N // 2,) * 3)
    cells = [tuple(int(v) for v in g.integers(0, N, 3)) for _ in range(40)]
    cells += [(0, 0, 0), (N - 1, N - 1, N - 1), (1, 5, N - 1), (N - 2, 0, 7), (0, N - 1, 0), (N - 1, 3, 0)]
    cells += [tuple(int(v) for v in c) for c in np.argwhere(inp.mask == 0)[::97]]
    return inp, H, p, f, e, cells


@pytest.mark.parametrize("sweeps", [1, 2])
@pytest.mark.parametrize("order", [0, 1])
def test_sweep_window(crest, order, sweeps):
    inp, H, p, f, e, cells = crest
    whole = omg.smooth(p, f, H.fine, sweeps, (omg.RED, omg.BLACK) if order == 0 else (omg.BLACK, omg.RED))
    for c in cells:
        v, _ = win.sweep_at(inp.rho, inp.mask, p, f, inp.h, c, order, sweeps)
        assert v == whole[c], c


def test_residual_restrict_window(crest):
    inp, H, p, f, e, cells = crest
    whole = omg.restrict(omg.residual(p, f, H.fine))
    for c in cells:
        cc = (c[0] // 2, c[1] // 2, c[2] // 2)
        v, _ = win.residual_restrict_at(inp.rho, inp.mask, p, f, inp.h, cc)
        assert abs(v - whole[cc]) <= 1e-15 * np.abs(whole).max(), cc


def test_prolong_add_window(crest):
    inp, H, p, f, e, cells = crest
    whole = omg.prolong_add(p, e, H.fine)
    for c in cells:
        v, _ = win.prolong_add_at(inp.rho, inp.mask, p, e, inp.h, c)
        assert v == whole[c], c
