"""Small random problems shared by the oracle pin tests (inputs only)."""
import numpy as np

from oracle.multigrid import setup
from oracle.operator import Level, close_faces, diagonal


def random_level(N, seed, body=True, contrast=1.0, h=None):
    """Random positive face coefficients, an optional box-shaped body, faces closed."""
    g = np.random.default_rng(seed)
    lo = 1.0 / contrast if contrast > 1 else 0.5
    bx, by, bz = (np.exp(g.uniform(np.log(lo), np.log(2.0), (N, N, N))) for _ in range(3))
    mask = np.ones((N, N, N), dtype=bool)
    if body:
        a = N // 4
        mask[a:a + max(1, N // 4), a:a + max(2, N // 3), a:a + max(2, N // 2)] = False
    bx, by, bz = close_faces(bx, by, bz, mask)
    lev = Level(bx, by, bz, mask, 1.0 / N if h is None else h)
    lev.mask = mask & (diagonal(lev) > 0)
    return lev


def random_hierarchy(N, seed, body=True, contrast=1.0):
    lev = random_level(N, seed, body, contrast)
    return setup(lev.bx, lev.by, lev.bz, lev.mask, lev.h)


def relerr(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))
