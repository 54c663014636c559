"""Seeded synthetic inputs for the pressure-projection workloads.

This module only builds inputs: the VOF fraction phi, the cell density rho,
the body mask and the right-hand side f.  It holds none of the solver's
arithmetic (no face coefficients, no operator, no smoothing, no transfers)
and imports neither the oracle nor the HIP package, so both of those can be
fed from it without sharing code.

Conventions (shared by every consumer):
  * N cells per side, h = 1/N, cell (i, j, k) centred at ((i+1/2)h, (j+1/2)h, (k+1/2)h);
  * arrays are C-contiguous with shape (N, N, N) indexed [k, j, i] (x fastest);
  * x and y are periodic, z has walls at z = 0 and z = 1;
  * mask = 1 for fluid (water or air) cells, 0 for cells inside the immersed body.

Physics behind the recipe (paper section 2):
  * density from the VOF fraction, eq. (density): rho = lambda + (1 - lambda) H(phi)
    with lambda = rho_air / rho_water = 1e-3 and H the identity on a tanh-mollified
    phi, i.e. rho = phi + 1e-3 (1 - phi): water has rho = 1, air rho = 1e-3;
  * the Poisson source is a divergence, eq. (poisson1): f = div(u / dt + R).  Here
    f is the discrete divergence of a seeded N(0, 1) cell velocity field, formed from
    face velocities (mean of the two adjacent cells), with zero normal velocity on
    the z walls and on every face that touches the body (the no-flux condition of
    eq. (neumann) for a body at rest).  Its sum over fluid cells telescopes to zero;
    the fluid mean is removed anyway to clean up rounding.

Seeds: numpy.random.default_rng([1410, field, index]) with
  field 0 = cell velocity (index = z-slab k), field 1 = adjoint weights w (index = b),
  field 2 = free-surface modes, field 3 = crest features,
  field 4 = batch velocity (index = b*N + k).
Every random draw is per z-slab or per batch item, so large grids are generated
slab by slab and are bitwise reproducible whatever the chunking.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

SEED = 1410
F_VELOCITY, F_WEIGHTS, F_SURFACE, F_CREST, F_BATCH_VELOCITY = 0, 1, 2, 3, 4
LAMBDA = 1.0e-3  # rho_air / rho_water

# Immersed ellipsoid body: semi-axes along x, y, z.
BODY_SEMI_AXES = (0.3, 0.08, 0.06)


def rng(field: int, index: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED, field, index])


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _over_slabs(N: int, fn, min_n: int = 128) -> None:
    """Run fn(k0, k1) over contiguous z ranges covering 0..N-1, on a thread pool for
    large grids (numpy releases the GIL on slab-sized arrays).  Every draw and every
    value of a slab depends on its index only, so the result is the same bits whatever
    the split."""
    W = _workers() if N >= min_n else 1
    if W == 1:
        fn(0, N)
        return
    step = -(-N // (4 * W))
    with ThreadPoolExecutor(W) as ex:
        for fut in [ex.submit(fn, k0, min(N, k0 + step)) for k0 in range(0, N, step)]:
            fut.result()


def centres(N: int) -> np.ndarray:
    return (np.arange(N, dtype=np.float64) + 0.5) / N


@dataclasses.dataclass
class Inputs:
    """One synthetic workload: C-contiguous (N, N, N) arrays indexed [k, j, i]."""
    name: str
    N: int
    rho: np.ndarray        # float64 cell density (1 inside the body; unused there)
    mask: np.ndarray       # uint8, 1 = fluid, 0 = body
    f: np.ndarray          # float64 right-hand side, zero fluid mean, 0 in the body

    @property
    def h(self) -> float:
        return 1.0 / self.N

    @property
    def n(self) -> int:
        return self.N ** 3


# ---------------------------------------------------------------- geometry

def density_from_phi(phi: np.ndarray, lam: float = LAMBDA) -> np.ndarray:
    """Eq. (density) with H = identity on an already mollified phi."""
    return phi + lam * (1.0 - phi)


def flat_phi_column(N: int, smear_cells: float) -> np.ndarray:
    """phi(z) = (1 - tanh((z - 1/2) / (smear_cells h))) / 2: water below z = 1/2."""
    z = centres(N)
    return 0.5 * (1.0 - np.tanh((z - 0.5) / (smear_cells / N)))


def wavy_surface_modes():
    """16 distinct integer wavevectors (kx, ky) from the half plane, 1 <= |k| <= 8,
    amplitude 0.02/|k| and a uniform random phase each (seeded, field 2)."""
    cand = [(kx, ky) for ky in range(0, 9) for kx in range(-8, 9)
            if (ky > 0 or kx > 0) and 1 <= kx * kx + ky * ky <= 64]
    g = rng(F_SURFACE)
    pick = g.choice(len(cand), size=16, replace=False)
    theta = g.uniform(0.0, 2.0 * math.pi, size=16)
    return [(cand[p][0], cand[p][1], 0.02 / math.hypot(*cand[p]), th)
            for p, th in zip(pick, theta)]


def wavy_surface(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """z_s(x, y) = 1/2 + sum_m a_m cos(2 pi (kx x + ky y) + theta_m) (broadcasting)."""
    zs = 0.5 + np.zeros(np.broadcast(x, y).shape)
    for kx, ky, a, th in wavy_surface_modes():
        zs = zs + a * np.cos(2.0 * math.pi * (kx * x + ky * y) + th)
    return zs


def stokes_eta(x):
    """Third-order Stokes wave, slope ka = 0.3, k = 4 pi, crests at x = 1/4 and 3/4."""
    k = 4.0 * math.pi
    ka = 0.3
    a = ka / k
    th = k * (x - 0.25)
    return 0.5 + a * (np.cos(th) + 0.5 * ka * np.cos(2 * th) + 0.375 * ka * ka * np.cos(3 * th))


def body_mask_slab(N: int, k: int, centre) -> np.ndarray:
    """mask for z-slab k: 0 where the cell centre is strictly inside the ellipsoid."""
    x = centres(N)
    z = (k + 0.5) / N
    ax, ay, az = BODY_SEMI_AXES
    cx, cy, cz = centre
    q = (((x[None, :] - cx) / ax) ** 2 + ((x[:, None] - cy) / ay) ** 2 + ((z - cz) / az) ** 2)
    return (q >= 1.0).astype(np.uint8)


def body_psi_corners(N: int, centre, axes=BODY_SEMI_AXES) -> np.ndarray:
    """The body as a level set at the cell corners (i h, j h, k h), k = 0..N, shape
    (N+1, N, N): psi = (|(x - c) / a| - 1) min(a), positive in the fluid, negative in
    the body, zero on the ellipsoid (the paper builds psi from hull panels; an
    analytic ellipsoid stands in)."""
    g = np.arange(N) / N
    gz = np.arange(N + 1) / N
    q = (((g[None, None, :] - centre[0]) / axes[0]) ** 2 + ((g[None, :, None] - centre[1]) / axes[1]) ** 2
         + ((gz[:, None, None] - centre[2]) / axes[2]) ** 2)
    return (np.sqrt(q) - 1.0) * min(axes)


def wavy_cut(N: int):
    """The wavy-interface field with the ellipsoid as a cut-cell body: (rho, psi).
    rho comes from the interface everywhere (cut cells hold fluid); psi at corners."""
    x = centres(N)
    zs = wavy_surface(x[None, :], x[:, None])
    zc = float(wavy_surface(np.array(0.5), np.array(0.5)))
    h = 1.0 / N
    z = centres(N)[:, None, None]
    rho = density_from_phi(0.5 * (1.0 - np.tanh((z - zs[None]) / (2.0 * h))))
    return rho, body_psi_corners(N, (0.5, 0.5, zc))


# ---------------------------------------------------------------- right-hand side

def _velocity_slab(field: int, index: int, N: int) -> np.ndarray:
    return rng(field, index).standard_normal((3, N, N))


def divergence_rhs(mask: np.ndarray, field: int = F_VELOCITY, index0: int = 0,
                   out: np.ndarray | None = None) -> np.ndarray:
    """f = discrete divergence of a seeded N(0,1) cell velocity field.

    Face velocity = mean of the two adjacent cell velocities times the open-face
    indicator (both cells fluid; z walls closed).  Slab k draws its velocity from
    rng(field, index0 + k).  Returns f with its fluid mean removed and 0 in the body.
    """
    N = mask.shape[0]
    inv_h = float(N)
    f = np.empty((N, N, N)) if out is None else out
    m = mask.astype(bool)
    sums = np.zeros(N)
    counts = np.zeros(N, dtype=np.int64)

    def slabs(k0, k1):
        u_prev = _velocity_slab(field, index0 + k0 - 1, N) if k0 > 0 else None
        u_cur = _velocity_slab(field, index0 + k0, N)
        for k in range(k0, k1):
            u_next = _velocity_slab(field, index0 + k + 1, N) if k + 1 < N else None
            mk = m[k]
            ux, uy, uz = u_cur
            # x faces: low face of cell i sits between i-1 (periodic) and i
            ox = mk & np.roll(mk, 1, axis=1)
            Ux = np.where(ox, 0.5 * (ux + np.roll(ux, 1, axis=1)), 0.0)
            oy = mk & np.roll(mk, 1, axis=0)
            Uy = np.where(oy, 0.5 * (uy + np.roll(uy, 1, axis=0)), 0.0)
            div = (np.roll(Ux, -1, axis=1) - Ux) + (np.roll(Uy, -1, axis=0) - Uy)
            if k > 0:   # face between k-1 and k
                Uz_lo = np.where(mk & m[k - 1], 0.5 * (uz + u_prev[2]), 0.0)
            else:
                Uz_lo = 0.0
            if k + 1 < N:   # face between k and k+1
                Uz_hi = np.where(mk & m[k + 1], 0.5 * (uz + u_next[2]), 0.0)
            else:
                Uz_hi = 0.0
            div = div + (Uz_hi - Uz_lo)
            f[k] = np.where(mk, div * inv_h, 0.0)
            sums[k] = float(f[k][mk].sum())
            counts[k] = int(mk.sum())
            u_prev, u_cur = u_cur, u_next

    _over_slabs(N, slabs)
    # the fluid mean, summed slab by slab in z order
    total = 0.0
    for k in range(N):
        total += float(sums[k])
    mean = total / int(counts.sum())

    def remove(k0, k1):
        for k in range(k0, k1):
            f[k] = np.where(m[k], f[k] - mean, 0.0)

    _over_slabs(N, remove)
    return f


def adjoint_weights(N: int, batch: int) -> np.ndarray:
    """w_b ~ N(0, 1) per cell, b = 0..batch-1 (field 1, index b)."""
    return np.stack([rng(F_WEIGHTS, b).standard_normal((N, N, N)) for b in range(batch)])


def batch_rhs(mask: np.ndarray, batch: int) -> np.ndarray:
    """batch right-hand sides, item b from velocity seeds (field 4, index b*N + k)."""
    N = mask.shape[0]
    out = np.empty((batch, N, N, N))
    for b in range(batch):
        divergence_rhs(mask, F_BATCH_VELOCITY, b * N, out=out[b])
    return out


# ---------------------------------------------------------------- workloads

def flat(N: int, smear_cells: float = 2.0, name: str = "flat") -> Inputs:
    """Flat interface at z = 1/2, no body (the 32^3, 128^3 and 512^3 workloads)."""
    col = density_from_phi(flat_phi_column(N, smear_cells))
    rho = np.empty((N, N, N))
    rho[...] = col[:, None, None]
    mask = np.ones((N, N, N), dtype=np.uint8)
    return Inputs(name, N, rho, mask, divergence_rhs(mask))


def wavy_body(N: int, name: str = "wavy_body") -> Inputs:
    """Random-phase wavy interface smeared over 2 cells plus the ellipsoid body."""
    x = centres(N)
    zs = wavy_surface(x[None, :], x[:, None])          # [j, i]
    zc = float(wavy_surface(np.array(0.5), np.array(0.5)))
    rho = np.empty((N, N, N))
    mask = np.empty((N, N, N), dtype=np.uint8)
    h = 1.0 / N

    def slabs(k0, k1):
        for k in range(k0, k1):
            z = (k + 0.5) * h
            phi = 0.5 * (1.0 - np.tanh((z - zs) / (2.0 * h)))
            mk = body_mask_slab(N, k, (0.5, 0.5, zc))
            mask[k] = mk
            rho[k] = np.where(mk == 1, density_from_phi(phi), 1.0)

    _over_slabs(N, slabs)
    return Inputs(name, N, rho, mask, divergence_rhs(mask))


def crest_features(N: int):
    """Seeded overturning-crest features around the x = 3/4 crest (field 3)."""
    h = 1.0 / N
    g = rng(F_CREST)
    yc = g.uniform(0.3, 0.7)
    xc = 0.75
    emax = float(stokes_eta(xc))
    drops = np.column_stack([g.uniform(xc - 0.05, xc + 0.15, 64), g.uniform(yc - 0.2, yc + 0.2, 64),
                             g.uniform(emax + 0.02, emax + 0.12, 64), g.uniform(2 * h, 8 * h, 64)])
    bubbles = np.column_stack([g.uniform(xc - 0.1, xc + 0.1, 64), g.uniform(yc - 0.2, yc + 0.2, 64),
                               g.uniform(emax - 0.2, emax - 0.07, 64), g.uniform(2 * h, 8 * h, 64)])
    return dict(xc=xc, yc=yc, emax=emax, drops=drops, bubbles=bubbles)


def _stokes_distance_slab(N: int, k: int, feat) -> np.ndarray:
    """signed distance (negative in water) for z-slab k, shape [j, i]."""
    h = 1.0 / N
    x = centres(N)
    z = (k + 0.5) * h
    eta = stokes_eta(x)
    d = np.broadcast_to(z - eta[None, :], (N, N)).copy()
    yc, xc, emax = feat["yc"], feat["xc"], feat["emax"]
    band = np.abs(x[:, None] - yc) - 0.2                  # [j, 1]
    # water lip (y-aligned cylinder), then trapped air cavity under it
    for (zx, zz, r, water) in ((xc + 0.04, emax - 0.01, 0.02, True),
                               (xc + 0.04, emax - 0.04, 0.015, False)):
        rc = np.sqrt((x[None, :] - zx) ** 2 + (z - zz) ** 2) - r
        dc = np.maximum(rc, band)
        d = np.minimum(d, dc) if water else np.maximum(d, -dc)
    for spheres, water in ((feat["drops"], True), (feat["bubbles"], False)):
        for sx, sy, sz, r in spheres:
            if abs(z - sz) > r + 4 * h:
                continue
            i0 = max(int((sx - r) * N) - 4, 0)
            i1 = min(int((sx + r) * N) + 5, N)
            j0 = max(int((sy - r) * N) - 4, 0)
            j1 = min(int((sy + r) * N) + 5, N)
            xs = x[i0:i1][None, :]
            ys = x[j0:j1][:, None]
            ds = np.sqrt((xs - sx) ** 2 + (ys - sy) ** 2 + (z - sz) ** 2) - r
            sub = d[j0:j1, i0:i1]
            d[j0:j1, i0:i1] = np.minimum(sub, ds) if water else np.maximum(sub, -ds)
    return d


def stokes_crest(N: int, name: str = "stokes_crest") -> Inputs:
    """Steep Stokes wave (slope 0.3) with a seeded overturning crest, plus the body."""
    h = 1.0 / N
    feat = crest_features(N)
    zc = float(stokes_eta(0.5))
    rho = np.empty((N, N, N))
    mask = np.empty((N, N, N), dtype=np.uint8)

    def slabs(k0, k1):
        for k in range(k0, k1):
            d = _stokes_distance_slab(N, k, feat)
            phi = 0.5 * (1.0 - np.tanh(d / h))
            mk = body_mask_slab(N, k, (0.5, 0.5, zc))
            mask[k] = mk
            rho[k] = np.where(mk == 1, density_from_phi(phi), 1.0)

    _over_slabs(N, slabs)
    return Inputs(name, N, rho, mask, divergence_rhs(mask))


# name -> (builder, default N)
WORKLOADS = {
    "c1": (lambda N: flat(N, 2.0, "c1_flat_smear2"), 32),
    "c2": (lambda N: wavy_body(N, "c2_wavy_body"), 256),
    "c3": (lambda N: flat(N, 1.0, "c3_flat_smear1"), 512),
    "c4": (lambda N: flat(N, 2.0, "c4_flat_smear2"), 128),
    "c5": (lambda N: stokes_crest(N, "c5_stokes_crest"), 1024),
}


def make(config: str, N: int | None = None) -> Inputs:
    builder, n0 = WORKLOADS[config]
    return builder(n0 if N is None else N)


def fingerprint(*arrays) -> str:
    """SHA-256 over the raw bytes of the given arrays (determinism checks)."""
    hsh = hashlib.sha256()
    for a in arrays:
        hsh.update(np.ascontiguousarray(a).tobytes())
    return hsh.hexdigest()
