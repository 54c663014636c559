"""Python binding of the multigrid pressure solve (thin wrapper over the C ABI).

torch supplies device memory (the workspace and outputs) and the stream; every step
of the solve runs in the HIP library.  Arrays are contiguous CUDA tensors of shape
(N, N, N) (or (B, N, N, N) for batched right-hand sides), indexed [k, j, i].
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (MG_COARSEN_DENSITY, MG_EBREAKDOWN, MG_ENOCONV, MG_FP64, MG_FROM_RHO, MG_KRYLOV, MG_MIXED, MG_OK,
                   MG_POST, MG_PRE, MG_PREC_F32, MG_PREC_F64, MgStats)


class MGError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what} failed ({_lib.ERROR_NAMES.get(code, code)}): {_lib.last_error()}")


def _check(rc: int, what: str):
    if rc < 0:
        raise MGError(rc, what)
    return rc


def _ptr(t: torch.Tensor | None, dtype=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("solver arrays must be CUDA (HIP) tensors")
    if not t.is_contiguous():
        raise ValueError("solver arrays must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _grid_n(t: torch.Tensor) -> int:
    n = t.shape[-1]
    if t.shape[-3:] != (n, n, n):
        raise ValueError(f"expected (..., N, N, N) arrays, got {tuple(t.shape)}")
    return n


def _flags(mixed: bool, krylov: bool) -> int:
    return (MG_MIXED if mixed else MG_FP64) | (MG_KRYLOV if krylov else 0)


def workspace_size(n: int, mixed: bool = False, krylov: bool = False) -> int:
    return int(_lib.load().mg_workspace_size(_lib.dims3(n), _flags(mixed, krylov)))


def coeffs_from_rho(rho: torch.Tensor, mask: torch.Tensor):
    """(bx, by, bz): face products 1/rho x open area, beta_f = o_f 2/(rho_L + rho_R)."""
    n = _grid_n(rho)
    bx, by, bz = (torch.empty_like(rho) for _ in range(3))
    _check(_lib.load().mg_coeffs_from_rho(_ptr(rho, torch.float64), _ptr(mask, torch.uint8), _lib.dims3(n),
                                          _ptr(bx), _ptr(by), _ptr(bz), _stream(rho.device)), "mg_coeffs_from_rho")
    return bx, by, bz


class MG:
    """A multigrid hierarchy on a caller-owned torch workspace.

    mixed: FP32 V-cycles inside FP64 refinement.  krylov: flexible CG preconditioned
    by one V-cycle per step (outer iteration), instead of plain V-cycle iteration.
    lanes: extra streams on which a batched solve runs right-hand sides concurrently
    (mg_add_lanes; each lane's scratch is one more workspace tensor slice).
    """

    def __init__(self, bx, by, bz, mask, h: float | None = None, mixed: bool = False, krylov: bool = False,
                 _rho=None, _density_coarsening: bool = False, lanes: int = 0):
        lib = _lib.load()
        ref = bx if _rho is None else _rho
        n = _grid_n(ref)
        self.n = n
        self.h = 1.0 / n if h is None else float(h)
        self.mixed = bool(mixed)
        self.krylov = bool(krylov)
        self.device = ref.device
        flags = (_flags(mixed, krylov) | (MG_COARSEN_DENSITY if _density_coarsening else 0)
                 | (MG_FROM_RHO if _rho is not None else 0))
        size = lib.mg_workspace_size(_lib.dims3(n), flags)
        if size == 0:
            raise ValueError(f"unsupported grid {n}^3")
        self.workspace = torch.empty(size, dtype=torch.uint8, device=ref.device)
        ctx = ctypes.c_void_p()
        if _rho is None:
            rc = lib.mg_setup(ctypes.byref(ctx), _ptr(self.workspace), size, _ptr(bx, torch.float64),
                              _ptr(by, torch.float64), _ptr(bz, torch.float64), _ptr(mask, torch.uint8),
                              _lib.dims3(n), self.h, flags, _stream(ref.device))
        else:
            rc = lib.mg_setup_from_rho(ctypes.byref(ctx), _ptr(self.workspace), size, _ptr(_rho, torch.float64),
                                       _ptr(mask, torch.uint8), _lib.dims3(n), self.h, flags, _stream(ref.device))
        _check(rc, "mg_setup")
        self._ctx = ctx
        self._destroy = lib.mg_destroy   # kept so that teardown at interpreter exit still finds it
        self.levels = lib.mg_level_info(ctx, 0, None, None)
        self.lanes = int(lanes)
        self.lane_workspace = None
        if self.lanes > 0:
            per = lib.mg_lane_workspace_size(_lib.dims3(n), flags)
            self.lane_workspace = torch.empty(self.lanes * per, dtype=torch.uint8, device=ref.device)
            _check(lib.mg_add_lanes(ctx, _ptr(self.lane_workspace), self.lanes * per, self.lanes), "mg_add_lanes")

    @classmethod
    def from_rho(cls, rho, mask, h=None, mixed=False, krylov=False, coarsening="face", lanes=0):
        """Hierarchy from the cell density.  coarsening = "face" moves the face products
        to the coarse grids (section 3.1); "density" restricts density and areas apart,
        the variant the paper rejects (for comparison)."""
        if coarsening not in ("face", "density"):
            raise ValueError("coarsening must be 'face' or 'density'")
        return cls(None, None, None, mask, h, mixed, krylov, _rho=rho, _density_coarsening=coarsening == "density",
                   lanes=lanes)

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        destroy = getattr(self, "_destroy", None)
        if ctx is not None and ctx.value and destroy is not None:
            destroy(ctx)
            self._ctx = None

    def _sync_stream(self):
        _lib.load().mg_set_stream(self._ctx, _stream(self.device))

    # ---------------------------------------------------------------- solve

    def solve(self, f, p=None, tol: float = 1e-10, max_cycles: int = 100, raise_on_fail: bool = True,
              static_scratch: bool = False):
        """Solve A p = P f (batched over a leading axis).  Returns (p, hist, stats).

        hist is a list (per batch item) of relative residuals, the first for the guess.
        static_scratch: call mg_solve_static, whose scratch is the library's static
        device array instead of this hierarchy's workspace (grids up to 128^3 in FP64,
        64^3 mixed or flexible CG).
        """
        self._sync_stream()
        batched = f.dim() == 4
        B = f.shape[0] if batched else 1
        if p is None:
            p = torch.zeros_like(f)
        hist = np.zeros(B * (max_cycles + 1), dtype=np.float64)
        n_hist = (ctypes.c_int * B)()
        stats = MgStats()
        lib = _lib.load()
        entry = lib.mg_solve_static if static_scratch else lib.mg_solve
        rc = entry(self._ctx, _ptr(f, torch.float64), _ptr(p, torch.float64), B, float(tol), int(max_cycles),
                   hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n_hist, ctypes.byref(stats))
        if rc < 0 and (raise_on_fail or rc not in (MG_ENOCONV, MG_EBREAKDOWN)):
            raise MGError(rc, "mg_solve_static" if static_scratch else "mg_solve")
        rows = hist.reshape(B, max_cycles + 1)
        hists = [rows[b, :n_hist[b]].tolist() for b in range(B)]
        out = stats.as_dict()
        out["status"] = rc
        return p, (hists if batched else hists[0]), out

    def apply(self, p):
        self._sync_stream()
        Ap = torch.empty_like(p)
        B = p.shape[0] if p.dim() == 4 else 1
        _check(_lib.load().mg_apply(self._ctx, _ptr(p, torch.float64), _ptr(Ap), B), "mg_apply")
        return Ap

    def coeff_grad(self, mu, p, faces: bool = False):
        """dL/drho (and dL/dbeta on the low faces if faces=True) from adjoint and primal solutions."""
        self._sync_stream()
        B = p.shape[0] if p.dim() == 4 else 1
        shape = p.shape[-3:]
        grho = torch.empty(shape, dtype=torch.float64, device=p.device)
        g = [torch.empty(shape, dtype=torch.float64, device=p.device) for _ in range(3)] if faces else [None] * 3
        _check(_lib.load().mg_coeff_grad(self._ctx, _ptr(mu, torch.float64), _ptr(p, torch.float64), B,
                                         _ptr(g[0]), _ptr(g[1]), _ptr(g[2]), _ptr(grho)), "mg_coeff_grad")
        return (grho, tuple(g)) if faces else grho

    # ---------------------------------------------------------------- Runge-Kutta stage

    def divergence(self, u, r=None, dt: float = 1.0):
        """f = div(U + dt R) / dt from face velocities u = (ux, uy, uz) (and R)."""
        self._sync_stream()
        f = torch.empty_like(u[0])
        rr = (None, None, None) if r is None else r
        _check(_lib.load().mg_divergence(self._ctx, *(_ptr(t, torch.float64) for t in u),
                                         *(_ptr(t, torch.float64) for t in rr), float(dt), _ptr(f)), "mg_divergence")
        return f

    def project(self, u, p, r=None, dt: float = 1.0):
        """u <- u + dt R - dt beta grad p on open faces, 0 on closed ones (in place)."""
        self._sync_stream()
        rr = (None, None, None) if r is None else r
        _check(_lib.load().mg_project(self._ctx, *(_ptr(t, torch.float64) for t in u),
                                      *(_ptr(t, torch.float64) for t in rr), float(dt), _ptr(p, torch.float64)),
               "mg_project")
        return u

    # ---------------------------------------------------------------- components

    def level_info(self, level: int):
        n = ctypes.c_int()
        h = ctypes.c_double()
        _check(_lib.load().mg_level_info(self._ctx, level, ctypes.byref(n), ctypes.byref(h)), "mg_level_info")
        return n.value, h.value

    def level_coeffs(self, level: int):
        self._sync_stream()
        n, _ = self.level_info(level)
        out = [torch.empty((n, n, n), dtype=torch.float64, device=self.device) for _ in range(3)]
        mask = torch.empty((n, n, n), dtype=torch.uint8, device=self.device)
        _check(_lib.load().mg_level_coeffs(self._ctx, level, *(_ptr(t) for t in out), _ptr(mask)), "mg_level_coeffs")
        return out[0], out[1], out[2], mask

    @staticmethod
    def _prec(t):
        return MG_PREC_F32 if t.dtype == torch.float32 else MG_PREC_F64

    def smooth(self, level, p, f, sweeps=1, order=MG_PRE):
        self._sync_stream()
        _check(_lib.load().mg_smooth(self._ctx, self._prec(p), level, _ptr(p, p.dtype), _ptr(f, p.dtype), sweeps,
                                     order), "mg_smooth")
        return p

    def residual_restrict(self, level, p, f):
        self._sync_stream()
        n, _ = self.level_info(level + 1)
        fc = torch.empty((n, n, n), dtype=p.dtype, device=p.device)
        _check(_lib.load().mg_residual_restrict(self._ctx, self._prec(p), level, _ptr(p, p.dtype), _ptr(f, p.dtype),
                                                _ptr(fc)), "mg_residual_restrict")
        return fc

    def prolong_add(self, level, ec, p):
        self._sync_stream()
        _check(_lib.load().mg_prolong_add(self._ctx, self._prec(p), level, _ptr(ec, p.dtype), _ptr(p, p.dtype)),
               "mg_prolong_add")
        return p

    def coarse_solve(self, f):
        self._sync_stream()
        e = torch.empty_like(f)
        _check(_lib.load().mg_coarse_solve(self._ctx, self._prec(f), _ptr(f, f.dtype), _ptr(e)), "mg_coarse_solve")
        return e

    def vcycle(self, p, f):
        self._sync_stream()
        _check(_lib.load().mg_vcycle(self._ctx, self._prec(p), _ptr(p, p.dtype), _ptr(f, p.dtype)), "mg_vcycle")
        return p


__all__ = ["MG", "MGError", "coeffs_from_rho", "workspace_size", "MG_PRE", "MG_POST", "MG_OK"]
