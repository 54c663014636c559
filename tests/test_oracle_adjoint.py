"""Pins for oracle.adjoint: adjoint identity and central finite differences."""
import numpy as np
import pytest

import fields
from oracle import adjoint, exact
from oracle.multigrid import setup, solve
from oracle.operator import face_coeffs_from_rho
from tests.oracle_helpers import relerr


def exact_p(rho, mask, f, h):
    H = setup(*face_coeffs_from_rho(rho, mask), mask, h)
    return exact.solve_sparse(H.fine, f)


def small_problem(N=8, body=True):
    inp = fields.wavy_body(N) if body else fields.flat(N, 2.0)
    return inp


def test_adjoint_identity():
    """w . p = mu . f for p = A^+ P f, mu = A^+ P w (A symmetric, same gauge)."""
    inp = fields.flat(16, 2.0)
    H = setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    w = fields.adjoint_weights(16, 2)
    p = np.stack([solve(H, inp.f, tol=1e-13)[0], solve(H, -2 * inp.f, tol=1e-13)[0]])
    mu = adjoint.adjoint_solve(H, w, tol=1e-13)
    fs = np.stack([inp.f, -2 * inp.f])
    for b in range(2):
        lhs = np.sum(w[b] * p[b])
        rhs = np.sum(mu[b] * fs[b])
        assert abs(lhs - rhs) <= 1e-9 * abs(lhs)


@pytest.mark.parametrize("body", [False, True])
def test_density_gradient_central_differences(body):
    """dL/drho by the adjoint against (L(rho + eps e_c) - L(rho - eps e_c)) / 2 eps,
    with every solve done by the sparse direct solver."""
    N = 8
    inp = small_problem(N, body)
    H = setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    w = fields.adjoint_weights(N, 1)[0]
    p = exact.solve_sparse(H.fine, inp.f)
    mu = exact.solve_sparse(H.fine, w)
    g = adjoint.density_gradient(adjoint.face_gradient(mu, p, H.fine), H.fine)
    cells = np.random.default_rng(80).choice(N ** 3, 12, replace=False)
    # cells next to the interface, where the gradient is largest
    cells = np.concatenate([cells, np.ravel_multi_index(([N // 2, N // 2 - 1], [1, 2], [3, 4]), (N, N, N))])
    for c in cells:
        idx = np.unravel_index(c, (N, N, N))
        if not inp.mask[idx]:
            continue
        eps = 1e-6 * inp.rho[idx]
        rp = inp.rho.copy()
        rp[idx] += eps
        rm = inp.rho.copy()
        rm[idx] -= eps
        Lp = np.sum(w * exact_p(rp, inp.mask, inp.f, inp.h))
        Lm = np.sum(w * exact_p(rm, inp.mask, inp.f, inp.h))
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - g[idx]) <= 1e-5 * abs(g).max(), (idx, fd, g[idx])


def test_rhs_gradient_is_adjoint_solution():
    """p is linear in f, so dL/df_c is exact by one difference."""
    N = 8
    inp = small_problem(N, True)
    H = setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    w = fields.adjoint_weights(N, 1)[0]
    mu = exact.solve_sparse(H.fine, w)
    p0 = exact.solve_sparse(H.fine, inp.f)
    for c in (5, 77, 300):
        idx = np.unravel_index(c, (N, N, N))
        if not inp.mask[idx]:
            continue
        f1 = inp.f.copy()
        f1[idx] += 1.0
        dL = np.sum(w * (exact.solve_sparse(H.fine, f1) - p0))
        assert abs(dL - mu[idx]) <= 1e-9 * np.abs(mu).max()


def test_gradients_driver_matches_direct():
    inp = fields.flat(16, 2.0)
    H = setup(*face_coeffs_from_rho(inp.rho, inp.mask), inp.mask, inp.h)
    w = fields.adjoint_weights(16, 2)
    fs = np.stack([inp.f, inp.f[::-1].copy()])
    p = np.stack([exact.solve_fft_z(H.fine, fb) for fb in fs])
    mu, grho = adjoint.gradients(H, p, w, tol=1e-13)
    mu_x = np.stack([exact.solve_fft_z(H.fine, wb) for wb in w])
    assert relerr(mu, mu_x) < 1e-9
    g_x = adjoint.density_gradient(adjoint.face_gradient(mu_x, p, H.fine), H.fine)
    assert relerr(grho, g_x) < 1e-9
