"""Input generators: determinism, compatibility and the shape of each workload."""
import numpy as np

import fields


def test_deterministic_fingerprints():
    a = fields.make("c1", 16)
    b = fields.make("c1", 16)
    assert fields.fingerprint(a.rho, a.mask, a.f) == fields.fingerprint(b.rho, b.mask, b.f)
    c = fields.make("c2", 16)
    assert fields.fingerprint(c.f) != fields.fingerprint(a.f)


def test_rhs_is_compatible_and_zero_in_body():
    for name in ("c1", "c2", "c5"):
        inp = fields.make(name, 32)
        m = inp.mask.astype(bool)
        assert abs(inp.f[m].sum()) < 1e-9 * np.abs(inp.f).sum()
        assert np.all(inp.f[~m] == 0)
        # divergence of unit-variance face-averaged velocities: std about 1.22 N
        assert 1.0 < inp.f[m].std() / inp.N < 1.4


def test_density_range_and_body():
    inp = fields.make("c2", 64)
    m = inp.mask.astype(bool)
    assert inp.rho[m].min() >= 1e-3 - 1e-15 and inp.rho.max() <= 1.0
    assert np.all(inp.rho[~m] == 1.0)
    # the ellipsoid (0.3, 0.08, 0.06) at 64^3 covers about 4/3 pi abc N^3 cells
    expected = 4.0 / 3.0 * np.pi * 0.3 * 0.08 * 0.06 * 64 ** 3
    assert 0.8 * expected < (~m).sum() < 1.2 * expected


def test_flat_interface_values():
    inp = fields.make("c1", 32)
    col = inp.rho[:, 0, 0]
    phi = (col - 1e-3) / (1 - 1e-3)
    # 2-cell smear: cells next to z = 1/2 sit at +-1/4 of the smear length
    assert abs(phi[15] - 0.5 * (1 - np.tanh(-0.25))) < 1e-12
    assert abs(phi[16] - 0.5 * (1 - np.tanh(0.25))) < 1e-12


def test_batch_and_weights_are_distinct_seeds():
    inp = fields.make("c4", 8)
    fb = fields.batch_rhs(inp.mask, 3)
    assert fb.shape == (3, 8, 8, 8)
    assert not np.allclose(fb[0], fb[1])
    w = fields.adjoint_weights(8, 2)
    assert w.shape == (2, 8, 8, 8) and not np.allclose(w[0], w[1])
