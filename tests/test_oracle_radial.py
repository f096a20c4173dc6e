"""Pins for the oracle's radial transport step of a polar grid (the standard
upwind half of a 2D split step: Section 3's dimensional splitting, with the
residual scheme along r in polar geometry and closed inner/outer edges).

Each test ties it to something other than itself:
  * exact rational brute force on tiny columns: slopes from exact centre
    gaps, fluxes as exact integrals of the upwind row's linear profile over
    the swept interval (not the closed-form face value), geometric factors;
  * zero velocity is the identity, bit for bit;
  * every column's mass sum_j A_j q_j (A_j the row's area per unit angle) is
    conserved (closed edges);
  * constant q with constant u: interior rows change by the closed form
    q (1 - dt u / r_j), r_j the row's centre (the flux divergence of polar
    geometry), the edge rows by their single face.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from brute import radial_exact, to_fr


def _area(re):
    return 0.5 * (re[1:] ** 2 - re[:-1] ** 2)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_radial_brute_force_tiny(seed):
    rng = np.random.default_rng(400 + seed)
    R = int(rng.integers(4, 8))
    w = rng.integers(1, 6, size=R)
    re = (16 + np.concatenate([[0], np.cumsum(w)])).astype(np.float64) / 16.0
    q = (rng.integers(-8, 9, size=(R, 2)) / 4.0 + 3.0).astype(np.float64)
    u = (rng.integers(-6, 7, size=(R + 1, 2)) / 32.0).astype(np.float64)
    dt = 1.0 / 8.0
    got = oracle.radial(re, q, u, dt)
    for col in range(2):
        want = radial_exact(to_fr(re), to_fr(q[:, col]), to_fr(u[:, col]), Fr(dt))
        want = np.array([float(v) for v in want])
        assert np.max(np.abs(got[:, col] - want)) <= 1e-14 * np.max(np.abs(want)), col


def test_radial_zero_velocity_identity():
    rng = np.random.default_rng(5)
    re = np.geomspace(0.4, 2.5, 65)
    q = rng.uniform(0.5, 2.0, (64, 100))
    out = oracle.radial(re, q, np.zeros((65, 100)), 0.37)
    assert np.array_equal(out, q)


def test_radial_conserves_column_mass():
    rng = np.random.default_rng(6)
    re = np.geomspace(0.4, 2.5, 129)
    q = 1.0 + 0.3 * rng.standard_normal((128, 50))
    u = 0.05 * rng.standard_normal((129, 50))
    dt = 0.4 * np.min(np.diff(re)) / np.max(np.abs(u))
    out = oracle.radial(re, q, u, dt)
    a = _area(re)[:, None]
    m0 = np.sum(q * a, axis=0)
    m1 = np.sum(out * a, axis=0)
    assert np.max(np.abs(m1 - m0) / np.sum(np.abs(q * a), axis=0)) <= 1e-14


def test_radial_constant_state_closed_form():
    re = np.geomspace(0.4, 2.5, 41)
    R = 40
    q0, u0, dt = 1.7, 0.02, 0.03
    out = oracle.radial(re, np.full((R, 3), q0), np.full((R + 1, 3), u0), dt)
    c = 0.5 * (re[1:] + re[:-1])
    a = _area(re)
    want = q0 * (1.0 - dt * u0 / c)
    want[0] = q0 - dt * re[1] * u0 * q0 / a[0]
    want[-1] = q0 + dt * re[R - 1] * u0 * q0 / a[-1]
    assert np.allclose(out, want[:, None], rtol=1e-14, atol=0)
