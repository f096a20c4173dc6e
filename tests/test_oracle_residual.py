"""Pins for the oracle's residual upwind step (Eq. splitting_second).

The paper gives the reconstruction (PLM with the van Leer harmonic slope,
Section 3.1) and says the residual is solved by standard upwind methods; the
flux form used here is a reading (the swept-interval average of the upwind
linear profile).  Pins:
  * exact rational brute force that integrates the upwind linear profile over
    the swept interval (independent of the closed-form face state);
  * identity when dv = 0; constants preserved under constant dv; total mass
    conserved (Eq. qmass_total);
  * dv*dt equal to the cell size on a uniform mesh moves the profile exactly
    one cell (footnote of Section 4.1);
  * no new extrema with constant dv and Courant number <= 1;
  * second-order convergence on smooth data.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from brute import residual_exact, to_fr, vl_slope_exact
from paper_2305_05362_amd import workloads as W


def _row(edges):
    return oracle.Rows.single(edges)


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_tiny(seed):
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(4, 9))
    w = rng.integers(1, 6, size=n)
    e = np.concatenate([[0], np.cumsum(w)]).astype(np.float64) / 32
    q = rng.integers(-8, 9, size=n).astype(np.float64) / 8.0 + 1.0
    dv = rng.integers(-4, 5, size=n).astype(np.float64) / 16.0
    dt = 1.0 / 16
    got = oracle.residual(_row(e), q, dv, dt)
    want = np.array([float(x) for x in residual_exact(to_fr(e), to_fr(q), to_fr(dv), to_fr([dt])[0])])
    assert np.max(np.abs(got - want)) < 1e-14 * 8


def test_van_leer_slope_cases():
    # harmonic mean of the two one-sided slopes; zero at extrema (Section 3.1)
    e = to_fr(np.arange(7, dtype=np.float64))
    q = to_fr([0.0, 1.0, 3.0, 2.0, 2.0, 5.0])
    assert vl_slope_exact(e, q, 1) == Fr(4, 3)   # 2*2*1/(2+1)
    assert vl_slope_exact(e, q, 2) == 0          # local max
    assert vl_slope_exact(e, q, 4) == 0          # flat on one side


def test_identity_when_dv_zero():
    rng = np.random.default_rng(1)
    e = W.stretched_edges(40, 20.0, rng)
    q = rng.standard_normal(40)
    out = oracle.residual(_row(e), q, np.zeros(40), 0.3)
    assert np.array_equal(out, q)


def test_constant_state_and_mass():
    rng = np.random.default_rng(2)
    n = 64
    e = W.stretched_edges(n, 20.0, rng)
    dx = np.diff(e)
    out = oracle.residual(_row(e), np.full(n, 1.75), np.full(n, 0.4), 0.5 * dx.min() / 0.4)
    assert np.max(np.abs(out - 1.75)) < 1e-14
    q = 1.0 + rng.standard_normal(n)
    dv = rng.standard_normal(n)
    dt = 0.5 * np.min(np.minimum(dx, np.roll(dx, 1)) / np.abs(dv))
    out = oracle.residual(_row(e), q, dv, dt)
    assert abs(np.sum(out * dx) - np.sum(q * dx)) < 1e-14 * np.sum(np.abs(q * dx)) * 4


@pytest.mark.parametrize("sign", [1, -1])
def test_courant_one_is_exact_roll(sign):
    n = 32
    e = W.uniform_edges(n, 0.0, 1.0)
    q = np.random.default_rng(3).standard_normal(n)
    out = oracle.residual(_row(e), q, np.full(n, sign * 1.0), 1.0 / n)
    assert np.max(np.abs(out - np.roll(q, sign))) < 1e-13


def test_no_new_extrema_constant_velocity():
    rng = np.random.default_rng(4)
    n = 100
    e = W.stretched_edges(n, 8.0, rng)
    dx = np.diff(e)
    q = np.where(np.arange(n) % 37 < 15, 2.0, 0.5) + 0.2 * np.sin(np.arange(n))
    for v in (0.7, -0.7):
        dt = 0.9 * dx.min() / abs(v)
        out = q.copy()
        for _ in range(50):
            out = oracle.residual(_row(e), out, np.full(n, v), dt)
        assert out.max() <= q.max() + 1e-13 and out.min() >= q.min() - 1e-13


def test_second_order_smooth():
    errs = []
    for n in (64, 128, 256):
        e = W.uniform_edges(n, 0.0, 1.0)
        q0 = W.sine_cell_averages(e, 1.0, 0.5)
        v, dt = 1.0, 0.5 / n
        steps = int(round(1.0 / (v * dt)))
        q = q0.copy()
        for _ in range(steps):
            q = oracle.residual(_row(e), q, np.full(n, v), dt)
        errs.append(np.mean(np.abs(q - q0)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > 1.8, rates


def test_step_is_shift_then_residual():
    wl = W.small_polar(3, 64)
    rows = oracle.Rows.from_workload(wl)
    a = oracle.step(rows, wl.q0, wl.v0, wl.dv, wl.dt, 5, 1)
    b = oracle.residual(rows, oracle.shift(rows, wl.q0, wl.v0, wl.dt, 5), wl.dv, wl.dt)
    assert np.array_equal(a, b)
