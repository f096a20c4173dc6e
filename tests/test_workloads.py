"""Pins for the input generators (meshes of Appendix B, configuration shapes)."""
import math

import numpy as np
import pytest
from scipy import integrate

from paper_2305_05362_amd import workloads as W


@pytest.mark.parametrize("abc", [(0.2, 0.3, 9.0), (math.pi / 2, math.pi / 2 + 0.1, 5.0),
                                 (1.0, 1.1, 9.0), (0.1387, 0.2773, 15.0)])
def test_bump_cumulative_matches_quadrature(abc):
    a, b, c = abc
    xmin, xmax = -math.pi, math.pi
    inorm = W.bump_norm(xmin, xmax, a, b, c)
    # Eq. Inorm against numerical quadrature of psi
    q, _ = integrate.quad(lambda s: W.bump_density(np.array([s]), a, b, c)[0],
                          xmin, xmax, points=[-b, -a, a, b], limit=200)
    assert abs(q - inorm) < 1e-10
    xs = np.linspace(xmin, xmax, 41)
    for x in xs:
        q, _ = integrate.quad(lambda s: W.bump_density(np.array([s]), a, b, c)[0],
                              xmin, x, points=[p for p in (-b, -a, a, b) if xmin < p < x] or None,
                              limit=200)
        assert abs(W.bump_cumulative(x, xmin, xmax, a, b, c) - q / inorm) < 1e-11
    assert abs(W.bump_cumulative(xmax, xmin, xmax, a, b, c) - 1.0) < 1e-15


def test_bump_edges_index_property_and_ratio():
    n = 2048
    e = W.bump_edges(n, -math.pi, math.pi, 0.2, 0.3, 9.0)
    F = n * W.bump_cumulative(e, -math.pi, math.pi, 0.2, 0.3, 9.0)
    assert np.max(np.abs(F - np.arange(n + 1))) < 1e-9
    dx = np.diff(e)
    assert np.all(dx > 0)
    assert abs(dx.max() / dx.min() - 10.0) < 1e-6


def test_stretched_edges_ratio():
    e = W.stretched_edges(5000, 20.0, np.random.default_rng(0))
    dx = np.diff(e)
    assert e[0] == 0.0 and e[-1] == 1.0 and np.all(dx > 0)
    assert dx.max() / dx.min() <= 20.0 + 1e-9


def test_sine_cell_averages_exact():
    e = W.stretched_edges(50, 5.0, np.random.default_rng(1))
    q = W.sine_cell_averages(e, 1.0, 0.5, 3, 0.4)
    for i in (0, 17, 49):
        v, _ = integrate.quad(lambda x: 1 + 0.5 * math.sin(2 * math.pi * 3 * x + 0.4), e[i], e[i + 1])
        assert abs(q[i] - v / (e[i + 1] - e[i])) < 1e-12


def test_polar_recipe_shapes():
    wl = W.small_polar(6, 128)
    assert wl.q0.shape == (6, 128) and wl.dv.shape == (6, 128)
    rc = 0.5 * (wl.meta["r_edges"][:-1] + wl.meta["r_edges"][1:])
    assert np.allclose(wl.v0, rc ** -1.5)
    dx = np.diff(wl.edges)
    lim = np.minimum(dx, np.roll(dx, 1))
    assert np.max(np.abs(wl.dv) * wl.dt / lim[None, :]) <= 0.5 + 1e-12


def test_cfg1_shape():
    wl = W.cfg1()
    assert wl.n_cells == 256 and wl.v0[0] * wl.dt * 256 == pytest.approx(10.3)
