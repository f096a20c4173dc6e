"""Pins for the oracle's fourth-order conversion between centre values and
cell averages (Section 3.1's remark that Q_i = <Q>_i is a second-order
assumption, with the correction <Q>_i = Q_i + (Q_{i+1} - 2 Q_i + Q_{i-1})/24),
and for the step on a state of centre values built from it.

Each test ties it to something other than itself:
  * exactness, in exact rational arithmetic: centre values of a cubic on a
    uniform mesh, and of a quadratic on a stretched mesh, give the exact cell
    averages in every cell whose stencil does not wrap (the expansion
    <q> = q + dx^2 q''/24 + dx^4 q''''/1920 and the three-point second
    derivative's exactness for quadratics);
  * on a uniform periodic mesh it is the paper's printed formula, and it
    conserves sum_i Q_i (the global conservation the paper notes);
  * convergence against analytic cell averages of a smooth periodic function:
    fourth order on uniform and on smoothly stretched meshes, for both the
    conversion and its inverse;
  * the point the correction makes: a point-sampled function shifted on a
    smoothly stretched mesh converges at second order when the centre values
    are taken as averages, at fourth order with the conversion around the
    step (against the exact shifted point values).
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from paper_2305_05362_amd import workloads as W

L = 2.0 * math.pi


def _poly_avg_exact(coef, a, b):
    """Exact average of sum_k coef[k] x^k over [a, b] (Fractions)."""
    P = lambda x: sum(c * x ** (k + 1) / (k + 1) for k, c in enumerate(coef))
    return (P(b) - P(a)) / (b - a)


def _poly_val(coef, x):
    return sum(c * x ** k for k, c in enumerate(coef))


def _exactness(edges, coef, tol):
    x = [Fr(float(v)) for v in edges]
    n = len(edges) - 1
    centres = [(x[i] + x[i + 1]) / 2 for i in range(n)]
    q = np.array([float(_poly_val(coef, c)) for c in centres])
    got = oracle.average4(oracle.Rows.single(edges), q)
    for i in range(1, n - 1):
        want = float(_poly_avg_exact(coef, x[i], x[i + 1]))
        assert abs(got[i] - want) <= tol * max(1.0, abs(want)), (i, got[i], want)
    return got


def test_cubic_exact_on_uniform_mesh():
    edges = np.arange(17) / 16.0
    coef = [Fr(1, 3), Fr(-2, 7), Fr(5, 2), Fr(-11, 5)]
    _exactness(edges, coef, 2e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_quadratic_exact_on_stretched_mesh(seed):
    edges = W.stretched_edges(23, 8.0, np.random.default_rng(seed))
    coef = [Fr(3, 7), Fr(-5, 3), Fr(9, 4)]
    _exactness(edges, coef, 1e-13)


def test_cubic_not_exact_on_stretched_mesh():
    # the three-point second derivative is only exact for quadratics there,
    # so a cubic must leave an error (the test above is discriminating)
    edges = W.stretched_edges(23, 8.0, np.random.default_rng(5))
    x = [Fr(float(v)) for v in edges]
    coef = [Fr(0), Fr(0), Fr(0), Fr(7)]
    q = np.array([float(_poly_val(coef, (x[i] + x[i + 1]) / 2)) for i in range(23)])
    got = oracle.average4(oracle.Rows.single(edges), q)
    err = max(abs(got[i] - float(_poly_avg_exact(coef, x[i], x[i + 1])))
              for i in range(1, 22))
    assert err > 1e-8


def test_uniform_is_the_printed_formula_and_conserves():
    rng = np.random.default_rng(3)
    edges = W.uniform_edges(40, -1.0, 3.0)
    q = rng.standard_normal(40)
    rows = oracle.Rows.single(edges)
    got = oracle.average4(rows, q)
    want = q + (np.roll(q, -1) - 2.0 * q + np.roll(q, 1)) / 24.0
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)
    assert abs(got.sum() - q.sum()) <= 1e-13 * np.abs(q).sum()
    back = oracle.point4(rows, q)
    assert abs(back.sum() - q.sum()) <= 1e-13 * np.abs(q).sum()


def _f(x):
    return np.sin(x) + 0.3 * np.cos(3.0 * x)


def _F(x):
    return -np.cos(x) + 0.1 * np.sin(3.0 * x)


def _mesh(kind, n):
    if kind == "uniform":
        return W.uniform_edges(n, -math.pi, math.pi)
    xi = np.linspace(-math.pi, math.pi, n + 1)
    x = xi + 0.5 * np.sin(xi)                  # smooth stretching, ratio up to 3
    x[0], x[-1] = -math.pi, math.pi
    return x


def _orders(errs):
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


NS = [64, 128, 256, 512]


@pytest.mark.parametrize("kind", ["uniform", "smooth"])
def test_conversions_converge_at_fourth_order(kind):
    e_avg, e_inv = [], []
    for n in NS:
        x = _mesh(kind, n)
        c = 0.5 * (x[1:] + x[:-1])
        avg = (_F(x[1:]) - _F(x[:-1])) / np.diff(x)
        rows = oracle.Rows.single(x)
        e_avg.append(np.max(np.abs(oracle.average4(rows, _f(c)) - avg)))
        e_inv.append(np.max(np.abs(oracle.point4(rows, avg) - _f(c))))
    assert min(_orders(e_avg)) >= 3.9
    assert min(_orders(e_inv)) >= 3.9


def test_step_on_centre_values_lifts_the_second_order_cap():
    """Shift of centre values by 0.2137 of the period, order 5, no residual,
    on the smoothly stretched mesh: against the exact shifted point values."""
    s = 0.2137 * L
    e4, e2 = [], []
    for n in NS:
        x = _mesh("smooth", n)
        c = 0.5 * (x[1:] + x[:-1])
        rows = oracle.Rows.single(x)
        want = _f(c - s)
        e4.append(np.max(np.abs(
            oracle.step_point4(rows, _f(c), np.array([1.0]), None, s, 5, 1) - want)))
        e2.append(np.max(np.abs(
            oracle.step(rows, _f(c), np.array([1.0]), None, s, 5, 1) - want)))
    assert min(_orders(e4)) >= 3.9
    assert max(_orders(e2)) <= 2.1
    assert e4[-1] < 1e-3 * e2[-1]
