"""On a uniform periodic mesh the shift is one (P+1)-point stencil on the cell
values (the paper finds RAM equivalent to FARGO on uniform meshes, Sec. 4.1;
FARGO's integer shift, Sec. 1): the oracle's shift against the
stencil written out from the Lagrange weights of the cumulative (the reading
the GPU's uniform-run tiles and their transpose in the backward step rest
on), FP64, to rounding.

With the shifted node of cell i in source cell i - K at theta (a shift of
(K - theta) cells), its partial integral is sum_e g_e M_{i-K+e}, g_e the
stencil weights above the node summed down to e (e >= 0) or minus those
below summed up to e (e < 0), so the destination value is
sum_d ([d == 0] + g_{d-1} - g_d) Q_{i-K+d}, d = -LO .. P-LO.  The weights
sum to one; the shift by a whole number of cells is a cyclic permutation.
"""
import numpy as np
import pytest

import oracle
from paper_2305_05362_amd import workloads as W


def lagrange_weights(theta, p):
    lo = (p - 1) // 2
    nodes = np.arange(p + 1) - lo
    w = np.ones(p + 1)
    for a in range(p + 1):
        for b in range(p + 1):
            if b != a:
                w[a] *= (theta - nodes[b]) / (nodes[a] - nodes[b])
    return w


def stencil(theta, p):
    lo = (p - 1) // 2
    w = lagrange_weights(theta, p)
    g = {}
    for e in range(0, p - lo):
        g[e] = w[lo + 1 + e:].sum()
    for e in range(-lo, 0):
        g[e] = -w[:lo + e + 1].sum()
    return {d: (1.0 if d == 0 else 0.0) + g.get(d - 1, 0.0) - g.get(d, 0.0)
            for d in range(-lo, p - lo + 1)}


def _shift(q, n, s, order):
    e = W.uniform_edges(n, 0.0, 1.0)
    rows = oracle.Rows(np.array([0, n]), e, True)
    return oracle.shift(rows, q, np.array([s]), 1.0, order)


@pytest.mark.parametrize("order", [1, 3, 5])
@pytest.mark.parametrize("theta", [0.0, 0.3, 0.77])
@pytest.mark.parametrize("k", [0, 3, -2, 67])
def test_uniform_shift_is_the_stencil(order, theta, k):
    n = 64
    rng = np.random.default_rng(order * 100 + k)
    q = 1.0 + rng.standard_normal(n)
    got = _shift(q, n, (k - theta) / n, order)
    cc = stencil(theta, order)
    want = np.zeros(n)
    for d, c in cc.items():
        want += c * np.roll(q, k - d)        # Q_{i-K+d}
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(q))


@pytest.mark.parametrize("order", [1, 3, 5])
def test_stencil_weights_sum_to_one_and_reduce(order):
    for theta in (0.0, 0.25, 0.9):
        cc = stencil(theta, order)
        assert abs(sum(cc.values()) - 1.0) <= 1e-15
    # theta = 0: the identity on the node's own cell
    cc = stencil(0.0, order)
    assert cc[0] == 1.0 and all(v == 0.0 for d, v in cc.items() if d != 0)
    # first order: the donor-cell (upwind) weights 1 - theta, theta
    if order == 1:
        cc = stencil(0.3, 1)
        assert abs(cc[0] - 0.7) <= 1e-15 and abs(cc[1] - 0.3) <= 1e-15
