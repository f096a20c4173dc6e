"""Pins for the oracle's adjoint of the limited (PLM / PPM) bulk shift.

The limited shift is nonlinear; its adjoint is the transpose of the Jacobian
at the forward state.  Each test ties it to something other than itself:
  * the full Jacobian by central differences of the (separately pinned)
    forward oracle on tiny rows, column by column; a column whose differences
    at eps and eps/2 disagree holds a limiter switching point inside the
    interval and is skipped (counted, and required to be rare);
  * the v0 derivative by central differences in s;
  * PLM shifted by less than a cell is the swept-interval upwind step, so its
    adjoint equals the residual adjoint with dv = s/dt (that adjoint is
    pinned by its own finite differences and dot-product tests).
"""
import numpy as np
import pytest

import oracle
from paper_2305_05362_amd import workloads as W


def _row(e):
    return oracle.Rows.single(e)


def _jac_fd(e, q, s, recon, eps):
    n = len(q)
    J = np.empty((n, n))
    for k in range(n):
        d = np.zeros(n)
        d[k] = eps
        fp = oracle.shift_recon(_row(e), q + d, np.array([s]), 1.0, recon)
        fm = oracle.shift_recon(_row(e), q - d, np.array([s]), 1.0, recon)
        J[:, k] = (fp - fm) / (2 * eps)
    return J


@pytest.mark.parametrize("recon", [oracle.PLM, oracle.PPM])
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_adjoint_is_jacobian_transpose(recon, seed):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(7, 13))
    w = rng.uniform(0.5, 2.0, n)
    e = np.concatenate([[0.0], np.cumsum(w)]) / np.sum(w)
    q = 1.0 + 0.5 * np.sin(2 * np.pi * 0.5 * (e[:-1] + e[1:])) + 0.2 * rng.standard_normal(n)
    skipped = 0
    for s in (0.037, -0.61, 2.3, rng.uniform(-5, 5)):
        qb = rng.standard_normal(n)
        got, _ = oracle.shift_recon_adjoint(_row(e), q, qb, np.array([s]), 1.0, recon)
        J1 = _jac_fd(e, q, s, recon, 1e-6)
        J2 = _jac_fd(e, q, s, recon, 5e-7)
        smooth = np.max(np.abs(J1 - J2), axis=0) <= 1e-6 * (1 + np.max(np.abs(J1), axis=0))
        skipped += int(np.sum(~smooth))
        want = J1.T @ qb
        scale = np.max(np.abs(J1.T @ np.abs(qb))) + 1e-300
        assert np.all(np.abs(got - want)[smooth] <= 1e-7 * scale), (s, got - want)
    assert skipped <= 2, skipped


@pytest.mark.parametrize("recon", [oracle.PLM, oracle.PPM])
def test_v0_derivative_by_differences(recon):
    wl = W.small_polar(3, 300)
    rows = oracle.Rows.from_workload(wl)
    rng = np.random.default_rng(4)
    qb = rng.standard_normal(wl.n_cells)
    _, v0b = oracle.shift_recon_adjoint(rows, wl.q0, qb, wl.v0, wl.dt, recon)
    for r in range(wl.n_rows):
        eps = 1e-7 * abs(wl.v0[r])

        def f(dv):
            v = wl.v0.copy()
            v[r] += dv
            return float(np.dot(qb, oracle.shift_recon(rows, wl.q0, v, wl.dt, recon)))

        fd = (f(eps) - f(-eps)) / (2 * eps)
        assert abs(v0b[r] - fd) <= 1e-5 * max(abs(fd), 1e-3), (r, v0b[r], fd)


def test_plm_subcell_adjoint_is_residual_adjoint():
    rng = np.random.default_rng(13)
    n = 200
    e = W.stretched_edges(n, 6.0, rng, 0.0, 1.0)
    q = 1.0 + 0.5 * np.sin(2 * np.pi * 5 * 0.5 * (e[:-1] + e[1:])) + 0.1 * rng.standard_normal(n)
    qb = rng.standard_normal(n)
    rows = _row(e)
    for s in (0.6 * np.min(np.diff(e)), -0.45 * np.min(np.diff(e))):
        got, _ = oracle.shift_recon_adjoint(rows, q, qb, np.array([s]), 1.0, oracle.PLM)
        want, _ = oracle.residual_adjoint(rows, q, np.full(n, s), qb, 1.0)
        assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want)), s
