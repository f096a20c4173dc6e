"""Rows whose last tile is shorter than the interpolation stencil: that tile's
window overlaps itself (and, across the row's end, the first tile's), so some
window cells collect terms from three tiles.  The FP64 adjoints against the
oracle (Section 3's shift transposed; Section 3.1's limited shift and
residual transposed) at the FP64 bars, and bit-equal over repeated calls (the
shared cells are summed in a fixed order, not by atomics).

Per-row meshes (the ragged kernels, tiles of 251 cells): rows of 3 x 251 + 3,
251 + 1, 2 x 251 + 4, 4 x 251 + 2, 8 and 300 cells.  A shared mesh (the
general kernel, tiles of 1019 cells): rows of 2 x 1019 + 3 cells.  Lagrange
orders 1, 3, 5 with and without the residual, and both limited shifts.
"""
import numpy as np
import pytest
import torch

import oracle
from parity import CELL_F64, assert_parity
from paper_2305_05362_amd import _lib as R
from paper_2305_05362_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=dtype, device=DEV)


def _ragged(order):
    rng = np.random.default_rng(61)
    lens = np.array([251 * 3 + 3, 251 + 1, 251 * 2 + 4, 251 * 4 + 2, 8, 300])
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    edges, q, dv = [], [], []
    for n in lens:
        e = W.stretched_edges(int(n), 6.0, rng)
        edges.append(e)
        q.append(1.0 + 0.3 * rng.standard_normal(n))
        dv.append(0.3 * np.minimum(np.diff(e), np.roll(np.diff(e), 1)) * rng.uniform(-1, 1, n))
    v0 = rng.uniform(-30.0, 30.0, len(lens)) / lens
    return W.Workload("short_tiles", len(lens), 0, row_ptr, np.concatenate(edges), False,
                      np.concatenate(q), np.concatenate(dv), v0, 1.0, order, 1)


def _shared(order):
    rng = np.random.default_rng(67)
    n, n_rows = 2 * 1019 + 3, 3
    e = W.stretched_edges(n, 6.0, rng)
    q = 1.0 + 0.3 * rng.standard_normal((n_rows, n))
    dvv = 0.3 * np.minimum(np.diff(e), np.roll(np.diff(e), 1))
    dv = dvv[None, :] * rng.uniform(-1, 1, (n_rows, n))
    v0 = np.array([0.37, -23.1, 412.6]) / n
    return W.Workload("short_tiles_shared", n_rows, n, np.arange(n_rows + 1) * n, e, True, q,
                      dv, v0, 1.0, order, 1)


CASES = {"ragged": _ragged, "shared": _shared}


def _repeat(fn, k=3):
    outs = [fn() for _ in range(k)]
    torch.cuda.synchronize()
    for o in outs[1:]:
        for x, y in zip(outs[0], o):
            if x is not None:
                assert torch.equal(x, y)
    return outs[0]


@pytest.mark.parametrize("residual", [False, True])
@pytest.mark.parametrize("order", [1, 3, 5])
@pytest.mark.parametrize("kind", list(CASES))
def test_step_adjoint_short_last_tiles(kind, order, residual):
    wl = CASES[kind](order)
    orows = oracle.Rows.from_workload(wl)
    rng = np.random.default_rng(order)
    qf = wl.q0.reshape(-1)
    qh = oracle.shift(orows, qf, wl.v0, wl.dt, order) if residual else None
    dv = wl.dv.reshape(-1) if residual else None
    rbar = rng.standard_normal(wl.n_cells)
    rows = R.Rows.from_workload(wl, DEV)
    v0 = dev(wl.v0)

    def call():
        out = torch.full((wl.n_cells,), float("nan"), dtype=torch.float64, device=DEV)
        dvb = torch.zeros(wl.n_cells, dtype=torch.float64, device=DEV) if residual else None
        v0b = torch.zeros(wl.n_rows, dtype=torch.float64, device=DEV)
        R.ram_step_adjoint(rows, dev(qf), None if qh is None else dev(qh),
                           None if dv is None else dev(dv), dev(rbar), out, v0, wl.dt, order,
                           dvb, v0b)
        return out, dvb, v0b
    out, dvb, v0b = _repeat(call)
    rb = rbar
    rdvb = None
    if residual:
        rb, rdvb = oracle.residual_adjoint(orows, qh, dv, rbar, wl.dt)
    ref, rv = oracle.shift_adjoint(orows, qf, rb, wl.v0, wl.dt, order)
    assert_parity(out.cpu().numpy(), ref, 1e-12, CELL_F64, "qbar")
    if residual:
        assert_parity(dvb.cpu().numpy(), rdvb, 1e-12, CELL_F64, "dvbar")
    assert np.max(np.abs(v0b.cpu().numpy() - rv)) <= 1e-10 * np.max(np.abs(rv))


@pytest.mark.parametrize("recon", [R.RAM_RECON_PLM, R.RAM_RECON_PPM])
@pytest.mark.parametrize("kind", list(CASES))
def test_limited_adjoint_short_last_tiles(kind, recon):
    wl = CASES[kind](5)
    orows = oracle.Rows.from_workload(wl)
    qf = wl.q0.reshape(-1)
    qb = np.random.default_rng(9).standard_normal(wl.n_cells)
    rows = R.Rows.from_workload(wl, DEV)
    v0 = dev(wl.v0)

    def call():
        out = torch.full((wl.n_cells,), float("nan"), dtype=torch.float64, device=DEV)
        v0b = torch.zeros(wl.n_rows, dtype=torch.float64, device=DEV)
        R.ram_shift_limited_adjoint(rows, dev(qf), dev(qb), out, v0, wl.dt, recon, v0b)
        return out, v0b
    out, v0b = _repeat(call)
    ref, rv = oracle.shift_recon_adjoint(orows, qf, qb, wl.v0, wl.dt, recon)
    assert_parity(out.cpu().numpy(), ref, 1e-12, CELL_F64, "qbar")
    assert np.max(np.abs(v0b.cpu().numpy() - rv)) <= 1e-10 * np.max(np.abs(rv))
