"""Parity of the trajectory-recording step and the one-step adjoint (C ABI)
with the FP64 oracle.

* ram_step_record: every recorded state equals ram_step's bit for bit; the
  recorded post-shift states match the oracle's shift to 1e-12 relative L1.
* ram_step_adjoint: qbar, dvbar and v0bar against the oracle's residual
  transpose followed by its shift transpose, FP64 <= 1e-12 relative L1 (v0bar
  <= 1e-10 of its largest entry: a sum of many signed terms); FP32 state
  <= 1e-5 against the oracle run on the same FP32 inputs (v0bar <= 1e-3: it
  sums differences of the FP32 reconstruction slope), also on a uniform mesh
  whose tiles all take the transposed stencil (orders 1, 3 and 5, with and
  without the residual, shifts of many cells and of whole periods), and one
  row of 2^18 + 5 cells with a shorter cell (both paths, at scale).
  Covered: rows of
  one and of several tiles, ragged batches with per-row meshes, large shifts,
  a tile whose source window overflows the on-chip buffer, and steps without
  a residual.
"""
import numpy as np
import pytest
import torch

import oracle
from parity import CELL_F32, CELL_F32_ADJ, CELL_F64, assert_parity
from paper_2305_05362_amd import _lib as R
from paper_2305_05362_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=dtype, device=DEV)


def rel_l1(a, b):
    return float(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))


def _uniform(order, n_rows=5, n=3500, seed=13):
    """Rows on one uniform mesh: every tile lies in the mesh's uniform run
    (the FP32 paths then share one set of weights per tile)."""
    rng = np.random.default_rng(seed)
    e = W.uniform_edges(n, 0.0, 1.0)
    xc = 0.5 * (e[:-1] + e[1:])
    q = 1.0 + 0.3 * np.sin(2 * np.pi * xc)[None, :] + 0.05 * rng.standard_normal((n_rows, n))
    dv = 0.2 / n * rng.uniform(-1, 1, (n_rows, n))
    v0 = rng.uniform(-40.0, 40.0, n_rows) / n
    return W.Workload("uniform", n_rows, n, np.arange(n_rows + 1) * n, e, True, q, dv, v0,
                      1.0, order, 1)


def _cases():
    return {
        "polar_one_tile": lambda o: W.small_polar(6, 800, order=o),
        "polar_tiles": lambda o: W.small_polar(3, 3500, order=o),
        "ragged": lambda o: W.small_ragged(12, 6, 2600, seed=31, order=o),
        "uniform": lambda o: _uniform(o),
    }


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind", ["polar_tiles", "ragged"])
def test_step_record_matches_step(kind, dtype):
    wl = _cases()[kind](5)
    rows = R.Rows.from_workload(wl, DEV)
    k = 5
    scan = R.RAM_SCAN_F64
    traj = torch.empty((k + 1, wl.n_cells), dtype=dtype, device=DEV)
    half = torch.empty((k, wl.n_cells), dtype=dtype, device=DEV)
    traj[0] = dev(wl.q0, dtype)
    v0, dv = dev(wl.v0), dev(wl.dv, dtype)
    R.ram_step_record(rows, traj, half, v0, dv, wl.dt, wl.order, k, scan)
    q = dev(wl.q0, dtype)
    for i in range(k):
        R.ram_step(rows, q, v0, dv, wl.dt, wl.order, 1, scan)
        assert torch.equal(q, traj[i + 1]), i
    torch.cuda.synchronize()
    if dtype == torch.float64:
        orows = oracle.Rows.from_workload(wl)
        for i in (0, k - 1):
            ref = oracle.shift(orows, traj[i].cpu().numpy(), wl.v0, wl.dt, wl.order)
            assert_parity(half[i].cpu().numpy(), ref, 1e-12, CELL_F64)


def _oracle_step_adjoint(wl, qf, qh, dv, rbar, v0, order):
    orows = oracle.Rows.from_workload(wl)
    dvb = None
    if dv is not None:
        rbar, dvb = oracle.residual_adjoint(orows, qh, dv, rbar, wl.dt)
    qb, v0b = oracle.shift_adjoint(orows, qf, rbar, v0, wl.dt, order)
    return qb, dvb, v0b


def _gpu_step_adjoint(wl, qf, qh, dv, rbar, v0, order, dtype):
    rows = R.Rows.from_workload(wl, DEV)
    qb = torch.empty(wl.n_cells, dtype=dtype, device=DEV)
    dvb = torch.zeros(wl.n_cells, dtype=dtype, device=DEV) if dv is not None else None
    v0b = torch.zeros(wl.n_rows, dtype=torch.float64, device=DEV)
    R.ram_step_adjoint(rows, dev(qf, dtype), None if qh is None else dev(qh, dtype),
                       None if dv is None else dev(dv, dtype), dev(rbar, dtype), qb,
                       dev(v0), wl.dt, order, dvb, v0b)
    torch.cuda.synchronize()
    return (qb.cpu().numpy().astype(np.float64),
            None if dvb is None else dvb.cpu().numpy().astype(np.float64),
            v0b.cpu().numpy())


def _inputs(wl, seed):
    rng = np.random.default_rng(seed)
    qf = wl.q0.reshape(-1).astype(np.float64)
    orows = oracle.Rows.from_workload(wl)
    qh = oracle.shift(orows, qf, wl.v0, wl.dt, wl.order)
    rbar = rng.standard_normal(wl.n_cells)
    return qf, qh, rbar


@pytest.mark.parametrize("order", [1, 3, 5])
@pytest.mark.parametrize("kind", ["polar_one_tile", "polar_tiles", "ragged"])
def test_step_adjoint_fp64(kind, order):
    wl = _cases()[kind](order)
    qf, qh, rbar = _inputs(wl, order)
    dv = wl.dv.reshape(-1)
    for mult in (1.0, -23.7):
        v0 = wl.v0 * mult
        got = _gpu_step_adjoint(wl, qf, qh, dv, rbar, v0, order, torch.float64)
        ref = _oracle_step_adjoint(wl, qf, qh, dv, rbar, v0, order)
        assert_parity(got[0], ref[0], 1e-12, CELL_F64, what=str(mult))
        assert_parity(got[1], ref[1], 1e-12, CELL_F64, what=str(mult))
        assert np.max(np.abs(got[2] - ref[2])) <= 1e-10 * np.max(np.abs(ref[2])), mult


@pytest.mark.parametrize("kind", ["polar_tiles", "ragged"])
def test_step_adjoint_without_residual(kind):
    wl = _cases()[kind](5)
    qf, _, rbar = _inputs(wl, 7)
    got = _gpu_step_adjoint(wl, qf, None, None, rbar, wl.v0, 5, torch.float64)
    ref = _oracle_step_adjoint(wl, qf, None, None, rbar, wl.v0, 5)
    assert_parity(got[0], ref[0], 1e-12, CELL_F64)
    assert np.max(np.abs(got[2] - ref[2])) <= 1e-10 * np.max(np.abs(ref[2]))


def test_step_adjoint_window_overflow():
    # 256 coarse cells then a 20x finer region: shifted by half the period, a
    # destination tile's source window exceeds the on-chip buffer.
    coarse = np.linspace(0.0, 0.5, 257)
    fine = np.linspace(0.5, 1.0, 256 * 20 + 1)[1:]
    e = np.concatenate([coarse, fine])
    n = len(e) - 1
    rng = np.random.default_rng(5)
    q = 1.0 + 0.2 * rng.standard_normal(n)
    dxmin = np.minimum(np.diff(e), np.roll(np.diff(e), 1))
    dv = 0.4 * dxmin * rng.uniform(-1, 1, n)
    for s in (-0.5, -0.37):
        wl = W.Workload("row", 1, n, np.array([0, n]), e, True, q[None, :], dv[None, :],
                        np.array([s]), 1.0, 5, 1)
        qh = oracle.shift(oracle.Rows.from_workload(wl), q, wl.v0, 1.0, 5)
        rbar = rng.standard_normal(n)
        got = _gpu_step_adjoint(wl, q, qh, dv, rbar, wl.v0, 5, torch.float64)
        ref = _oracle_step_adjoint(wl, q, qh, dv, rbar, wl.v0, 5)
        assert_parity(got[0], ref[0], 1e-12, CELL_F64, what=str(s))
        assert_parity(got[1], ref[1], 1e-12, CELL_F64, what=str(s))
        assert abs(got[2][0] - ref[2][0]) <= 1e-10 * abs(ref[2][0]), s


@pytest.mark.parametrize("kind", ["polar_tiles", "ragged", "uniform"])
def test_step_adjoint_fp32(kind):
    wl = _cases()[kind](5)
    qf, qh, rbar = _inputs(wl, 11)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    qf, qh, rbar, dv = f32(qf), f32(qh), f32(rbar), f32(wl.dv.reshape(-1))
    got = _gpu_step_adjoint(wl, qf, qh, dv, rbar, wl.v0, 5, torch.float32)
    ref = _oracle_step_adjoint(wl, qf, qh, dv, rbar, wl.v0, 5)
    for i in (0, 1):
        err, ec = assert_parity(got[i], ref[i], 1e-5, CELL_F32_ADJ, f"{kind} {i}")
        print(f"{kind} FP32 {'qbar' if i == 0 else 'dvbar'} rel-L1 {err:.2e}, max cell {ec:.2e}")
    # v0bar sums differences of the FP32 reconstruction slope between
    # neighbouring nodes: about 1e-4 relative rounding
    v0err = np.max(np.abs(got[2] - ref[2])) / np.max(np.abs(ref[2]))
    print(f"{kind} FP32 v0bar max rel {v0err:.2e}")
    assert v0err <= 1e-3


@pytest.mark.parametrize("residual", [True, False])
@pytest.mark.parametrize("order", [1, 3, 5])
def test_step_adjoint_fp32_uniform_stencil(order, residual):
    # every tile of a uniform mesh gathers through the transposed stencil;
    # rows shifted by under a cell, by tens of cells and by whole periods
    # either way
    wl = _uniform(order, n_rows=6, n=2600, seed=17 + order)
    n = wl.n_cols
    wl.v0[:] = np.array([0.37, -0.81, 23.6, -41.2, n + 5.3, -2 * n - 0.45]) / n
    qf, qh, rbar = _inputs(wl, 29)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    qf, rbar = f32(qf), f32(rbar)
    qh = f32(qh) if residual else None
    dv = f32(wl.dv.reshape(-1)) if residual else None
    got = _gpu_step_adjoint(wl, qf, qh, dv, rbar, wl.v0, order, torch.float32)
    ref = _oracle_step_adjoint(wl, qf, qh, dv, rbar, wl.v0, order)
    err = rel_l1(got[0], ref[0])
    print(f"order {order} residual {residual} FP32 qbar rel-L1 {err:.2e}")
    assert err <= 1e-5
    if residual:
        assert_parity(got[1], ref[1], 1e-5, CELL_F32_ADJ)
    v0err = np.max(np.abs(got[2] - ref[2])) / np.max(np.abs(ref[2]))
    print(f"order {order} residual {residual} FP32 v0bar max rel {v0err:.2e}")
    assert v0err <= 1e-3


def test_step_adjoint_fp32_long_row():
    # one long uniform row with a 10 % shorter cell: ~260 tiles, most through
    # the transposed stencil, those that see the cell through the scatter;
    # the atomics on the cells shared by neighbouring windows at scale
    n = (1 << 18) + 5
    rng = np.random.default_rng(41)
    e = W.uniform_edges(n, 0.0, 1.0).copy()
    e[100001:] -= 0.1 * (e[1] - e[0])
    e = e * (1.0 / e[-1])
    xc = 0.5 * (e[:-1] + e[1:])
    q = 1.0 + 0.3 * np.sin(2 * np.pi * xc)[None, :] + 0.05 * rng.standard_normal((2, n))
    dv = 0.2 * np.diff(e).min() * rng.uniform(-1, 1, (2, n))
    v0 = np.array([0.41, -2017.3]) / n
    wl = W.Workload("long", 2, n, np.arange(3) * n, e, True, q, dv, v0, 1.0, 5, 1)
    qf, qh, rbar = _inputs(wl, 43)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    qf, qh, rbar, dvf = f32(qf), f32(qh), f32(rbar), f32(dv.reshape(-1))
    got = _gpu_step_adjoint(wl, qf, qh, dvf, rbar, v0, 5, torch.float32)
    ref = _oracle_step_adjoint(wl, qf, qh, dvf, rbar, v0, 5)
    assert_parity(got[0], ref[0], 1e-5, CELL_F32_ADJ)
    assert_parity(got[1], ref[1], 1e-5, CELL_F32_ADJ)
    assert np.max(np.abs(got[2] - ref[2])) <= 1e-3 * np.max(np.abs(ref[2]))
