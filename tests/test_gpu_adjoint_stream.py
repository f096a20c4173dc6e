"""The streaming step adjoint (FP32 state, shared mesh, rows of a multiple of
four cells: k_adjf_uni / k_adjf_gen on the shift's tile plan) against the
FP64 oracle's residual transpose followed by its shift transpose (Section 3,
Steps 1-3 and the residual step of Section 3.1, transposed), run on the same
FP32-rounded inputs; and the general shared-mesh adjoint (schedule 4) held to
the same bars on the same inputs.

Bars: those of test_gpu_step_adjoint.py's FP32 cases (rel-L1 1e-5, per cell
1e-4 of max |ref|, v0bar 1e-3 of its largest entry: v0bar sums differences of
the FP32 reconstruction slope between neighbouring nodes).  A node's weight
on the wrong window cell, a missed shared cell or a wrong face term is off by
far more.

Cases: the refined polar mesh (uniform-run tiles next to searching tiles)
with and without the residual and with and without v0bar, orders 1, 3 and 5,
shifts of a fraction of a cell up to whole periods either way; rows of 264
and 300 cells (windows that wrap the row: the gathering path); a coarse half
next to a 20x finer half (windows beyond the LDS: the gathering path); one
row of 2^18 + 8 cells with a shorter cell; and the 2048 x 16384 refined disk
on sampled rows.
"""
import numpy as np
import pytest
import torch

import oracle
from parity import CELL_F32_ADJ, assert_parity
from paper_2305_05362_amd import _lib as R
from paper_2305_05362_amd import workloads as W
from test_gpu_step_adjoint import _gpu_step_adjoint, _oracle_step_adjoint

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


@pytest.fixture
def ctx():
    c = R.context(0)
    c.set_schedule(0)
    yield c
    c.set_schedule(0)


def _inputs(wl, seed, residual=True):
    rng = np.random.default_rng(seed)
    qf = f32(wl.q0.reshape(-1))
    qh = f32(oracle.shift(oracle.Rows.from_workload(wl), qf, wl.v0, wl.dt, wl.order))
    rbar = f32(rng.standard_normal(wl.n_cells))
    dv = f32(wl.dv.reshape(-1)) if residual else None
    return qf, (qh if residual else None), dv, rbar


def _check(wl, got, ref, what, residual=True, v0=True):
    e0, c0 = assert_parity(got[0], ref[0], 1e-5, CELL_F32_ADJ, f"{what} qbar")
    msg = f"{what}: qbar rel-L1 {e0:.2e} cell {c0:.2e}"
    if residual:
        e1, c1 = assert_parity(got[1], ref[1], 1e-5, CELL_F32_ADJ, f"{what} dvbar")
        msg += f", dvbar {e1:.2e} cell {c1:.2e}"
    if v0:
        v0err = np.max(np.abs(got[2] - ref[2])) / np.max(np.abs(ref[2]))
        msg += f", v0bar max rel {v0err:.2e}"
        assert v0err <= 1e-3, what
    print(msg)


def _run(ctx, wl, inputs, order, sched, v0=True):
    qf, qh, dv, rbar = inputs
    ctx.set_schedule(sched)
    got = _gpu_step_adjoint(wl, qf, qh, dv, rbar, wl.v0, order, torch.float32)
    if not v0:
        got = (got[0], got[1], None)
    return got


@pytest.mark.parametrize("residual", [True, False])
@pytest.mark.parametrize("order", [1, 3, 5])
def test_stream_adjoint_polar(ctx, order, residual):
    wl = W.small_polar(12, 4096, order=order)
    n = wl.n_cols
    wl.v0[:] = wl.v0 * np.array([1.0, -1.0, 7.3, -11.9, 0.02, -0.05,
                                 n * 0.37, -n * 0.81, 1.0, -2.0, 3.0, -4.0])
    inputs = _inputs(wl, 3 + order, residual)
    ref = _oracle_step_adjoint(wl, inputs[0], inputs[1], inputs[2], inputs[3], wl.v0, order)
    for sched in (0, 4):
        got = _run(ctx, wl, inputs, order, sched)
        _check(wl, got, ref, f"p={order} res={residual} sched={sched}", residual)


def test_stream_adjoint_without_v0bar(ctx):
    # only qbar and dvbar asked for: the v0bar terms are skipped
    wl = W.small_polar(6, 2048, order=5)
    qf, qh, dv, rbar = _inputs(wl, 19)
    ref = _oracle_step_adjoint(wl, qf, qh, dv, rbar, wl.v0, 5)
    rows = R.Rows.from_workload(wl, DEV)
    qb = torch.empty(wl.n_cells, dtype=torch.float32, device=DEV)
    dvb = torch.zeros(wl.n_cells, dtype=torch.float32, device=DEV)
    t = lambda a: torch.as_tensor(a, dtype=torch.float32, device=DEV)
    R.ram_step_adjoint(rows, t(qf), t(qh), t(dv), t(rbar), qb,
                       torch.as_tensor(wl.v0, dtype=torch.float64, device=DEV), wl.dt, 5, dvb,
                       None)
    torch.cuda.synchronize()
    got = (qb.cpu().numpy().astype(np.float64), dvb.cpu().numpy().astype(np.float64), None)
    _check(wl, got, ref, "no v0bar", True, v0=False)


@pytest.mark.parametrize("n", [264, 300])
def test_stream_adjoint_short_rows(ctx, n):
    # a row barely longer than a tile: the last tile is short and the windows
    # of shifted tiles wrap the row
    rng = np.random.default_rng(n)
    e = W.stretched_edges(n, 8.0, rng)
    n_rows = 4
    q = 1.0 + 0.2 * rng.standard_normal((n_rows, n))
    dv = 0.3 * np.diff(e).min() * rng.uniform(-1, 1, (n_rows, n))
    v0 = np.array([0.3, -17.2, n + 0.6, -1.7 * n]) / n
    wl = W.Workload("short", n_rows, n, np.arange(n_rows + 1) * n, e, True, q, dv, v0,
                    1.0, 5, 1)
    inputs = _inputs(wl, 7)
    ref = _oracle_step_adjoint(wl, inputs[0], inputs[1], inputs[2], inputs[3], wl.v0, 5)
    for sched in (0, 4):
        _check(wl, _run(ctx, wl, inputs, 5, sched), ref, f"n={n} sched={sched}")


def test_stream_adjoint_window_overflow(ctx):
    # 256 coarse cells then a 20x finer region: shifted by half the period a
    # tile's window exceeds the LDS, and its cells are gathered
    coarse = np.linspace(0.0, 0.5, 257)
    fine = np.linspace(0.5, 1.0, 256 * 20 + 1)[1:]
    e = np.concatenate([coarse, fine])
    n = len(e) - 1
    rng = np.random.default_rng(5)
    q = 1.0 + 0.2 * rng.standard_normal((2, n))
    dxmin = np.minimum(np.diff(e), np.roll(np.diff(e), 1))
    dv = 0.4 * dxmin * rng.uniform(-1, 1, (2, n))
    wl = W.Workload("row", 2, n, np.arange(3) * n, e, True, q, dv, np.array([-0.5, -0.37]),
                    1.0, 5, 1)
    inputs = _inputs(wl, 9)
    ref = _oracle_step_adjoint(wl, inputs[0], inputs[1], inputs[2], inputs[3], wl.v0, 5)
    _check(wl, _run(ctx, wl, inputs, 5, 0), ref, "overflow")


def test_stream_adjoint_long_row(ctx):
    # one long uniform row with a 10 % shorter cell: ~1000 tiles, most in the
    # uniform run, those that see the cell searching; the atomics on the cells
    # shared by neighbouring windows at scale
    n = (1 << 18) + 8
    rng = np.random.default_rng(41)
    e = W.uniform_edges(n, 0.0, 1.0).copy()
    e[100001:] -= 0.1 * (e[1] - e[0])
    e = e * (1.0 / e[-1])
    xc = 0.5 * (e[:-1] + e[1:])
    q = 1.0 + 0.3 * np.sin(2 * np.pi * xc)[None, :] + 0.05 * rng.standard_normal((2, n))
    dv = 0.2 * np.diff(e).min() * rng.uniform(-1, 1, (2, n))
    v0 = np.array([0.41, -2017.3]) / n
    wl = W.Workload("long", 2, n, np.arange(3) * n, e, True, q, dv, v0, 1.0, 5, 1)
    inputs = _inputs(wl, 43)
    ref = _oracle_step_adjoint(wl, inputs[0], inputs[1], inputs[2], inputs[3], wl.v0, 5)
    _check(wl, _run(ctx, wl, inputs, 5, 0), ref, "long row")


def test_stream_adjoint_cfg5_sampled_rows(ctx):
    # the 2048 x 16384 refined disk at full size (the launch the bench times),
    # checked on sampled rows against the oracle row by row
    wl = W.cfg5()
    n = wl.n_cols
    rng = np.random.default_rng(20230542)
    qf = f32(wl.q0.reshape(-1))
    dv = f32(wl.dv.reshape(-1))
    rbar = f32(rng.standard_normal(wl.n_cells))
    pick = sorted(set([0, 1, 1023, 2047]) | set(rng.integers(0, wl.n_rows, 8).tolist()))
    one = oracle.Rows.single(wl.edges)
    qh = np.empty(wl.n_cells)
    # Q^{n+1/2} from the oracle on the sampled rows; the rest from the GPU
    # shift (FP32; only the sampled rows are checked, and rows are independent)
    rows = R.Rows.from_workload(wl, DEV)
    t32 = lambda a: torch.as_tensor(a, dtype=torch.float32, device=DEV)
    v0 = torch.as_tensor(wl.v0, dtype=torch.float64, device=DEV)
    half = torch.empty(wl.n_cells, dtype=torch.float32, device=DEV)
    R.ram_shift(rows, t32(qf), half, v0, wl.dt, 5, R.RAM_SUM_DIRECT)
    qh[:] = half.cpu().numpy()
    for r in pick:
        s = slice(r * n, (r + 1) * n)
        qh[s] = f32(oracle.shift(one, qf[s], wl.v0[r:r + 1], wl.dt, 5))
    qb = torch.empty(wl.n_cells, dtype=torch.float32, device=DEV)
    dvb = torch.zeros(wl.n_cells, dtype=torch.float32, device=DEV)
    v0b = torch.zeros(wl.n_rows, dtype=torch.float64, device=DEV)
    R.ram_step_adjoint(rows, t32(qf), t32(qh), t32(dv), t32(rbar), qb, v0, wl.dt, 5, dvb, v0b)
    torch.cuda.synchronize()
    gq, gd, gv = (qb.cpu().numpy().astype(np.float64), dvb.cpu().numpy().astype(np.float64),
                  v0b.cpu().numpy())
    rv = []
    for r in pick:
        s = slice(r * n, (r + 1) * n)
        rq, rdvb = oracle.residual_adjoint(one, qh[s], dv[s], rbar[s], wl.dt)
        rqb, rv0 = oracle.shift_adjoint(one, qf[s], rq, wl.v0[r:r + 1], wl.dt, 5)
        _check(wl, (gq[s], gd[s], None), (rqb, rdvb, None), f"cfg5 row {r}", v0=False)
        rv.append(rv0[0])
    # v0bar against the largest of the sampled rows' (the rows far from the
    # density bump hold a constant state, whose exact v0bar is zero)
    rv, gvp = np.array(rv), gv[pick]
    v0err = np.max(np.abs(gvp - rv)) / np.max(np.abs(rv))
    print(f"cfg5 v0bar max error / max |v0bar| {v0err:.2e}")
    assert v0err <= 1e-3


@pytest.mark.parametrize("kind,dtype,residual,n_steps", [
    ("polar", torch.float32, True, 5), ("polar", torch.float32, True, 4),
    ("polar", torch.float32, False, 3), ("polar", torch.float64, True, 3),
    ("ragged", torch.float32, True, 3)])
def test_adjoint_steps_equal_single_steps(ctx, kind, dtype, residual, n_steps):
    # ram_step_adjoint_steps over a recorded trajectory equals the same steps
    # walked back with ram_step_adjoint, bit for bit (one tile plan shared by
    # the steps; an odd count ends in the workspace and is copied back)
    wl = (W.small_polar(24, 4096, order=5) if kind == "polar"
          else W.small_ragged(24, 8, 3000, seed=51, order=5))
    rows = R.Rows.from_workload(wl, DEV)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=dtype, device=DEV)
    v0 = torch.as_tensor(wl.v0, dtype=torch.float64, device=DEV)
    dv = t(wl.dv) if residual else None
    traj = torch.empty((n_steps + 1, wl.n_cells), dtype=dtype, device=DEV)
    half = torch.empty((n_steps, wl.n_cells), dtype=dtype, device=DEV) if residual else None
    traj[0] = t(wl.q0)
    R.ram_step_record(rows, traj, half, v0, dv, wl.dt, 5, n_steps)
    g = t(np.random.default_rng(3).standard_normal(wl.n_cells))
    # one step at a time
    qa, qb = g.clone(), torch.empty_like(g)
    dva = torch.zeros_like(dv) if residual else None
    v0a = torch.zeros_like(v0)
    for k in range(n_steps - 1, -1, -1):
        R.ram_step_adjoint(rows, traj[k], half[k] if residual else None, dv, qa, qb, v0,
                           wl.dt, 5, dva, v0a)
        qa, qb = qb, qa
    # all at once
    q = g.clone()
    work = torch.full_like(g, float("nan"))
    dvb = torch.zeros_like(dv) if residual else None
    v0b = torch.zeros_like(v0)
    R.ram_step_adjoint_steps(rows, traj, half, dv, q, work, v0, wl.dt, 5, n_steps, dvb, v0b)
    torch.cuda.synchronize()
    assert torch.equal(q, qa)
    if residual:
        assert torch.equal(dvb, dva)
    assert torch.equal(v0b, v0a)
    assert float(q.abs().max()) > 0.0 and float(v0b.abs().max()) > 0.0
