"""The streaming shift on per-row meshes: FP32 state, no residual velocity,
calls of at least four steps at the default schedule (k_plan_rag once per
call, then k_step_rag a step), against the FP64 oracle run for the same
steps from the same FP32-rounded start (paper §3, Steps 1-3; Eq.
mass_shift_algo with each cumulative mode).

Bars: the one-step bars of test_gpu_ragged_fp32.py (derived there from the
FP32 rounding of the partial integrals on ratio-20 random meshes), times the
number of steps: each step adds its own rounding, and over four steps the
growth of the order-5 shift on these meshes stays small.  A node planned into
the wrong cell, a wrong weight or a wrong whole-cell sum is off by at least
2e-3 of max |Q| in one step, above every bar here.

Cases: ragged rows of 8 to 2600 cells (one to eleven tiles, rows shorter
than a tile whose window wraps the row more than once, shifts of up to 30
mean cells either way), orders 1, 3 and 5; rows whose coarse half lands on a
20x finer half (windows beyond the LDS: the direct path); uniform rows with
a mesh each; the full cfg3 batch (4096 rows of 64 to 8192 cells) on sampled
rows; and the general per-row kernel (schedule 4) on the same inputs, held
to the same bars.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2305_05362_amd import _lib as R
from paper_2305_05362_amd import workloads as W
from test_gpu_ragged_fp32 import (CELL_BAR, PLAIN_CELL_BAR, PLAIN_ROW_BAR, ROW_BAR,
                                  check, fp32_workload, row_errors)

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
STEPS = 4
MODES = (("f64_prefix", R.RAM_SCAN_F64), ("twosum", R.RAM_SCAN_F32_TWOSUM),
         ("direct", R.RAM_SUM_DIRECT), ("plain", R.RAM_SCAN_F32))


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.fixture
def ctx():
    c = R.context(0)
    c.set_schedule(0)
    yield c
    c.set_schedule(0)


def run(ctx, wl, scan, order, steps=STEPS):
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0.reshape(-1), torch.float32)
    ctx.ram_step(rows, q, dev(wl.v0), None, wl.dt, order, steps, scan)
    torch.cuda.synchronize()
    return q.cpu().numpy().astype(np.float64)


def check_modes(ctx, wl, ref, order, label, rows=None):
    for name, scan in MODES:
        got = run(ctx, wl, scan, order)
        if rows is not None:
            full = np.zeros_like(got)
            for r in rows:
                full[int(wl.row_ptr[r]):int(wl.row_ptr[r + 1])] = ref[r]
            errs = row_errors(wl, got, full, rows)
        else:
            errs = row_errors(wl, got, ref)
        if name == "plain":
            check(errs, STEPS * PLAIN_ROW_BAR, STEPS * PLAIN_CELL_BAR, f"{label} {name}")
        else:
            check(errs, STEPS * ROW_BAR, STEPS * CELL_BAR[order], f"{label} {name}")


@pytest.mark.parametrize("order", [1, 3, 5])
def test_ragged_stream_vs_oracle(ctx, order):
    wl = fp32_workload(W.small_ragged(40, 8, 2600, seed=41, order=order, with_dv=False))
    ref = oracle.step(oracle.Rows.from_workload(wl), wl.q0, wl.v0, None, wl.dt, order, STEPS)
    check_modes(ctx, wl, ref, order, f"stream p={order}")


def test_ragged_general_kernel_same_bars(ctx):
    # schedule 4 keeps the general per-row kernel (a search a node a step)
    wl = fp32_workload(W.small_ragged(40, 8, 2600, seed=41, order=5, with_dv=False))
    ref = oracle.step(oracle.Rows.from_workload(wl), wl.q0, wl.v0, None, wl.dt, 5, STEPS)
    ctx.set_schedule(4)
    check_modes(ctx, wl, ref, 5, "general p=5")


def test_ragged_stream_window_overflow(ctx):
    # the first row's coarse tiles land on its 20x finer half (windows beyond
    # the LDS: those tiles sum from global memory), the second is random
    coarse = np.linspace(0.0, 0.5, 1025)
    fine = np.linspace(0.5, 1.0, 1024 * 20 + 1)[1:]
    e1 = np.concatenate([coarse, fine])
    rng = np.random.default_rng(17)
    e2 = W.stretched_edges(3000, 20.0, rng)
    rows_e = [e1, e2]
    lens = np.array([len(e) - 1 for e in rows_e])
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    q0 = np.concatenate([1.0 + 0.2 * rng.standard_normal(n) for n in lens])
    v0 = np.array([0.37, -41.3 / 3000])
    wl = fp32_workload(W.Workload("ovf", 2, 0, row_ptr, np.concatenate(rows_e), False, q0,
                                  None, v0, 1.0, 5, STEPS))
    ref = oracle.step(oracle.Rows.from_workload(wl), wl.q0, wl.v0, None, wl.dt, 5, STEPS)
    check_modes(ctx, wl, ref, 5, "overflow")


def test_uniform_rows_own_meshes(ctx):
    # rows of one length, each with its own random mesh (not shared)
    rng = np.random.default_rng(23)
    n_rows, n = 6, 3000
    edges = np.concatenate([W.stretched_edges(n, 20.0, rng) for _ in range(n_rows)])
    q0 = 1.0 + 0.2 * rng.standard_normal(n_rows * n)
    v0 = rng.uniform(-25.0, 25.0, n_rows) / n
    wl = fp32_workload(W.Workload("rows", n_rows, n, np.arange(n_rows + 1) * n, edges,
                                  False, q0, None, v0, 1.0, 5, STEPS))
    ref = oracle.step(oracle.Rows.from_workload(wl), wl.q0, wl.v0, None, wl.dt, 5, STEPS)
    check_modes(ctx, wl, ref, 5, "own meshes")


def test_cfg3_full_size_stream_sampled_rows(ctx):
    wl = fp32_workload(W.cfg3())
    rng = np.random.default_rng(20230541)
    pick = sorted(set([0, 1, 2047, 4095]) | set(rng.integers(0, wl.n_rows, 12).tolist()))
    refs = {}
    for r in pick:
        a, b = int(wl.row_ptr[r]), int(wl.row_ptr[r + 1])
        refs[r] = oracle.step(oracle.Rows.single(wl.row_edges(r)), wl.q0[a:b],
                              wl.v0[r:r + 1], None, wl.dt, 5, STEPS)
    check_modes(ctx, wl, refs, 5, "cfg3", rows=pick)
