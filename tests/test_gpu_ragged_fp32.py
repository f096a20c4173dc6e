"""FP32 state on per-row (ragged) meshes against the FP64 oracle.

The compensated cumulative of paper §3.2 (Eq. mass_shift_algo, the sum term)
in the mixed-precision form: FP32 state and stencil weights, the window
cumulative in FP64, in two-sum FP32 or in plain FP32.  The oracle reads the
same FP32 input widened to FP64 (one step from the same start; the per-step
reading of the FP32 gate).

Bars, per row, in the Δx-weighted relative L1 of the error norm (§4.1,
Eq. e1, made relative):

* FP64 prefix, two-sum FP32 prefix, and RAM_SUM_DIRECT (which takes the FP64
  prefix on per-row meshes): <= 1e-6.
* Per cell, max |got - ref| / max |ref| <= 2e-5 (p = 1), 1e-4 (p = 3),
  2e-4 (p = 5).  Derivation: a destination cell up to 20x smaller than its
  source cell gets its mass as the difference of two partial integrals of
  that source cell (each up to 20x the result), each a sum of p + 1 terms
  with FP32 Lagrange weights.  On these random meshes (neighbouring cells up
  to 20x apart) the weights of a degree-p stencil are not O(1): their
  absolute sum grows to tens at p = 3 and about a hundred at p = 5, so the
  rounding of one partial integral reaches sum|w| x 2^-24 of a cell mass and
  the worst cell about 20 x sum|w| x 2^-24 x (a few): ~1e-6, ~2e-5, ~1e-4.
  The bars sit 2x above those and still 10x or more below what a wrong node,
  weight or whole-cell sum produces (>= 2e-3 of max |Q|).
* Plain FP32 prefix: the window cumulative of up to ~2000 cells carries an
  absolute rounding of about (window length) x 2^-24 of a cell mass in every
  difference, amplified up to 20x in the smallest cells: rel-L1 <= 1e-4 per
  row and per cell <= 2e-3 relative to max |ref|.  The test reports the
  measured figure beside the compensated ones.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2305_05362_amd import _lib as R
from paper_2305_05362_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

COMPENSATED = (("f64_prefix", R.RAM_SCAN_F64), ("twosum", R.RAM_SCAN_F32_TWOSUM),
               ("direct", R.RAM_SUM_DIRECT))
ROW_BAR = 1e-6
CELL_BAR = {1: 2e-5, 3: 1e-4, 5: 2e-4}
PLAIN_ROW_BAR = 1e-4
PLAIN_CELL_BAR = 2e-3


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def row_errors(wl, got, ref, rows=None):
    """Per row: Δx-weighted rel-L1 and max |got - ref| / max |ref|."""
    out = []
    for r in (range(wl.n_rows) if rows is None else rows):
        a, b = int(wl.row_ptr[r]), int(wl.row_ptr[r + 1])
        dx = np.diff(wl.row_edges(r))
        g, f = got[a:b], ref[a:b]
        rl1 = float(np.sum(np.abs(g - f) * dx) / np.sum(np.abs(f) * dx))
        cell = float(np.max(np.abs(g - f)) / np.max(np.abs(f)))
        out.append((r, rl1, cell))
    return out


def fp32_workload(wl):
    """The workload with Q0 and δv rounded to FP32 (kept as FP64 values)."""
    q = wl.q0.astype(np.float32).astype(np.float64)
    dv = None if wl.dv is None else wl.dv.astype(np.float32).astype(np.float64)
    return W.Workload(wl.name + "_f32", wl.n_rows, wl.n_cols, wl.row_ptr, wl.edges,
                      wl.edges_shared, q, dv, wl.v0, wl.dt, wl.order, wl.steps)


def gpu_fp32_step(wl, scan, order, with_dv, shift_only=False):
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0, torch.float32)
    if shift_only:
        qo = torch.empty_like(q)
        R.ram_shift(rows, q, qo, dev(wl.v0), wl.dt, order, scan)
        q = qo
    else:
        dv = dev(wl.dv, torch.float32) if with_dv else None
        R.ram_step(rows, q, dev(wl.v0), dv, wl.dt, order, 1, scan)
    torch.cuda.synchronize()
    return q.cpu().numpy().astype(np.float64)


def check(errs, row_bar, cell_bar, label):
    worst_row = max(errs, key=lambda e: e[1])
    worst_cell = max(errs, key=lambda e: e[2])
    print(f"{label}: worst row rel-L1 {worst_row[1]:.3e} (row {worst_row[0]}), "
          f"worst cell {worst_cell[2]:.3e} (row {worst_cell[0]})")
    assert worst_row[1] <= row_bar, (label, worst_row)
    assert worst_cell[2] <= cell_bar, (label, worst_cell)


@pytest.mark.parametrize("order", [1, 3, 5])
@pytest.mark.parametrize("mode", ["shift", "step"])
def test_small_ragged_fp32_vs_oracle(order, mode):
    # rows of 8 .. 2600 cells (one to three tiles, ragged tails), cell-size
    # ratio 20, shifts of -30 .. 30 mean cells; the step fuses the residual
    wl = fp32_workload(W.small_ragged(40, 8, 2600, seed=41, order=order))
    orows = oracle.Rows.from_workload(wl)
    if mode == "shift":
        ref = oracle.shift(orows, wl.q0, wl.v0, wl.dt, order)
    else:
        ref = oracle.step(orows, wl.q0, wl.v0, wl.dv, wl.dt, order, 1)
    for name, scan in COMPENSATED:
        got = gpu_fp32_step(wl, scan, order, True, shift_only=mode == "shift")
        check(row_errors(wl, got, ref), ROW_BAR, CELL_BAR[order], f"{mode} p={order} {name}")
    got = gpu_fp32_step(wl, R.RAM_SCAN_F32, order, True, shift_only=mode == "shift")
    check(row_errors(wl, got, ref), PLAIN_ROW_BAR, PLAIN_CELL_BAR, f"{mode} p={order} plain")


def test_ragged_fp32_window_overflow():
    # a per-row mesh whose coarse tiles land on a 20x finer half: the source
    # window exceeds the LDS capacity and the direct (global-memory) path runs
    coarse = np.linspace(0.0, 0.5, 1025)
    fine = np.linspace(0.5, 1.0, 1024 * 20 + 1)[1:]
    e1 = np.concatenate([coarse, fine])
    rng = np.random.default_rng(17)
    e2 = W.stretched_edges(3000, 20.0, rng)
    rows_e = [e1, e2]
    lens = np.array([len(e) - 1 for e in rows_e])
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    edges = np.concatenate(rows_e)
    q0 = np.concatenate([1.0 + 0.2 * rng.standard_normal(n) for n in lens])
    v0 = np.array([0.37, -41.3 / 3000])
    wl = fp32_workload(W.Workload("ovf", 2, 0, row_ptr, edges, False, q0, None, v0, 1.0,
                                  5, 1))
    ref = oracle.shift(oracle.Rows.from_workload(wl), wl.q0, wl.v0, wl.dt, 5)
    for name, scan in COMPENSATED:
        got = gpu_fp32_step(wl, scan, 5, False, shift_only=True)
        check(row_errors(wl, got, ref), ROW_BAR, CELL_BAR[5], f"overflow {name}")


@pytest.fixture(scope="module")
def cfg3_f32():
    return fp32_workload(W.cfg3())


def test_cfg3_full_size_fp32_sampled_rows(cfg3_f32):
    # the full 4096-row batch in one launch, as the bench times it; the oracle
    # recomputes sampled rows on their own (rows are independent)
    wl = cfg3_f32
    rng = np.random.default_rng(20230539)
    pick = sorted(set([0, 1, 2047, 4095]) | set(rng.integers(0, wl.n_rows, 12).tolist()))
    refs = {}
    for r in pick:
        a, b = int(wl.row_ptr[r]), int(wl.row_ptr[r + 1])
        refs[r] = oracle.shift(oracle.Rows.single(wl.row_edges(r)), wl.q0[a:b],
                               wl.v0[r:r + 1], wl.dt, 5)
    modes = COMPENSATED + (("plain", R.RAM_SCAN_F32),)
    for name, scan in modes:
        got = gpu_fp32_step(wl, scan, 5, False)
        full = np.zeros_like(got)
        for r in pick:
            full[int(wl.row_ptr[r]):int(wl.row_ptr[r + 1])] = refs[r]
        errs = row_errors(wl, got, full, pick)
        if name == "plain":
            check(errs, PLAIN_ROW_BAR, PLAIN_CELL_BAR, f"cfg3 {name}")
        else:
            check(errs, ROW_BAR, CELL_BAR[5], f"cfg3 {name}")
