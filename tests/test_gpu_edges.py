"""Edge cases of the C ABI against the FP64 oracle.

* zero shift (dt = 0, or v0 = 0 on some rows): the step is the identity up to
  the rounding of Q dx / dx (relative L1 <= 1e-15);
* negative dt (the profile moves the other way), large |v0 dt| on short rows;
* zero steps: the state is untouched, bit for bit;
* one very long row (2^20 cells, about a thousand tiles) and many very short
  ragged rows (the stencil's minimum, p + 1 cells, and a few more);
* the FP64 bar is 1e-12 relative L1 throughout, FP32 1e-6 for one step.
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


@pytest.mark.parametrize("scan", [R.RAM_SCAN_F64, R.RAM_SUM_DIRECT])
def test_zero_shift_is_identity(scan):
    wl = W.small_polar(4, 3000)
    rows = R.Rows.from_workload(wl, DEV)
    q0 = dev(wl.q0)
    for dt, v0 in ((0.0, wl.v0), (wl.dt, np.where(np.arange(wl.n_rows) % 2 == 0, 0.0, wl.v0))):
        q = q0.clone()
        dv = dev(np.zeros_like(wl.dv))
        R.ram_step(rows, q, dev(v0), dv, dt, 5, 3, scan)
        torch.cuda.synchronize()
        got = q.cpu().numpy().reshape(wl.n_rows, -1)
        ref = oracle.step(oracle.Rows.from_workload(wl), wl.q0, v0, None, dt, 5, 3)
        ref = ref.reshape(wl.n_rows, -1)
        assert_parity(got.reshape(-1), ref.reshape(-1), 1e-12, CELL_F64)
        still = v0 == 0.0 if dt != 0.0 else np.ones(wl.n_rows, bool)
        assert rel_l1(got[still].reshape(-1), wl.q0.reshape(wl.n_rows, -1)[still].reshape(-1)) \
            <= 1e-15


@pytest.mark.parametrize("scan", [R.RAM_SCAN_F64, R.RAM_SUM_DIRECT])
def test_negative_dt_and_short_rows(scan):
    wl = W.small_ragged(40, 6, 40, seed=17, order=5)
    rows = R.Rows.from_workload(wl, DEV)
    orows = oracle.Rows.from_workload(wl)
    # with the residual, dt reversed (half the Courant-limited step)
    q = dev(wl.q0)
    R.ram_step(rows, q, dev(wl.v0), dev(wl.dv), -0.5 * wl.dt, 5, 2, scan)
    torch.cuda.synchronize()
    ref = oracle.step(orows, wl.q0, wl.v0, wl.dv, -0.5 * wl.dt, 5, 2)
    assert_parity(q.cpu().numpy(), ref, 1e-12, CELL_F64)
    # shift only, shifts of many periods either way on rows of 6..40 cells
    for mult in (-37.5, 211.0):
        q = dev(wl.q0)
        R.ram_step(rows, q, dev(wl.v0 * mult), None, -wl.dt, 5, 2, scan)
        torch.cuda.synchronize()
        ref = oracle.step(orows, wl.q0, wl.v0 * mult, None, -wl.dt, 5, 2)
        assert_parity(q.cpu().numpy(), ref, 1e-12, CELL_F64, what=str(mult))


def test_zero_steps_leave_state_untouched():
    wl = W.small_polar(3, 2000)
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0)
    before = q.clone()
    R.ram_step(rows, q, dev(wl.v0), dev(wl.dv), wl.dt, 5, 0)
    torch.cuda.synchronize()
    assert torch.equal(q, before)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_one_long_row(dtype):
    n = 1 << 20
    rng = np.random.default_rng(23)
    e = W.stretched_edges(n, 20.0, rng, 0.0, 1.0)
    q = 1.0 + 0.3 * np.sin(2 * np.pi * 7 * 0.5 * (e[:-1] + e[1:])) + 0.01 * rng.standard_normal(n)
    dxm = np.minimum(np.diff(e), np.roll(np.diff(e), 1))
    dv = 0.3 * dxm * rng.uniform(-1, 1, n)
    wl = W.Workload("long", 1, n, np.array([0, n]), e, True, q[None, :], dv[None, :],
                    np.array([123.7 / n]), 1.0, 5, 1)
    qq = q.astype(np.float32).astype(np.float64) if dtype == torch.float32 else q
    dvv = dv.astype(np.float32).astype(np.float64) if dtype == torch.float32 else dv
    rows = R.Rows.from_workload(wl, DEV)
    for scan in ((R.RAM_SCAN_F64, R.RAM_SUM_DIRECT) if dtype == torch.float64 else
                 (R.RAM_SCAN_F32_TWOSUM, R.RAM_SUM_DIRECT)):
        qd = dev(qq, dtype)
        R.ram_step(rows, qd, dev(wl.v0), dev(dvv, dtype), 1.0, 5, 1, scan)
        torch.cuda.synchronize()
        ref = oracle.step(oracle.Rows.from_workload(wl), qq, wl.v0, dvv, 1.0, 5, 1)
        err = rel_l1(qd.cpu().numpy().astype(np.float64), ref)
        assert err <= (1e-12 if dtype == torch.float64 else 1e-6), (scan, err)


def test_many_tiny_ragged_rows():
    wl = W.small_ragged(20000, 6, 12, seed=29, order=5)
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0)
    R.ram_step(rows, q, dev(wl.v0), dev(wl.dv), wl.dt, 5, 3)
    torch.cuda.synchronize()
    ref = oracle.step(oracle.Rows.from_workload(wl), wl.q0, wl.v0, wl.dv, wl.dt, 5, 3)
    assert_parity(q.cpu().numpy(), ref, 1e-12, CELL_F64)
    # and the adjoint through the per-row path
    rng = np.random.default_rng(3)
    rbar = rng.standard_normal(wl.n_cells)
    orows = oracle.Rows.from_workload(wl)
    qh = oracle.shift(orows, wl.q0, wl.v0, wl.dt, 5)
    qb = torch.empty(wl.n_cells, dtype=torch.float64, device=DEV)
    dvb = torch.zeros(wl.n_cells, dtype=torch.float64, device=DEV)
    v0b = torch.zeros(wl.n_rows, dtype=torch.float64, device=DEV)
    R.ram_step_adjoint(rows, dev(wl.q0), dev(qh), dev(wl.dv), dev(rbar), qb, dev(wl.v0),
                       wl.dt, 5, dvb, v0b)
    torch.cuda.synchronize()
    r1, dvr = oracle.residual_adjoint(orows, qh, wl.dv, rbar, wl.dt)
    r0, v0r = oracle.shift_adjoint(orows, wl.q0, r1, wl.v0, wl.dt, 5)
    assert_parity(qb.cpu().numpy(), r0, 1e-12, CELL_F64)
    assert_parity(dvb.cpu().numpy(), dvr, 1e-12, CELL_F64)
    assert np.max(np.abs(v0b.cpu().numpy() - v0r)) <= 1e-10 * np.max(np.abs(v0r))
