"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: FP64 <= 1e-12 relative L1; FP32 state with compensated or FP64 prefix
sums, or direct sums, <= 1e-6 relative L1 for one step from the same FP32
input (the oracle reads it widened to FP64); integer work (the exact-permutation case) bitwise.
Full-size workloads are checked on sampled rows, which the oracle can compute
on their own because rows are independent.
"""
import numpy as np
import pytest
import torch

import oracle
from parity import CELL_F32, CELL_F32_ADJ, CELL_F64, assert_parity, max_cell
from paper_2305_05362_amd import _lib as R
from paper_2305_05362_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def rel_l1(a, b):
    return float(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))


def _one_row_workload(edges, q, v0, dt=1.0, dv=None):
    n = len(q)
    return W.Workload("row", 1, n, np.array([0, n]), np.asarray(edges, float), True,
                      np.asarray(q, float)[None, :], None if dv is None else np.asarray(dv)[None, :],
                      np.array([v0], float), dt, 5, 1)


def gpu_shift(wl, q, order, dtype=torch.float64, scan=R.RAM_SCAN_F64, v0=None, dt=None):
    rows = R.Rows.from_workload(wl, DEV)
    qi = dev(np.asarray(q).reshape(-1), dtype)
    qo = torch.empty_like(qi)
    v = dev(wl.v0 if v0 is None else v0)
    R.ram_shift(rows, qi, qo, v, wl.dt if dt is None else dt, order, scan)
    torch.cuda.synchronize()
    return qo.cpu().numpy().astype(np.float64)


def oracle_shift(wl, q, order, v0=None, dt=None):
    return oracle.shift(oracle.Rows.from_workload(wl), np.asarray(q, float).reshape(-1),
                        wl.v0 if v0 is None else v0, wl.dt if dt is None else dt, order)


# --------------------------------------------------------------------------
# bulk shift
# --------------------------------------------------------------------------

@pytest.mark.parametrize("order", [1, 3, 5])
def test_shift_polar_fp64(order):
    wl = W.small_polar(8, 700, order=order)
    for mult in (1.0, 37.3, -5.1):
        v0 = wl.v0 * mult
        got = gpu_shift(wl, wl.q0, order, v0=v0)
        ref = oracle_shift(wl, wl.q0, order, v0=v0)
        assert_parity(got, ref, 1e-12, CELL_F64, what=str((mult, rel_l1(got, ref))))


@pytest.mark.parametrize("order", [1, 3, 5])
def test_shift_ragged_fp64(order):
    wl = W.small_ragged(40, 6, 900, seed=11, order=order)
    got = gpu_shift(wl, wl.q0, order)
    ref = oracle_shift(wl, wl.q0, order)
    assert_parity(got, ref, 1e-12, CELL_F64)
    # per row too (short rows must not be swamped by long ones)
    for r in range(wl.n_rows):
        a, b = wl.row_ptr[r], wl.row_ptr[r + 1]
        assert_parity(got[a:b], ref[a:b], 1e-12, CELL_F64, what=str(r))


@pytest.mark.parametrize("n", [6, 7, 255, 256, 257, 513, 1000])
def test_shift_row_lengths_and_tails(n):
    rng = np.random.default_rng(n)
    e = W.stretched_edges(n, 20.0, rng, -1.0, 3.0)
    q = 1.0 + rng.standard_normal(n)
    wl = _one_row_workload(e, q, 0.0)
    for s in (0.0, 0.31, -2.7, 123.456):
        got = gpu_shift(wl, q, 5, v0=np.array([s]), dt=1.0)
        ref = oracle_shift(wl, q, 5, v0=np.array([s]), dt=1.0)
        assert_parity(got, ref, 1e-12, CELL_F64, what=str((n, s)))


def test_shift_window_overflow_direct_path():
    # coarse destination tiles landing on a 20x finer region: the source window
    # of a 256-cell tile exceeds the LDS capacity and takes the direct path.
    coarse = np.linspace(0.0, 0.5, 257)
    fine = np.linspace(0.5, 1.0, 256 * 20 + 1)[1:]
    e = np.concatenate([coarse, fine])
    n = len(e) - 1
    rng = np.random.default_rng(5)
    q = 1.0 + 0.2 * rng.standard_normal(n)
    wl = _one_row_workload(e, q, 0.0)
    for s in (-0.5, -0.37):
        got = gpu_shift(wl, q, 5, v0=np.array([s]), dt=1.0)
        ref = oracle_shift(wl, q, 5, v0=np.array([s]), dt=1.0)
        assert_parity(got, ref, 1e-12, CELL_F64)


@pytest.mark.parametrize("order", [1, 3, 5])
def test_integer_shift_bitwise(order):
    wl = W.cfg1()
    q = wl.q0.reshape(-1)
    for m in (10, -3, 263):
        got = gpu_shift(wl, q, order, v0=np.array([m / 256.0]), dt=1.0)
        assert np.array_equal(got, np.roll(q, m)), m


def test_shift_fp32_scans():
    wl = W.small_polar(16, 4096, order=5)
    q32 = wl.q0.astype(np.float32)
    ref = oracle_shift(wl, q32.astype(np.float64), 5)
    errs = {}
    for name, scan in (("f64", R.RAM_SCAN_F64), ("twosum", R.RAM_SCAN_F32_TWOSUM),
                       ("f32", R.RAM_SCAN_F32), ("direct", R.RAM_SUM_DIRECT)):
        got = gpu_shift(wl, q32, 5, torch.float32, scan)
        errs[name] = (rel_l1(got, ref), max_cell(got, ref))
    print("one-step (rel-L1, max cell) by scan precision:", errs)
    for name in ("f64", "twosum", "direct"):
        assert errs[name][0] <= 1e-6 and errs[name][1] <= CELL_F32, (name, errs[name])
    # the plain FP32 window prefix: window-long cumulative rounding (the
    # compensated modes exist to remove it), held to 1e-4 rel-L1
    assert errs["f32"][0] <= 1e-4, errs["f32"]


@pytest.mark.parametrize("order", [1, 3, 5])
@pytest.mark.parametrize("kind", ["polar_one_tile", "polar_tiles", "ragged", "overflow"])
def test_direct_sums_fp64(kind, order):
    # the direct-sum evaluation (no prefix) against the oracle: shift alone
    # and fused steps, FP64, on one- and several-tile rows, per-row meshes
    # (which take the FP64 prefix) and a window wider than the LDS buffer
    if kind == "overflow":
        coarse = np.linspace(0.0, 0.5, 257)
        fine = np.linspace(0.5, 1.0, 256 * 20 + 1)[1:]
        e = np.concatenate([coarse, fine])
        n = len(e) - 1
        rng = np.random.default_rng(order)
        q = 1.0 + 0.2 * rng.standard_normal(n)
        dxm = np.minimum(np.diff(e), np.roll(np.diff(e), 1))
        wl = W.Workload("ovf", 1, n, np.array([0, n]), e, True, q[None, :],
                        (0.4 * dxm * rng.uniform(-1, 1, n))[None, :], np.array([-0.37]),
                        1.0, order, 1)
    elif kind == "ragged":
        wl = W.small_ragged(12, 6, 2600, seed=31, order=order)
    else:
        wl = W.small_polar(6, 800, order=order) if kind == "polar_one_tile" else \
            W.small_polar(3, 3500, order=order)
    got = gpu_shift(wl, wl.q0, order, scan=R.RAM_SUM_DIRECT)
    assert_parity(got, oracle_shift(wl, wl.q0, order), 1e-12, CELL_F64)
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0.reshape(-1))
    R.ram_step(rows, q, dev(wl.v0), dev(wl.dv.reshape(-1)), wl.dt, order, 3, R.RAM_SUM_DIRECT)
    torch.cuda.synchronize()
    ref = oracle.step(oracle.Rows.from_workload(wl), wl.q0, wl.v0, wl.dv, wl.dt, order, 3)
    assert_parity(q.cpu().numpy(), ref, 1e-12, CELL_F64)


# --------------------------------------------------------------------------
# residual and step
# --------------------------------------------------------------------------

def gpu_residual(wl, q, dtype=torch.float64):
    rows = R.Rows.from_workload(wl, DEV)
    qi = dev(np.asarray(q).reshape(-1), dtype)
    qo = torch.empty_like(qi)
    R.ram_residual(rows, qi, qo, dev(wl.dv.reshape(-1), dtype), wl.dt)
    torch.cuda.synchronize()
    return qo.cpu().numpy().astype(np.float64)


def test_residual_polar_fp64():
    wl = W.small_polar(8, 700)
    got = gpu_residual(wl, wl.q0)
    ref = oracle.residual(oracle.Rows.from_workload(wl), wl.q0, wl.dv, wl.dt)
    assert_parity(got, ref, 1e-12, CELL_F64)


def test_residual_ragged_fp64():
    wl = W.small_ragged(30, 3, 800, seed=2)
    got = gpu_residual(wl, wl.q0)
    ref = oracle.residual(oracle.Rows.from_workload(wl), wl.q0, wl.dv, wl.dt)
    assert_parity(got, ref, 1e-12, CELL_F64)


def test_residual_fp32():
    wl = W.small_polar(8, 1000)
    q32 = wl.q0.astype(np.float32)
    dv32 = wl.dv.astype(np.float32)
    wl32 = W.Workload(wl.name, wl.n_rows, wl.n_cols, wl.row_ptr, wl.edges, True,
                      q32.astype(np.float64), dv32.astype(np.float64), wl.v0, wl.dt, 5, 1)
    got = gpu_residual(wl32, q32, torch.float32)
    ref = oracle.residual(oracle.Rows.from_workload(wl32), wl32.q0, wl32.dv, wl.dt)
    assert_parity(got, ref, 1e-6, CELL_F32)


def test_step_cfg1_fp64():
    wl = W.cfg1()
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0.reshape(-1))
    R.ram_step(rows, q, dev(wl.v0), None, wl.dt, 5, wl.steps)
    torch.cuda.synchronize()
    got = q.cpu().numpy()
    ref = oracle.step(oracle.Rows.from_workload(wl), wl.q0, wl.v0, None, wl.dt, 5, wl.steps)
    assert_parity(got, ref, 1e-12, CELL_F64)
    # and both sit within the order-5 truncation error of the exact roll
    assert rel_l1(got, np.roll(wl.q0.reshape(-1), 6)) < 1e-10


@pytest.mark.parametrize("steps", [1, 2, 7])
def test_step_polar_with_residual(steps):
    wl = W.small_polar(6, 900)
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0.reshape(-1))
    R.ram_step(rows, q, dev(wl.v0), dev(wl.dv.reshape(-1)), wl.dt, 5, steps)
    torch.cuda.synchronize()
    ref = oracle.step(oracle.Rows.from_workload(wl), wl.q0, wl.v0, wl.dv, wl.dt, 5, steps)
    assert_parity(q.cpu().numpy(), ref, 1e-12, CELL_F64)


def test_step_ragged_shift_only_odd_steps():
    wl = W.small_ragged(20, 8, 600, seed=4, with_dv=False)
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0)
    R.ram_step(rows, q, dev(wl.v0), None, wl.dt, 3, 5)
    torch.cuda.synchronize()
    ref = oracle.step(oracle.Rows.from_workload(wl), wl.q0, wl.v0, None, wl.dt, 3, 5)
    assert_parity(q.cpu().numpy(), ref, 1e-12, CELL_F64)


# --------------------------------------------------------------------------
# full-size workloads on sampled rows
# --------------------------------------------------------------------------

def _sample_rows(wl, rows):
    """The sub-batch of the given rows (shared mesh) for the oracle."""
    q = wl.q0.reshape(wl.n_rows, -1)[rows]
    dv = None if wl.dv is None else wl.dv.reshape(wl.n_rows, -1)[rows]
    n = wl.n_cols
    return W.Workload("sample", len(rows), n, np.arange(len(rows) + 1) * n, wl.edges,
                      True, q, dv, wl.v0[rows], wl.dt, wl.order, wl.steps)


def test_cfg2_full_size_sampled_rows():
    wl = W.cfg2(5)
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0.reshape(-1))
    R.ram_step(rows, q, dev(wl.v0), dev(wl.dv.reshape(-1)), wl.dt, 5, wl.steps)
    torch.cuda.synchronize()
    got = q.cpu().numpy().reshape(wl.n_rows, -1)
    pick = np.array([0, 1, 77, 255, 256, 400, 510, 511])
    sw = _sample_rows(wl, pick)
    ref = oracle.step(oracle.Rows.from_workload(sw), sw.q0, sw.v0, sw.dv, sw.dt, 5, wl.steps)
    assert_parity(got[pick].reshape(-1), ref, 1e-12, CELL_F64)


def test_cfg5_full_size_sampled_rows():
    wl = W.cfg5()
    rows = R.Rows.from_workload(wl, DEV)
    pick = np.array([0, 3, 1024, 2047])
    sw = _sample_rows(wl, pick)
    orows = oracle.Rows.from_workload(sw)
    # FP64, 3 steps
    q = dev(wl.q0.reshape(-1))
    R.ram_step(rows, q, dev(wl.v0), dev(wl.dv.reshape(-1)), wl.dt, 5, 3)
    torch.cuda.synchronize()
    got = q.cpu().numpy().reshape(wl.n_rows, -1)[pick].reshape(-1)
    ref = oracle.step(orows, sw.q0, sw.v0, sw.dv, sw.dt, 5, 3)
    assert_parity(got, ref, 1e-12, CELL_F64)
    # FP32 state, compensated scan, one step from the same FP32 input
    q32 = wl.q0.astype(np.float32)
    dv32 = wl.dv.astype(np.float32)
    q = dev(q32.reshape(-1), torch.float32)
    ref = oracle.step(orows, q32.reshape(wl.n_rows, -1)[pick].astype(np.float64), sw.v0,
                      dv32.reshape(wl.n_rows, -1)[pick].astype(np.float64), sw.dt, 5, 1)
    for scan in (R.RAM_SCAN_F32_TWOSUM, R.RAM_SUM_DIRECT):
        q = dev(q32.reshape(-1), torch.float32)
        R.ram_step(rows, q, dev(wl.v0), dev(dv32.reshape(-1), torch.float32), wl.dt, 5, 1,
                   scan)
        torch.cuda.synchronize()
        got = q.cpu().numpy().astype(np.float64).reshape(wl.n_rows, -1)[pick].reshape(-1)
        assert_parity(got, ref, 1e-6, CELL_F32, what=str(scan))


def test_stretched_disk_full_size_sampled_rows():
    # the disk on a mesh of random cell sizes: every tile locates its nodes
    # (no uniform-run stencil), at the full size in the default schedule
    wl = W.stretched_disk()
    rows = R.Rows.from_workload(wl, DEV)
    R.context(0).set_schedule(0)
    paths = R.context(0).ram_step_tile_paths(rows, dev(wl.v0), wl.dt, 5, True).cpu().numpy()
    assert (paths == R.RAM_TILE_UNIFORM).sum() == 0 and (paths == R.RAM_TILE_WINDOW).sum() > 0
    pick = np.array([0, 5, 1024, 2047])
    sw = _sample_rows(wl, pick)
    orows = oracle.Rows.from_workload(sw)
    q = dev(wl.q0.reshape(-1))
    R.ram_step(rows, q, dev(wl.v0), dev(wl.dv.reshape(-1)), wl.dt, 5, 2)
    torch.cuda.synchronize()
    got = q.cpu().numpy().reshape(wl.n_rows, -1)[pick].reshape(-1)
    ref = oracle.step(orows, sw.q0, sw.v0, sw.dv, sw.dt, 5, 2)
    assert_parity(got, ref, 1e-12, CELL_F64, what="FP64")
    q32 = wl.q0.astype(np.float32)
    dv32 = wl.dv.astype(np.float32)
    ref = oracle.step(orows, q32.reshape(wl.n_rows, -1)[pick].astype(np.float64), sw.v0,
                      dv32.reshape(wl.n_rows, -1)[pick].astype(np.float64), sw.dt, 5, 1)
    for scan in (R.RAM_SUM_DIRECT, R.RAM_SCAN_F32_TWOSUM):
        q = dev(q32.reshape(-1), torch.float32)
        R.ram_step(rows, q, dev(wl.v0), dev(dv32.reshape(-1), torch.float32), wl.dt, 5, 1,
                   scan)
        torch.cuda.synchronize()
        got = q.cpu().numpy().astype(np.float64).reshape(wl.n_rows, -1)[pick].reshape(-1)
        e1, ec = assert_parity(got, ref, 1e-6, CELL_F32, what=str(scan))
        print(f"stretched disk FP32 scan {scan}: rel-L1 {e1:.2e}, max cell {ec:.2e}")


def test_cfg3_full_size_sampled_rows():
    wl = W.cfg3()
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0)
    R.ram_step(rows, q, dev(wl.v0), None, wl.dt, 5, 2)
    torch.cuda.synchronize()
    got = q.cpu().numpy()
    orows = oracle.Rows.from_workload(wl)
    for r in (0, 1, 2047, 4095):
        a, b = wl.row_ptr[r], wl.row_ptr[r + 1]
        e = wl.row_edges(r)
        ref = oracle.step(oracle.Rows.single(e), wl.q0[a:b], wl.v0[r:r + 1], None, wl.dt, 5, 2)
        assert_parity(got[a:b], ref, 1e-12, CELL_F64, what=str(r))
    del orows


# --------------------------------------------------------------------------
# adjoints
# --------------------------------------------------------------------------

@pytest.mark.parametrize("order", [1, 3, 5])
@pytest.mark.parametrize("kind", ["polar", "ragged"])
def test_shift_adjoint_fp64(order, kind):
    wl = W.small_polar(6, 800, order=order) if kind == "polar" else \
        W.small_ragged(25, 6, 700, seed=9, order=order)
    rng = np.random.default_rng(order)
    rbar = rng.standard_normal(wl.n_cells)
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0.reshape(-1))
    qb = torch.empty_like(q)
    v0b = torch.zeros(wl.n_rows, dtype=torch.float64, device=DEV)
    for mult in (1.0, -23.7):
        v0 = wl.v0 * mult
        v0b.zero_()
        R.ram_shift_adjoint(rows, q, dev(rbar), qb, dev(v0), wl.dt, order, v0b)
        torch.cuda.synchronize()
        ref_qb, ref_v0b = oracle.shift_adjoint(oracle.Rows.from_workload(wl), wl.q0, rbar,
                                               v0, wl.dt, order)
        assert_parity(qb.cpu().numpy(), ref_qb, 1e-12, CELL_F64)
        got_v = v0b.cpu().numpy()
        assert np.max(np.abs(got_v - ref_v0b)) <= 1e-10 * np.max(np.abs(ref_v0b))


def test_shift_adjoint_dot_product_gpu():
    wl = W.small_ragged(10, 6, 500, seed=21)
    rng = np.random.default_rng(1)
    a, r = rng.standard_normal(wl.n_cells), rng.standard_normal(wl.n_cells)
    sa = gpu_shift(wl, a, 5)
    rows = R.Rows.from_workload(wl, DEV)
    qb = torch.empty(wl.n_cells, dtype=torch.float64, device=DEV)
    R.ram_shift_adjoint(rows, None, dev(r), qb, dev(wl.v0), wl.dt, 5)
    torch.cuda.synchronize()
    lhs, rhs = np.dot(sa, r), np.dot(a, qb.cpu().numpy())
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(sa * r))


def test_residual_adjoint_fp64():
    wl = W.small_polar(6, 900)
    rng = np.random.default_rng(3)
    rbar = rng.standard_normal(wl.n_cells)
    rows = R.Rows.from_workload(wl, DEV)
    qb = torch.empty(wl.n_cells, dtype=torch.float64, device=DEV)
    dvb = dev(np.full(wl.n_cells, 0.5))
    R.ram_residual_adjoint(rows, dev(wl.q0.reshape(-1)), dev(wl.dv.reshape(-1)),
                           dev(rbar), qb, wl.dt, dvb)
    torch.cuda.synchronize()
    ref_qb, ref_dvb = oracle.residual_adjoint(oracle.Rows.from_workload(wl), wl.q0, wl.dv,
                                              rbar, wl.dt)
    assert_parity(qb.cpu().numpy(), ref_qb, 1e-12, CELL_F64)
    assert_parity(dvb.cpu().numpy() - 0.5, ref_dvb, 1e-12, CELL_F64)


def test_residual_adjoint_ragged_fp64():
    wl = W.small_ragged(20, 3, 700, seed=8)
    rng = np.random.default_rng(4)
    rbar = rng.standard_normal(wl.n_cells)
    rows = R.Rows.from_workload(wl, DEV)
    qb = torch.empty(wl.n_cells, dtype=torch.float64, device=DEV)
    dvb = torch.zeros(wl.n_cells, dtype=torch.float64, device=DEV)
    R.ram_residual_adjoint(rows, dev(wl.q0), dev(wl.dv), dev(rbar), qb, wl.dt, dvb)
    torch.cuda.synchronize()
    ref_qb, ref_dvb = oracle.residual_adjoint(oracle.Rows.from_workload(wl), wl.q0, wl.dv,
                                              rbar, wl.dt)
    assert_parity(qb.cpu().numpy(), ref_qb, 1e-12, CELL_F64)
    assert_parity(dvb.cpu().numpy(), ref_dvb, 1e-12, CELL_F64)


# --------------------------------------------------------------------------
# error paths that need a context
# --------------------------------------------------------------------------

def test_validate_reports_mesh_and_cfl():
    wl = W.small_polar(2, 64)
    rows = R.Rows.from_workload(wl, DEV)
    R.ram_validate(rows, torch.float64, dev(wl.dv.reshape(-1)), wl.dt)
    with pytest.raises(R.RamError) as ei:
        R.ram_validate(rows, torch.float64, dev(wl.dv.reshape(-1)), wl.dt * 10)
    assert ei.value.status == R.RAM_E_CFL
    bad = wl.edges.copy()
    bad[5], bad[6] = bad[6], bad[5]
    rows_bad = R.Rows(dev(bad), wl.n_rows, wl.n_cols, None, True)
    with pytest.raises(R.RamError) as ei:
        R.ram_validate(rows_bad, torch.float64)
    assert ei.value.status == R.RAM_E_MESH


def test_unsupported_order_with_context():
    wl = W.small_polar(2, 64)
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0.reshape(-1))
    with pytest.raises(R.RamError) as ei:
        R.ram_shift(rows, q, torch.empty_like(q), dev(wl.v0), wl.dt, 4)
    assert ei.value.status == R.RAM_E_UNSUPPORTED
