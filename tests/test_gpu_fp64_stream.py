"""The FP64 step on a shared mesh at the default schedule (k_step64: tiles of
256 cells a wave on the streaming plan, every node's Lagrange weights in FP64
from its source cell's stencil data) against the FP64 oracle, relative L1 <= 1e-12
and per cell CELL_F64 (Section 3's bulk shift, Steps 1-3, then the residual
step of Section 3.1):

* a uniform mesh (every tile a uniform-run tile: no node plan) and the same
  mesh with edges perturbed by 1e-15 (still one run to the mesh's
  tolerance) shifted by whole cells, so that the shifted nodes fall on both
  sides of the source edges by rounding and a uniform tile's node must be
  moved to the neighbouring cell;
* the refined polar disk (uniform-run and planned tiles), both cumulative
  modes (FP64 window prefix, direct sums), orders 1, 3 and 5, with and
  without the residual, over one and three steps;
* a coarse half beside a 2x or 20x finer half (windows wider than the LDS
  buffer: nodes located and summed from global memory);
* shifts by whole cells of a uniform mesh: the permutation, to 1e-15;
* rows of 8, 13, 264 and 300 cells (windows that wrap the row) and of 1001
  cells (no 16-byte stores);
* the recorded trajectory's half steps (the shifted state before the
  residual) against the oracle's shift;
* the 2048 x 16384 disk on sampled rows.
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
SCANS = {"prefix": R.RAM_SCAN_F64, "direct": R.RAM_SUM_DIRECT}


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=torch.float64, device=DEV)


@pytest.fixture(autouse=True)
def default_schedule():
    c = R.context(0)
    c.set_schedule(0)
    yield
    c.set_schedule(0)


def _wl(edges, v0, seed, with_dv=True, n_rows=None):
    n = len(edges) - 1
    v0 = np.asarray(v0, dtype=np.float64)
    n_rows = len(v0) if n_rows is None else n_rows
    rng = np.random.default_rng(seed)
    xc = 0.5 * (edges[:-1] + edges[1:])
    q = 1.0 + 0.3 * np.sin(2 * np.pi * xc)[None, :] + 0.2 * rng.standard_normal((n_rows, n))
    dv = (0.2 * np.diff(edges).min() * rng.uniform(-1, 1, (n_rows, n))) if with_dv else None
    return W.Workload("fp64", n_rows, n, np.arange(n_rows + 1) * n, edges, True, q, dv, v0,
                      1.0, 5, 1)


def _step(wl, order, steps, scan, with_dv=True, what=""):
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0)
    dv = dev(wl.dv) if with_dv else None
    R.ram_step(rows, q, dev(wl.v0), dv, wl.dt, order, steps, scan)
    torch.cuda.synchronize()
    want = oracle.step(oracle.Rows.from_workload(wl), wl.q0, wl.v0,
                       wl.dv if with_dv else None, wl.dt, order, steps)
    e1, ec = assert_parity(q.cpu().numpy(), want, 1e-12, CELL_F64, what)
    print(f"{what}: rel-L1 {e1:.2e}, max cell {ec:.2e}")


def _uniform(n):
    return np.linspace(0.0, 1.0, n + 1)


@pytest.mark.parametrize("scan", list(SCANS))
@pytest.mark.parametrize("with_dv", [False, True])
def test_uniform_mesh(scan, with_dv):
    n = 4096
    v0 = np.array([0.3, 0.37, 5.21, -3.7, 2.5 * n + 7.3, -n - 0.61]) / n
    _step(_wl(_uniform(n), v0, 3), 5, 2, SCANS[scan], with_dv, f"uniform {scan} dv={with_dv}")


@pytest.mark.parametrize("scan", list(SCANS))
def test_whole_cell_shifts_on_a_rounded_mesh(scan):
    # edges off the grid by up to 1e-15: a shift by whole cells puts nodes a
    # rounding error below or above their source edge
    n = 4096
    rng = np.random.default_rng(7)
    e = _uniform(n)
    e[1:-1] += 1e-15 * rng.uniform(-1, 1, n - 1)
    v0 = np.array([3.0, -17.0, 1000.0, 0.0, n + 1.0, -2.0 * n - 5.0]) / n
    for with_dv in (False, True):
        _step(_wl(e, v0, 5, with_dv), 5, 1, SCANS[scan], with_dv, f"whole cells {scan}")


def _polar(order):
    wl = W.small_polar(12, 4096, order=order)
    n = wl.n_cols
    wl.v0[:] = wl.v0 * np.array([1.0, -1.0, 7.3, -11.9, 0.02, -0.05,
                                 n * 0.37, -n * 0.81, 1.0, -2.0, 3.0, -4.0])
    return wl


@pytest.mark.parametrize("steps", [1, 3])
@pytest.mark.parametrize("with_dv", [False, True])
@pytest.mark.parametrize("order", [1, 3, 5])
@pytest.mark.parametrize("scan", list(SCANS))
def test_polar_disk(scan, order, with_dv, steps):
    _step(_polar(order), order, steps, SCANS[scan], with_dv,
          f"polar {scan} order {order} dv={with_dv} steps {steps}")


@pytest.mark.parametrize("ratio", [2, 20])
@pytest.mark.parametrize("scan", list(SCANS))
def test_windows_beyond_the_lds(scan, ratio):
    # coarse tiles shifted onto the finer half: windows of about 520 cells
    # (ratio 2: beyond the prefix mode's LDS window, inside the direct mode's)
    # or thousands (ratio 20: beyond both)
    coarse = np.linspace(0.0, 0.5, 257)
    fine = np.linspace(0.5, 1.0, 256 * ratio + 1)[1:]
    e = np.concatenate([coarse, fine])
    for with_dv in (False, True):
        _step(_wl(e, [-0.5, -0.37, 0.41], 9, with_dv), 5, 1, SCANS[scan], with_dv,
              f"jump x{ratio} {scan} dv={with_dv}")


@pytest.mark.parametrize("scan", list(SCANS))
def test_whole_cell_shift_is_a_permutation(scan):
    # a shift by whole cells of a uniform mesh moves every value unchanged
    # (Section 1's integer shift): the single whole cell's mass is taken as is
    n = 4096
    v0 = np.array([0.0, 3.0, -17.0, 5.0 * n + 2.0]) / n
    wl = _wl(_uniform(n), v0, 11, with_dv=False)
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0)
    R.ram_step(rows, q, dev(wl.v0), None, wl.dt, 5, 1, SCANS[scan])
    torch.cuda.synchronize()
    got = q.cpu().numpy().reshape(wl.n_rows, n)
    for r, k in enumerate([0, 3, -17, 2]):
        want = np.roll(wl.q0.reshape(wl.n_rows, n)[r], k)
        err = np.sum(np.abs(got[r] - want)) / np.sum(np.abs(want))
        assert err <= 1e-15, (scan, r, err)


@pytest.mark.parametrize("n", [8, 13, 264, 300, 1001])
@pytest.mark.parametrize("scan", list(SCANS))
def test_short_and_odd_rows(scan, n):
    rng = np.random.default_rng(n)
    e = W.stretched_edges(n, 8.0, rng)
    v0 = np.array([0.3, -17.2, n + 0.6, -1.7 * n]) / n
    for with_dv in (False, True):
        _step(_wl(e, v0, n, with_dv), 5, 2, SCANS[scan], with_dv, f"n={n} {scan} dv={with_dv}")


def test_recorded_half_steps():
    wl = _polar(5)
    rows = R.Rows.from_workload(wl, DEV)
    k = 3
    traj = torch.empty((k + 1, wl.n_cells), dtype=torch.float64, device=DEV)
    half = torch.empty((k, wl.n_cells), dtype=torch.float64, device=DEV)
    traj[0] = dev(wl.q0)
    R.context(0).ram_step_record(rows, traj, half, dev(wl.v0), dev(wl.dv), wl.dt, 5, k)
    torch.cuda.synchronize()
    orows = oracle.Rows.from_workload(wl)
    q = wl.q0.reshape(-1)
    for s in range(k):
        qh = oracle.shift(orows, q, wl.v0, wl.dt, 5)
        assert_parity(half[s].cpu().numpy(), qh, 1e-12, CELL_F64, f"half step {s}")
        q = oracle.step(orows, q, wl.v0, wl.dv, wl.dt, 5, 1)
        assert_parity(traj[s + 1].cpu().numpy(), q, 1e-12, CELL_F64, f"step {s}")


@pytest.mark.parametrize("scan", list(SCANS))
def test_cfg5_sampled_rows(scan):
    wl = W.cfg5()
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0)
    R.ram_step(rows, q, dev(wl.v0), dev(wl.dv), wl.dt, 5, 1, SCANS[scan])
    torch.cuda.synchronize()
    got = q.cpu().numpy().reshape(wl.n_rows, -1)
    n = wl.n_cols
    one = oracle.Rows.single(wl.edges)
    for r in (0, 1, 700, 1024, 2047):
        s = slice(r * n, (r + 1) * n)
        want = oracle.step(one, wl.q0.reshape(-1)[s], wl.v0[r:r + 1], wl.dv.reshape(-1)[s],
                           wl.dt, 5, 1)
        e1, ec = assert_parity(got[r], want, 1e-12, CELL_F64, f"row {r}")
        print(f"cfg5 {scan} row {r}: rel-L1 {e1:.2e}, max cell {ec:.2e}")
