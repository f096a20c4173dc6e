"""The FP32 direct-sum step on tiles that lie in a uniform run of a shared mesh
(one stencil offset and one theta for every node of the tile, from the window
plan) against the FP64 oracle run on the same FP32 inputs, <= 1e-6 relative
L1:

* a uniform mesh (every tile takes the uniform path), shifts below a cell,
  of several cells and of many periods either way, with and without the
  residual, over one and five steps;
* the same mesh with one cell 0.1 % shorter (the rest stay the largest, so
  the run holds every other cell): the tiles that see it must not take the
  uniform path (the check would miss it by far more than 1e-6);
* a mesh of a coarse and a fine uniform half (the runs at the largest and at
  the smallest size), and the same with one fine cell 0.1 % longer;
* the polar disk's bump mesh, whose coarse run wraps over the periodic seam,
  with its fine run inside the bump and tiles straddling the runs' ends;
* the limited PLM / PPM step on the same three meshes (each node's cell
  cubic at the tile's shared theta), against the oracle's limited step;
* uniform rows of 6 .. 13 cells, whose windows wrap the row;
* a cell 10 % shorter or longer on either side of a boundary of the wave
  segments the uniform-run tables are built in;
* one row of 2^20 + 3 cells (segments of ~65k cells, ~1000 tiles a row);
* a limited step whose uniform tile's window starts at a run's first cell
  (its left neighbour off the run: the shared PPM weights must come from
  cells whose neighbourhood is in the run).

In a uniform tile the FP32 Lagrange step is one (P+1)-point stencil on the
cell values, so these cases also check its weights (from the Lagrange
weights at theta) and the residual on the run's constant geometry.
"""
import numpy as np
import pytest
import torch

import oracle
from parity import CELL_F32, assert_parity
from paper_2305_05362_amd import _lib as R
from paper_2305_05362_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=dtype, device=DEV)


def rel_l1(a, b):
    return float(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _rows(edges, n_rows, seed, shifts):
    n = len(edges) - 1
    rng = np.random.default_rng(seed)
    xc = 0.5 * (edges[:-1] + edges[1:])
    q = 1.0 + 0.3 * np.sin(2 * np.pi * xc)[None, :] + 0.05 * rng.standard_normal((n_rows, n))
    dv = 0.2 * np.diff(edges).min() * rng.uniform(-1, 1, (n_rows, n))
    wl = W.Workload("uni", n_rows, n, np.arange(n_rows + 1) * n, edges, True, f32(q),
                    f32(dv), np.asarray(shifts, dtype=np.float64), 1.0, 5, 1)
    return wl


def _check(wl, steps, with_dv, order=5):
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0, torch.float32)
    dv = dev(wl.dv, torch.float32) if with_dv else None
    R.ram_step(rows, q, dev(wl.v0), dv, wl.dt, order, steps, R.RAM_SUM_DIRECT)
    torch.cuda.synchronize()
    want = oracle.step(oracle.Rows.from_workload(wl), wl.q0, wl.v0,
                       wl.dv if with_dv else None, wl.dt, order, steps)
    e1, ec = assert_parity(q.cpu().numpy().astype(np.float64), want, 1e-6, CELL_F32, "step")
    print(f"rel-L1 {e1:.2e}, max cell {ec:.2e}")


SHIFTS = [0.3 / 4096, 0.37 / 4096, 5.21 / 4096, -3.7 / 4096, 2.5 + 7.3 / 4096, -1.0 - 0.61 / 4096]


@pytest.mark.parametrize("steps", [1, 5])
@pytest.mark.parametrize("with_dv", [False, True])
def test_uniform_mesh(steps, with_dv):
    e = W.uniform_edges(4096, 0.0, 1.0)
    _check(_rows(e, len(SHIFTS), 1, SHIFTS), steps, with_dv)


@pytest.mark.parametrize("order", [1, 3])
def test_uniform_mesh_lower_orders(order):
    # the stencil has order + 1 points
    e = W.uniform_edges(4096, 0.0, 1.0)
    _check(_rows(e, len(SHIFTS), 8, SHIFTS), 3, True, order)


@pytest.mark.parametrize("cell", [0, 1500, 4095])
def test_one_shorter_cell(cell):
    e = W.uniform_edges(4096, 0.0, 1.0).copy()
    h = e[1] - e[0]
    e[cell + 1:] -= 1e-3 * h          # cell `cell` is 0.1 % shorter
    e = e * (1.0 / e[-1])
    _check(_rows(e, len(SHIFTS), 2, SHIFTS), 3, True)


def _two_levels(perturb=None):
    # 1024 coarse cells on [0, 0.5), 4096 fine on [0.5, 1): both runs uniform
    e = np.concatenate([np.linspace(0.0, 0.5, 1025), np.linspace(0.5, 1.0, 4097)[1:]])
    if perturb is not None:
        h = e[perturb + 1] - e[perturb]
        e[perturb + 1:] += 1e-3 * h       # one fine cell 0.1 % longer
        e = e * (1.0 / e[-1])
    return e


@pytest.mark.parametrize("perturb", [None, 3000])
def test_coarse_and_fine_runs(perturb):
    # the fine run (the mesh's smallest size) takes the uniform path too; a
    # fine cell 0.1 % longer (neither the largest nor the smallest size) must
    # keep its tiles off it
    e = _two_levels(perturb)
    shifts = [0.3 / 4096, 20.3 / 4096, -7.7 / 4096, 0.71]
    _check(_rows(e, len(shifts), 6, shifts), 3, True)


def test_bump_mesh_runs_and_seam():
    wl = W.small_polar(8, 6000)
    w32 = _rows(wl.edges, 8, 3, wl.v0 * wl.dt)
    _check(w32, 4, True)


def _check_limited(wl, steps, recon):
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0, torch.float32)
    R.ram_step_limited(rows, q, dev(wl.v0), dev(wl.dv, torch.float32), wl.dt, recon, steps)
    torch.cuda.synchronize()
    want = oracle.step_recon(oracle.Rows.from_workload(wl), wl.q0, wl.v0, wl.dv, wl.dt,
                             recon, steps)
    e1, ec = assert_parity(q.cpu().numpy().astype(np.float64), want, 1e-6, CELL_F32, "limited")
    print(f"rel-L1 {e1:.2e}, max cell {ec:.2e}")


@pytest.mark.parametrize("recon", [R.RAM_RECON_PLM, R.RAM_RECON_PPM])
@pytest.mark.parametrize("mesh", ["uniform", "shorter", "bump"])
def test_limited_uniform_tiles(recon, mesh):
    # the limited cubic of each cell at the tile's shared theta
    if mesh == "bump":
        wl0 = W.small_polar(8, 6000)
        wl = _rows(wl0.edges, 8, 4, wl0.v0 * wl0.dt)
    else:
        e = W.uniform_edges(4096, 0.0, 1.0).copy()
        if mesh == "shorter":
            e[2001:] -= 1e-3 * (e[1] - e[0])
            e = e * (1.0 / e[-1])
        wl = _rows(e, len(SHIFTS), 5, SHIFTS)
    _check_limited(wl, 3, recon)


@pytest.mark.parametrize("n", [6, 7, 9, 13])
def test_tiny_uniform_rows(n):
    # rows of order+1 cells and a few more: the source window (the row's cells
    # plus the residual's halo and the stencil) wraps the row, every tile is
    # uniform
    e = W.uniform_edges(n, 0.0, 1.0)
    shifts = [0.3 / n, 2.7 / n, -1.4 / n, 5.05]
    _check(_rows(e, len(shifts), 7, shifts), 3, True)


@pytest.mark.parametrize("n,cell", [(4096, 255), (4096, 256), (4096, 3840), (4099, 256),
                                    (4099, 257), (4099, 4098)])
@pytest.mark.parametrize("sign", [-1.0, 1.0])
def test_run_tables_at_segment_boundaries(n, cell, sign):
    # the uniform-run tables are prefix counts built one wave segment
    # (ceil(n / 16) cells) at a time: one cell 10 % shorter (off the largest
    # size) or 10 % longer (then the largest, the rest off it but at the
    # smallest) on either side of a segment boundary must keep every tile that
    # sees it off the uniform path; misread, the error would be ~1e-4
    e = W.uniform_edges(n, 0.0, 1.0).copy()
    e[cell + 1:] += sign * 0.1 * (e[1] - e[0])
    e = e * (1.0 / e[-1])
    shifts = [0.3 / n, 5.21 / n, -3.7 / n, 0.5 + 1.7 / n]
    _check(_rows(e, len(shifts), 9, shifts), 2, True)


def test_long_row():
    # one row of 2^20 + 3 cells: wave segments of ~65k cells in the run
    # tables, a tile table of ~1000 tiles, a 10 % shorter cell deep inside,
    # shifts across many tiles
    n = (1 << 20) + 3
    e = W.uniform_edges(n, 0.0, 1.0).copy()
    e[700001:] -= 0.1 * (e[1] - e[0])
    e = e * (1.0 / e[-1])
    shifts = [0.37 / n, 3001.6 / n]
    _check(_rows(e, len(shifts), 10, shifts), 2, True)


@pytest.mark.parametrize("recon", [R.RAM_RECON_PLM, R.RAM_RECON_PPM])
def test_limited_window_at_run_start(recon):
    # 4096 coarse cells then 4096 four times finer: shifted by 1014.6 coarse
    # cells, the second tile's source window starts at cell 0, the coarse
    # run's first cell, whose left neighbour (across the seam) is fine.  The
    # tile is uniform; its limited weights must come from cells whose whole
    # neighbourhood is in the run
    e = np.concatenate([np.linspace(0.0, 0.8, 4097), np.linspace(0.8, 1.0, 4097)[1:]])
    hc = 0.8 / 4096
    shifts = [1014.6 * hc, 1014.6 * hc + 0.3 * hc, 3.3 * hc]
    wl = _rows(e, len(shifts), 11, shifts)
    _check_limited(wl, 2, recon)
