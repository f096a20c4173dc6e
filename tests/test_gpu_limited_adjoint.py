"""Parity of the limited shift's adjoint (ram_shift_limited_adjoint, C ABI)
with the FP64 oracle's transposed Jacobian.

qbar <= 1e-12 relative L1 and v0bar <= 1e-10 of its largest entry in FP64, on
shared meshes (one tile and several), ragged per-row meshes, rows of the
stencil's minimum length, shifts below a cell and of many cells and periods
either way, and a mesh with a 20x refinement jump; FP32 state <= 1e-6
against the oracle on the same FP32 inputs (the adjoint computes in FP64 and
rounds once); the 2048 x 16384 disk on sampled rows.
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
RECONS = [R.RAM_RECON_PLM, R.RAM_RECON_PPM]


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=dtype, device=DEV)


def rel_l1(a, b):
    return float(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))


def _gpu(wl, q, qb, v0, recon, dtype=torch.float64):
    rows = R.Rows.from_workload(wl, DEV)
    out = torch.empty(wl.n_cells, dtype=dtype, device=DEV)
    v0b = torch.zeros(wl.n_rows, dtype=torch.float64, device=DEV)
    R.ram_shift_limited_adjoint(rows, dev(q, dtype), dev(qb, dtype), out, dev(v0), wl.dt,
                                recon, v0b)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), v0b.cpu().numpy()


def _cases():
    return {
        "polar_one_tile": lambda: W.small_polar(6, 200),
        "polar_tiles": lambda: W.small_polar(3, 3500),
        "ragged": lambda: W.small_ragged(12, 6, 2600, seed=31),
        "tiny_rows": lambda: W.small_ragged(500, 6, 12, seed=37),
    }


@pytest.mark.parametrize("recon", RECONS)
@pytest.mark.parametrize("kind", ["polar_one_tile", "polar_tiles", "ragged", "tiny_rows"])
def test_limited_adjoint_fp64(kind, recon):
    wl = _cases()[kind]()
    orows = oracle.Rows.from_workload(wl)
    rng = np.random.default_rng(7)
    qb = rng.standard_normal(wl.n_cells)
    for mult in (1.0, -23.7, 0.0137, 411.0):
        v0 = wl.v0 * mult
        got, gv = _gpu(wl, wl.q0, qb, v0, recon)
        ref, rv = oracle.shift_recon_adjoint(orows, wl.q0, qb, v0, wl.dt, recon)
        assert_parity(got, ref, 1e-12, CELL_F64, what=str((mult, rel_l1(got, ref))))
        assert np.max(np.abs(gv - rv)) <= 1e-10 * np.max(np.abs(rv)), mult


@pytest.mark.parametrize("recon", RECONS)
def test_limited_adjoint_refinement_jump(recon):
    coarse = np.linspace(0.0, 0.5, 257)
    fine = np.linspace(0.5, 1.0, 256 * 20 + 1)[1:]
    e = np.concatenate([coarse, fine])
    n = len(e) - 1
    rng = np.random.default_rng(5)
    q = 1.0 + 0.2 * rng.standard_normal(n)
    qb = rng.standard_normal(n)
    for s in (-0.5, -0.37, 0.41):
        wl = W.Workload("row", 1, n, np.array([0, n]), e, True, q[None, :], None,
                        np.array([s]), 1.0, 5, 1)
        got, gv = _gpu(wl, q, qb, wl.v0, recon)
        ref, rv = oracle.shift_recon_adjoint(oracle.Rows.from_workload(wl), q, qb, wl.v0,
                                             1.0, recon)
        assert_parity(got, ref, 1e-12, CELL_F64, what=str(s))
        assert abs(gv[0] - rv[0]) <= 1e-10 * abs(rv[0]), s


@pytest.mark.parametrize("recon", RECONS)
@pytest.mark.parametrize("kind", ["polar_tiles", "ragged"])
def test_limited_adjoint_fp32(kind, recon):
    wl = _cases()[kind]()
    rng = np.random.default_rng(11)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    q = f32(wl.q0.reshape(-1))
    qb = f32(rng.standard_normal(wl.n_cells))
    got, gv = _gpu(wl, q, qb, wl.v0, recon, torch.float32)
    ref, rv = oracle.shift_recon_adjoint(oracle.Rows.from_workload(wl), q, qb, wl.v0, wl.dt,
                                         recon)
    assert_parity(got, ref, 1e-6, CELL_F32)
    assert np.max(np.abs(gv - rv)) <= 1e-10 * np.max(np.abs(rv))


@pytest.mark.parametrize("recon", RECONS)
def test_limited_adjoint_full_size_sampled_rows(recon):
    wl = W.cfg5()
    rows = R.Rows.from_workload(wl, DEV)
    rng = np.random.default_rng(2)
    qb = rng.standard_normal(wl.n_cells)
    out = torch.empty(wl.n_cells, dtype=torch.float64, device=DEV)
    v0b = torch.zeros(wl.n_rows, dtype=torch.float64, device=DEV)
    R.ram_shift_limited_adjoint(rows, dev(wl.q0), dev(qb), out, dev(wl.v0), wl.dt, recon, v0b)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(wl.n_rows, -1)
    gv = v0b.cpu().numpy()
    n = wl.n_cols
    # the density bump sits on the rows near r = 1 (row 1024); rows far from it
    # hold Q = 1 exactly, where v0bar is a sum that cancels to zero
    pick = (0, 1020, 1024, 1031, 2047)
    rvs = []
    for r in pick:
        sub = oracle.Rows(np.array([0, n]), wl.edges, True)
        ref, rv = oracle.shift_recon_adjoint(sub, wl.q0.reshape(wl.n_rows, -1)[r],
                                             qb.reshape(wl.n_rows, -1)[r], wl.v0[r:r + 1],
                                             wl.dt, recon)
        assert_parity(got[r], ref, 1e-12, CELL_F64, what=str(r))
        rvs.append(rv[0])
    rvs = np.array(rvs)
    assert np.max(np.abs(rvs)) > 0.0
    assert np.max(np.abs(gv[list(pick)] - rvs)) <= 1e-10 * np.max(np.abs(rvs))
