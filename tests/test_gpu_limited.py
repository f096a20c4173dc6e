"""Parity of the limited-reconstruction shift and step (C ABI) with the FP64
oracle.

* ram_shift_limited, PLM and PPM: FP64 <= 1e-12 relative L1 on shared meshes
  (one tile and several), ragged per-row meshes, many rows of the stencil's
  minimum length, shifts below a cell, of many cells and of many periods
  either way, and a tile whose window overflows the on-chip buffer (direct
  path); FP32 <= 1e-6 against the oracle run on the same FP32 inputs;
* ram_step_limited: without residual it is ram_shift_limited bit for bit; with
  it, ram_shift_limited then ram_residual (bit for bit on per-row meshes, to
  rounding where a shared mesh fuses the two into one kernel); it matches the
  oracle's split step over 1 and 5 steps (the 5-step loop is replayed from its
  captured graph on a second call);
* the 2048 x 16384 polar disk in the configuration the benchmark times, on
  sampled rows (FP32 and FP64), plus every row's mass conserved and no value
  outside the input's range on a uniform mesh.
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


def _cases():
    return {
        "polar_one_tile": lambda: W.small_polar(6, 800),
        "polar_tiles": lambda: W.small_polar(3, 3500),
        "ragged": lambda: W.small_ragged(12, 6, 2600, seed=31),
        "tiny_rows": lambda: W.small_ragged(3000, 6, 12, seed=37),
    }


def _gpu_shift(wl, q, v0, recon, dtype=torch.float64):
    rows = R.Rows.from_workload(wl, DEV)
    out = torch.empty(wl.n_cells, dtype=dtype, device=DEV)
    R.ram_shift_limited(rows, dev(q, dtype), out, dev(v0), wl.dt, recon)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("recon", RECONS)
@pytest.mark.parametrize("kind", ["polar_one_tile", "polar_tiles", "ragged", "tiny_rows"])
def test_shift_limited_fp64(kind, recon):
    wl = _cases()[kind]()
    orows = oracle.Rows.from_workload(wl)
    for mult in (1.0, -23.7, 0.0137, 411.0):
        v0 = wl.v0 * mult
        got = _gpu_shift(wl, wl.q0, v0, recon)
        ref = oracle.shift_recon(orows, wl.q0, v0, wl.dt, recon)
        assert_parity(got, ref, 1e-12, CELL_F64, what=str(mult))


@pytest.mark.parametrize("recon", RECONS)
def test_shift_limited_window_overflow(recon):
    # 256 coarse cells then a 20x finer region: shifted by half the period, a
    # tile's source window exceeds the on-chip buffer
    coarse = np.linspace(0.0, 0.5, 257)
    fine = np.linspace(0.5, 1.0, 256 * 20 + 1)[1:]
    e = np.concatenate([coarse, fine])
    n = len(e) - 1
    rng = np.random.default_rng(5)
    q = 1.0 + 0.2 * rng.standard_normal(n)
    for s in (-0.5, -0.37, 0.41):
        wl = W.Workload("row", 1, n, np.array([0, n]), e, True, q[None, :], None,
                        np.array([s]), 1.0, 5, 1)
        got = _gpu_shift(wl, q, wl.v0, recon)
        ref = oracle.shift_recon(oracle.Rows.from_workload(wl), q, wl.v0, 1.0, recon)
        assert_parity(got, ref, 1e-12, CELL_F64, what=str(s))
        # the same mesh as per-row edges
        wr = W.Workload("row", 1, 0, np.array([0, n]), e, False, q[None, :], None,
                        np.array([s]), 1.0, 5, 1)
        got = _gpu_shift(wr, q, wr.v0, recon)
        assert_parity(got, ref, 1e-12, CELL_F64, what=str(s))


@pytest.mark.parametrize("recon", RECONS)
@pytest.mark.parametrize("kind", ["polar_tiles", "ragged"])
def test_shift_limited_fp32(kind, recon):
    wl = _cases()[kind]()
    q32 = wl.q0.reshape(-1).astype(np.float32).astype(np.float64)
    orows = oracle.Rows.from_workload(wl)
    for mult in (1.0, -23.7):
        v0 = wl.v0 * mult
        got = _gpu_shift(wl, q32, v0, recon, torch.float32)
        ref = oracle.shift_recon(orows, q32, v0, wl.dt, recon)
        err, ec = assert_parity(got, ref, 1e-6, CELL_F32, what=str(mult))
        print(f"{kind} recon {recon} FP32 rel-L1 {err:.2e}")
        assert err <= 1e-6, (mult, err)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("recon", RECONS)
@pytest.mark.parametrize("kind", ["polar_tiles", "ragged"])
def test_step_limited_is_shift_then_residual(kind, recon, dtype):
    wl = _cases()[kind]()
    rows = R.Rows.from_workload(wl, DEV)
    v0, dv = dev(wl.v0), dev(wl.dv, dtype)
    q0 = dev(wl.q0, dtype)
    half = torch.empty_like(q0)
    want = torch.empty_like(q0)
    R.ram_shift_limited(rows, q0, half, v0, wl.dt, recon)
    R.ram_residual(rows, half, want, dv, wl.dt)
    # a step without residual is the shift, bit for bit
    q = q0.clone()
    R.ram_step_limited(rows, q, v0, None, wl.dt, recon, 1)
    torch.cuda.synchronize()
    assert torch.equal(q, half)
    q = q0.clone()
    R.ram_step_limited(rows, q, v0, dv, wl.dt, recon, 1)
    torch.cuda.synchronize()
    if kind == "ragged":
        # per-row meshes: the shift kernel, then the residual kernel
        assert torch.equal(q, want)
    else:
        # a shared mesh fuses the residual into the shift kernel (its own
        # rounding order)
        err = rel_l1(q.cpu().numpy().astype(np.float64), want.cpu().numpy().astype(np.float64))
        assert err <= (1e-15 if dtype == torch.float64 else 1e-7), err


@pytest.mark.parametrize("recon", RECONS)
def test_step_limited_fp64(recon):
    wl = _cases()["polar_tiles"]()
    rows = R.Rows.from_workload(wl, DEV)
    orows = oracle.Rows.from_workload(wl)
    for k in (1, 5):
        ref = oracle.step_recon(orows, wl.q0, wl.v0, wl.dv, wl.dt, recon, k)
        for call in range(2 if k >= 4 else 1):     # the second call replays the graph
            q = dev(wl.q0)
            R.ram_step_limited(rows, q, dev(wl.v0), dev(wl.dv), wl.dt, recon, k)
            torch.cuda.synchronize()
            assert_parity(q.cpu().numpy(), ref, 1e-12, CELL_F64, what=str((k, call)))
    # shift-only steps on ragged per-row meshes (an odd count ends in scratch)
    wr = _cases()["ragged"]()
    rows = R.Rows.from_workload(wr, DEV)
    ref = oracle.step_recon(oracle.Rows.from_workload(wr), wr.q0, wr.v0, None, wr.dt, recon, 5)
    q = dev(wr.q0)
    R.ram_step_limited(rows, q, dev(wr.v0), None, wr.dt, recon, 5)
    torch.cuda.synchronize()
    assert_parity(q.cpu().numpy(), ref, 1e-12, CELL_F64)


def _sample_rows(wl, rows):
    q = wl.q0.reshape(wl.n_rows, -1)[rows]
    dv = wl.dv.reshape(wl.n_rows, -1)[rows]
    n = wl.n_cols
    return W.Workload("sample", len(rows), n, np.arange(len(rows) + 1) * n, wl.edges,
                      True, q, dv, wl.v0[rows], wl.dt, wl.order, wl.steps)


@pytest.mark.parametrize("recon", RECONS)
def test_limited_full_size_sampled_rows(recon):
    wl = W.cfg5()
    rows = R.Rows.from_workload(wl, DEV)
    pick = np.array([0, 5, 1024, 2047])
    sw = _sample_rows(wl, pick)
    orows = oracle.Rows.from_workload(sw)
    # FP32 state, one step, the benchmark's launch configuration
    q32 = wl.q0.astype(np.float32)
    dv32 = wl.dv.astype(np.float32)
    q = dev(q32, torch.float32)
    R.ram_step_limited(rows, q, dev(wl.v0), dev(dv32, torch.float32), wl.dt, recon, 1)
    torch.cuda.synchronize()
    got = q.cpu().numpy().astype(np.float64).reshape(wl.n_rows, -1)[pick].reshape(-1)
    ref = oracle.step_recon(orows, q32.reshape(wl.n_rows, -1)[pick].astype(np.float64),
                            sw.v0, dv32.reshape(wl.n_rows, -1)[pick].astype(np.float64),
                            sw.dt, recon, 1)
    assert_parity(got, ref, 1e-6, CELL_F32)
    # FP64, two steps; every row's mass is conserved
    q = dev(wl.q0)
    R.ram_step_limited(rows, q, dev(wl.v0), dev(wl.dv), wl.dt, recon, 2)
    torch.cuda.synchronize()
    got = q.cpu().numpy().reshape(wl.n_rows, -1)
    ref = oracle.step_recon(orows, sw.q0, sw.v0, sw.dv, sw.dt, recon, 2)
    assert_parity(got[pick].reshape(-1), ref, 1e-12, CELL_F64)
    dx = np.diff(wl.edges)
    m0 = wl.q0.reshape(wl.n_rows, -1) @ dx
    m1 = got @ dx
    assert np.max(np.abs(m1 - m0) / m0) <= 1e-12


@pytest.mark.parametrize("recon", RECONS)
def test_limited_no_new_extrema_uniform(recon):
    n = 5000
    e = np.linspace(0.0, 1.0, n + 1)
    rng = np.random.default_rng(8)
    q = np.where(rng.random((4, n)) > 0.6, 2.0, -1.0) + 0.1 * rng.random((4, n))
    wl = W.Workload("steps", 4, n, np.arange(5) * n, e, True, q, None,
                    np.array([0.3137, -2.71, 0.0123, 57.77]), 1.0, 5, 1)
    got = _gpu_shift(wl, q, wl.v0, recon).reshape(4, n)
    assert got.min() >= q.min() - 1e-12 and got.max() <= q.max() + 1e-12
