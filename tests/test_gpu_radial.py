"""Radial transport and the 2D split step on a polar grid (C ABI) against the
FP64 oracle.

* ram_radial_step: FP64 <= 1e-12 relative L1 (and elementwise) against the
  oracle's radial step on small disks whose column count leaves a ragged last
  workgroup, and on the degenerate grids (one row: nothing moves; two rows:
  only first-order fluxes; one column); FP32 <= 1e-6 against the oracle run on
  the same FP32 inputs; every column's area-weighted mass conserved;
* the 2048 x 16384 disk the benchmark times: sampled columns (through the
  density bump, at both ends of the periodic range) against the oracle, FP32
  and FP64, and the column masses;
* ram_step_split2d: n steps of (row step, radial step) against the oracle's
  step (Lagrange, order 5 and 3) or limited step (PLM, PPM) followed by its
  radial step, over 1 and 5 steps (the 5-step loop replayed from its captured
  graph on a second call), on shared and per-row azimuthal meshes; bit for bit
  the same as ram_step then ram_radial_step called one by one; the whole
  disk's mass conserved at full size.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
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


def _disk(n_r, n_phi, cfg=2):
    wl = W.small_polar(n_r, n_phi, cfg)
    u = W.radial_velocity(wl, cfg, amp=0.05)
    dt = min(wl.dt, W.radial_cfl_dt(wl.meta["r_edges"], u, 0.5))
    return wl, u, dt


def _narrow(n_r, n_cols):
    """A disk of only n_cols (uniform) azimuthal cells: the first columns of a
    wider one, for the radial step alone."""
    wl, u, dt = _disk(n_r, 64)
    wl = dataclasses.replace(wl, n_cols=n_cols, row_ptr=np.arange(n_r + 1) * n_cols,
                             edges=W.uniform_edges(n_cols, -np.pi, np.pi),
                             q0=np.ascontiguousarray(wl.q0[:, :n_cols]),
                             dv=np.ascontiguousarray(wl.dv[:, :n_cols]))
    return wl, np.ascontiguousarray(u[:, :n_cols]), dt


def _gpu_radial(wl, q, u, dt, dtype=torch.float64):
    rows = R.Rows.from_workload(wl, DEV)
    out = torch.empty(wl.n_cells, dtype=dtype, device=DEV)
    R.ram_radial_step(rows, dev(q, dtype), out, dev(wl.meta["r_edges"]), dev(u, dtype), dt)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64).reshape(wl.n_rows, wl.n_cols)


def _col_mass(re, q):
    area = 0.5 * (re[1:] ** 2 - re[:-1] ** 2)
    return np.sum(area[:, None] * q, axis=0)


@pytest.mark.parametrize("shape", [(16, 700), (40, 256), (7, 1), (5, 3), (1, 300),
                                   (2, 513), (3, 257)])
def test_radial_fp64(shape):
    wl, u, dt = _disk(*shape) if shape[1] >= 64 else _narrow(*shape)
    want = oracle.radial(wl.meta["r_edges"], wl.q0, u, dt)
    got = _gpu_radial(wl, wl.q0, u, dt)
    assert rel_l1(got, want) <= 1e-12
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-13)
    if shape[0] == 1:
        np.testing.assert_array_equal(got, wl.q0)
    re = wl.meta["r_edges"]
    m0, m1 = _col_mass(re, wl.q0), _col_mass(re, got)
    assert np.max(np.abs(m1 - m0) / np.abs(m0)) <= 1e-13


@pytest.mark.parametrize("shape", [(16, 700), (33, 1025)])
def test_radial_fp32(shape):
    wl, u, dt = _disk(*shape)
    q32, u32 = f32(wl.q0), f32(u)
    want = oracle.radial(wl.meta["r_edges"], q32, u32, dt)
    got = _gpu_radial(wl, q32, u32, dt, torch.float32)
    assert rel_l1(got, want) <= 1e-6


def test_radial_rejects_ragged_and_alias():
    wl = W.small_ragged(4, 8, 40, seed=3)
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0)
    re = dev(np.linspace(1.0, 2.0, 5))
    u = torch.zeros(5 * 40, dtype=torch.float64, device=DEV)
    with pytest.raises(R.RamError):
        R.ram_radial_step(rows, q, torch.empty_like(q), re, u, 0.1)
    wl2, u2, dt2 = _disk(4, 64)
    rows2 = R.Rows.from_workload(wl2, DEV)
    q2 = dev(wl2.q0)
    with pytest.raises(R.RamError):
        R.ram_radial_step(rows2, q2, q2, dev(wl2.meta["r_edges"]), dev(u2), dt2)


@pytest.fixture(scope="module")
def big():
    wl = W.cfg5()
    u = W.radial_velocity(wl, 5)
    return wl, u


COLS = np.array([0, 1, 5000, 8190, 8192, 8200, 11111, 16383])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_radial_full_size_sampled(big, dtype):
    wl, u = big
    q = wl.q0 if dtype == torch.float64 else f32(wl.q0)
    uu = u if dtype == torch.float64 else f32(u)
    got = _gpu_radial(wl, q, uu, wl.dt, dtype)
    want = oracle.radial(wl.meta["r_edges"], np.ascontiguousarray(q[:, COLS]),
                         np.ascontiguousarray(uu[:, COLS]), wl.dt)
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    assert rel_l1(got[:, COLS], want) <= tol
    re = wl.meta["r_edges"]
    m0, m1 = _col_mass(re, q), _col_mass(re, got)
    mtol = 1e-13 if dtype == torch.float64 else 1e-6
    assert np.max(np.abs(m1 - m0) / np.abs(m0)) <= mtol


# ---------------------------------------------------------------------------
# the 2D split step
# ---------------------------------------------------------------------------

def _oracle_split(wl, u, dt, n, order=5, recon=0, q=None):
    orows = oracle.Rows.from_workload(wl)
    q = wl.q0.reshape(-1) if q is None else q
    for _ in range(n):
        if recon:
            q = oracle.step_recon(orows, q, wl.v0, wl.dv, dt, recon, 1)
        else:
            q = oracle.step(orows, q, wl.v0, wl.dv, dt, order, 1)
        q = oracle.radial(wl.meta["r_edges"], q.reshape(wl.n_rows, wl.n_cols), u, dt)
        q = q.reshape(-1)
    return q


def _gpu_split(wl, u, dt, n, order=5, recon=0, dtype=torch.float64, scan=R.RAM_SCAN_F64,
               calls=1):
    rows = R.Rows.from_workload(wl, DEV)
    outs = []
    for _ in range(calls):
        q = dev(wl.q0, dtype)
        R.ram_step_split2d(rows, q, dev(wl.v0), dev(wl.dv, dtype), dev(wl.meta["r_edges"]),
                           dev(u, dtype), dt, order, n, scan, recon)
        torch.cuda.synchronize()
        outs.append(q.cpu().numpy().astype(np.float64))
    return outs


def _per_row_mesh(wl, seed=11):
    """The same disk with its own randomly stretched azimuthal mesh per row."""
    rng = np.random.default_rng(seed)
    e = np.concatenate([W.stretched_edges(wl.n_cols, 4.0, rng, -np.pi, np.pi)
                        for _ in range(wl.n_rows)])
    dt = min(W.residual_cfl_dt(e[r * (wl.n_cols + 1):(r + 1) * (wl.n_cols + 1)],
                               wl.dv[r:r + 1], 0.5) for r in range(wl.n_rows))
    return dataclasses.replace(wl, edges=e, edges_shared=False), dt


@pytest.mark.parametrize("n", [1, 5])
@pytest.mark.parametrize("order", [3, 5])
def test_split2d_lagrange_fp64(n, order):
    wl, u, dt = _disk(12, 900)
    want = _oracle_split(wl, u, dt, n, order)
    for got in _gpu_split(wl, u, dt, n, order, calls=2):
        assert rel_l1(got, want) <= 1e-12


@pytest.mark.parametrize("n", [1, 5])
@pytest.mark.parametrize("recon", [R.RAM_RECON_PLM, R.RAM_RECON_PPM])
def test_split2d_limited_fp64(n, recon):
    wl, u, dt = _disk(10, 1300)
    want = _oracle_split(wl, u, dt, n, recon=recon)
    for got in _gpu_split(wl, u, dt, n, recon=recon, calls=2):
        assert rel_l1(got, want) <= 1e-12


def test_split2d_per_row_meshes():
    wl, u, _ = _disk(9, 600)
    wl, dt = _per_row_mesh(wl)
    dt = min(dt, W.radial_cfl_dt(wl.meta["r_edges"], u, 0.5))
    want = _oracle_split(wl, u, dt, 4)
    for got in _gpu_split(wl, u, dt, 4, calls=2):
        assert rel_l1(got, want) <= 1e-12
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0)
    with pytest.raises(R.RamError):
        R.ram_step_split2d(rows, q, dev(wl.v0), dev(wl.dv), dev(wl.meta["r_edges"]), dev(u),
                           dt, 5, 1, R.RAM_SCAN_F64, R.RAM_RECON_PLM)


def test_split2d_fp32_direct():
    wl, u, dt = _disk(12, 2600)
    q32, dv32, u32 = f32(wl.q0), f32(wl.dv), f32(u)
    w32 = dataclasses.replace(wl, q0=q32, dv=dv32)
    want = _oracle_split(w32, u32, dt, 3)
    got = _gpu_split(wl, u, dt, 3, dtype=torch.float32, scan=R.RAM_SUM_DIRECT)[0]
    assert rel_l1(got, want) <= 1e-6


def test_split2d_one_row_is_the_row_step():
    wl, u, dt = _disk(1, 700)
    rows = R.Rows.from_workload(wl, DEV)
    a = dev(wl.q0)
    R.ram_step(rows, a, dev(wl.v0), dev(wl.dv), dt, 5, 3, R.RAM_SCAN_F64)
    got = _gpu_split(wl, u, dt, 3)[0]
    np.testing.assert_array_equal(got, a.cpu().numpy())


@pytest.mark.parametrize("use_density", [False, True])
def test_split2d_full_size_matches_calls(big, use_density):
    """The benchmark's configuration: FP32, direct sums, order 5; the graphed
    split loop equals the row and radial steps called one by one, and the
    disk's mass (sum of area * Q) is conserved."""
    wl, u = big
    rows = R.Rows.from_workload(wl, DEV)
    ctx = R.context(0)
    if use_density:
        ctx.set_mesh_density(wl.meta["bump"], -np.pi, np.pi)
    try:
        q0 = dev(wl.q0, torch.float32)
        v0, dv, re, uu = dev(wl.v0), dev(wl.dv, torch.float32), dev(wl.meta["r_edges"]), \
            dev(u, torch.float32)
        n = 4
        a = q0.clone()
        ctx.ram_step_split2d(rows, a, v0, dv, re, uu, wl.dt, 5, n, R.RAM_SUM_DIRECT)
        b = q0.clone()
        t = torch.empty_like(b)
        for _ in range(n):
            ctx.ram_step(rows, b, v0, dv, wl.dt, 5, 1, R.RAM_SUM_DIRECT)
            ctx.ram_radial_step(rows, b, t, re, uu, wl.dt)
            b.copy_(t)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        area = torch.as_tensor(wl.meta["area"].reshape(-1), dtype=torch.float64, device=DEV)
        m0 = float((area * q0.double()).sum())
        m1 = float((area * a.double()).sum())
        assert abs(m1 - m0) / abs(m0) <= 1e-6
    finally:
        ctx.set_mesh_density(None)
