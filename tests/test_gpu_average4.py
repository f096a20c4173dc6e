"""The fourth-order conversion between centre values and cell averages, and
the step on a state of centre values (C ABI), against the FP64 oracle.

* ram_cell_average, both directions: FP64 <= 1e-12 relative L1 (and
  elementwise) against the oracle on the polar disk's shared bump mesh (tiles
  with a ragged last one), ragged per-row meshes, rows of one to three cells,
  and a uniform mesh; FP32 <= 1e-6 against the oracle run on the same FP32
  inputs;
* ram_step_point4: against the oracle's conversion, step (Lagrange order 3
  and 5, or limited PLM / PPM) and inverse conversion, over 1 and 5 steps
  (the 5-step loop replayed from its graph on a second call), on shared and
  ragged meshes;
* at the 2048 x 16384 disk's size in the benchmark's configuration: the
  graphed loop (which converts back and forth between two steps in one
  pass) equals the three calls made one by one to rounding, and sampled
  rows match the oracle;
* what the conversion is for, against the exact solution rather than the
  oracle: a point-sampled smooth function shifted on a smoothly stretched
  mesh converges at fourth order on the GPU with the conversion, at second
  order without.
"""
import math

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


def _cases():
    return {
        "polar_tiles": lambda: W.small_polar(6, 2600),
        "ragged": lambda: W.small_ragged(12, 6, 2600, seed=41),
        "tiny_rows": lambda: W.small_ragged(200, 1, 3, seed=43),
        "uniform": lambda: W.cfg1(),
    }


def _gpu_avg(wl, q, to_centre, dtype=torch.float64):
    rows = R.Rows.from_workload(wl, DEV)
    out = torch.empty(wl.n_cells, dtype=dtype, device=DEV)
    R.ram_cell_average(rows, dev(q, dtype), out, to_centre)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("to_centre", [False, True])
@pytest.mark.parametrize("kind", ["polar_tiles", "ragged", "tiny_rows", "uniform"])
def test_cell_average_fp64(kind, to_centre):
    wl = _cases()[kind]()
    q = wl.q0.reshape(-1)
    want = oracle.average4(oracle.Rows.from_workload(wl), q, to_centre)
    got = _gpu_avg(wl, q, to_centre)
    assert rel_l1(got, want) <= 1e-12
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("to_centre", [False, True])
@pytest.mark.parametrize("kind", ["polar_tiles", "ragged"])
def test_cell_average_fp32(kind, to_centre):
    wl = _cases()[kind]()
    q = f32(wl.q0.reshape(-1))
    want = oracle.average4(oracle.Rows.from_workload(wl), q, to_centre)
    got = _gpu_avg(wl, q, to_centre, torch.float32)
    assert rel_l1(got, want) <= 1e-6


def test_cell_average_rejects_alias():
    wl = W.small_polar(3, 300)
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0)
    with pytest.raises(R.RamError):
        R.ram_cell_average(rows, q, q)


def _oracle_point4(wl, q, n, order=5, recon=0, dv=True):
    orows = oracle.Rows.from_workload(wl)
    d = wl.dv if dv else None
    q = np.asarray(q, dtype=np.float64).reshape(-1)
    for _ in range(n):
        a = oracle.average4(orows, q)
        if recon:
            a = oracle.step_recon(orows, a, wl.v0, d, wl.dt, recon, 1)
        else:
            a = oracle.step(orows, a, wl.v0, d, wl.dt, order, 1)
        q = oracle.point4(orows, a)
    return q


def _gpu_point4(wl, n, order=5, recon=0, dtype=torch.float64, scan=R.RAM_SCAN_F64, calls=1,
                dv=True):
    rows = R.Rows.from_workload(wl, DEV)
    outs = []
    d = dev(wl.dv, dtype) if dv else None
    for _ in range(calls):
        q = dev(wl.q0, dtype)
        R.ram_step_point4(rows, q, dev(wl.v0), d, wl.dt, order, n, scan, recon)
        torch.cuda.synchronize()
        outs.append(q.cpu().numpy().astype(np.float64))
    return outs


@pytest.mark.parametrize("n", [1, 5])
@pytest.mark.parametrize("order", [3, 5])
def test_step_point4_lagrange_shared(n, order):
    wl = W.small_polar(8, 1500)
    want = _oracle_point4(wl, wl.q0, n, order)
    for got in _gpu_point4(wl, n, order, calls=2):
        assert rel_l1(got, want) <= 1e-12


def test_step_point4_ragged():
    wl = W.small_ragged(10, 8, 2000, seed=47, with_dv=False)
    want = _oracle_point4(wl, wl.q0, 5, dv=False)
    for got in _gpu_point4(wl, 5, calls=2, dv=False):
        assert rel_l1(got, want) <= 1e-12


@pytest.mark.parametrize("recon", [R.RAM_RECON_PLM, R.RAM_RECON_PPM])
def test_step_point4_limited(recon):
    wl = W.small_polar(6, 1300)
    want = _oracle_point4(wl, wl.q0, 5, recon=recon)
    for got in _gpu_point4(wl, 5, recon=recon, calls=2):
        assert rel_l1(got, want) <= 1e-12
    wr = W.small_ragged(4, 8, 100, seed=5)
    rows = R.Rows.from_workload(wr, DEV)
    with pytest.raises(R.RamError):
        R.ram_step_point4(rows, dev(wr.q0), dev(wr.v0), None, wr.dt, 5, 1,
                          R.RAM_SCAN_F64, recon)


@pytest.mark.parametrize("kind", ["shared", "ragged"])
def test_between_steps_pass_is_the_two_conversions(kind):
    # FP64, ten steps: the loop's one-pass conversion between steps against
    # separate calls (inverse, then forward conversion), to rounding
    wl = W.small_polar(5, 1100) if kind == "shared" else W.small_ragged(9, 4, 1500, seed=53,
                                                                        with_dv=False)
    dvt = dev(wl.dv) if wl.dv is not None else None
    rows = R.Rows.from_workload(wl, DEV)
    a = dev(wl.q0)
    R.ram_step_point4(rows, a, dev(wl.v0), dvt, wl.dt, 3, 10)
    b = dev(wl.q0)
    for _ in range(10):
        R.ram_step_point4(rows, b, dev(wl.v0), dvt, wl.dt, 3, 1)
    torch.cuda.synchronize()
    assert float((a - b).abs().max()) <= 1e-13 * float(b.abs().max())


def test_step_point4_fp32_direct():
    wl = W.small_polar(6, 2600)
    import dataclasses
    w32 = dataclasses.replace(wl, q0=f32(wl.q0), dv=f32(wl.dv))
    want = _oracle_point4(w32, w32.q0, 3)
    got = _gpu_point4(w32, 3, dtype=torch.float32, scan=R.RAM_SUM_DIRECT)[0]
    assert rel_l1(got, want) <= 1e-6


@pytest.fixture(scope="module")
def big():
    return W.cfg5()


@pytest.mark.parametrize("use_density", [False, True])
def test_step_point4_full_size(big, use_density):
    wl = big
    rows = R.Rows.from_workload(wl, DEV)
    ctx = R.context(0)
    if use_density:
        ctx.set_mesh_density(wl.meta["bump"], -np.pi, np.pi)
    try:
        q0 = dev(wl.q0, torch.float32)
        v0, dv = dev(wl.v0), dev(wl.dv, torch.float32)
        n = 4
        a = q0.clone()
        ctx.ram_step_point4(rows, a, v0, dv, wl.dt, 5, n, R.RAM_SUM_DIRECT)
        b = q0.clone()
        t = torch.empty_like(b)
        for _ in range(n):
            ctx.ram_cell_average(rows, b, t, False)
            ctx.ram_step(rows, t, v0, dv, wl.dt, 5, 1, R.RAM_SUM_DIRECT)
            ctx.ram_cell_average(rows, t, b, True)
        torch.cuda.synchronize()
        assert float((a - b).abs().max()) <= 1e-6 * float(b.abs().max())
        # sampled rows against the oracle, one step from FP32-rounded inputs
        pick = np.array([0, 1020, 1024, 2047])
        one = q0.clone()
        ctx.ram_step_point4(rows, one, v0, dv, wl.dt, 5, 1, R.RAM_SUM_DIRECT)
        torch.cuda.synchronize()
        got = one.cpu().numpy().astype(np.float64).reshape(wl.n_rows, -1)[pick]
        n_c = wl.n_cols
        sub = oracle.Rows(np.arange(len(pick) + 1) * n_c, wl.edges, True)
        q_s = f32(wl.q0[pick])
        avg = oracle.average4(sub, q_s)
        avg = oracle.step(sub, avg, wl.v0[pick], f32(wl.dv[pick]), wl.dt, 5, 1)
        want = oracle.point4(sub, avg).reshape(len(pick), -1)
        assert rel_l1(got, want) <= 1e-6
    finally:
        ctx.set_mesh_density(None)


def _f(x):
    return np.sin(x) + 0.3 * np.cos(3.0 * x)


def test_fourth_order_against_exact_solution():
    """Shift by 0.2137 of the period, order 5, FP64, no residual, on a
    smoothly stretched mesh of 64..512 cells: error against the exact
    shifted centre values."""
    s = 0.2137 * 2.0 * math.pi
    e4, e2 = [], []
    for n in (64, 128, 256, 512):
        xi = np.linspace(-math.pi, math.pi, n + 1)
        x = xi + 0.5 * np.sin(xi)
        x[0], x[-1] = -math.pi, math.pi
        c = 0.5 * (x[1:] + x[:-1])
        rows = R.Rows(torch.as_tensor(x, dtype=torch.float64, device=DEV), 1, n, None, True)
        v0 = torch.ones(1, dtype=torch.float64, device=DEV)
        want = _f(c - s)
        a = dev(_f(c))
        R.ram_step_point4(rows, a, v0, None, s, 5, 1)
        b = dev(_f(c))
        R.ram_step(rows, b, v0, None, s, 5, 1, R.RAM_SCAN_F64)
        torch.cuda.synchronize()
        e4.append(np.max(np.abs(a.cpu().numpy() - want)))
        e2.append(np.max(np.abs(b.cpu().numpy() - want)))
    o4 = [math.log2(e4[i] / e4[i + 1]) for i in range(3)]
    o2 = [math.log2(e2[i] / e2[i + 1]) for i in range(3)]
    assert min(o4) >= 3.9, o4
    assert max(o2) <= 2.1, o2
