"""The mesh-density index (closed-form source cell, paper Section 3.2.1 and
App. B) on the GPU.

* the closed form alone (ram_mesh_density_cells) puts every cell centre of the
  periodic-bump mesh in its own cell and every node within one cell of its
  index: the device formula reproduces the mesh generator's F;
* a step with the index agrees with the bucket-index step of the same
  general kernel (schedule 4) to rounding (the same source cells; the kernel
  variant is compiled on its own): 1e-15
  relative L1 in FP64, 1e-7 in FP32, with and without the residual, one step
  and a captured multi-step loop, the 2048 x 16384 disk too; and it matches
  the oracle to 1e-12;
* wrong parameters give the same results (the cell is checked against the
  nodes), and invalid parameters are rejected.
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


def rel_l1(a, b):
    return float(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=dtype, device=DEV)


@pytest.fixture
def ctx():
    c = R.context(0)
    yield c
    c.set_mesh_density(None)
    c.set_schedule(0)


def test_closed_form_matches_mesh(ctx):
    for n in (300, 2048, 16384):
        wl = W.polar(2, n, 2, 5, 1)
        e = wl.edges
        bump = wl.meta["bump"]
        xc = dev(0.5 * (e[:-1] + e[1:]))
        cells = ctx.mesh_density_cells(bump, -math.pi, math.pi, n, xc).cpu().numpy()
        assert np.array_equal(cells, np.arange(n)), n
        cn = ctx.mesh_density_cells(bump, -math.pi, math.pi, n, dev(e[:-1])).cpu().numpy()
        assert np.all(np.abs(cn - np.arange(n)) <= 1), n


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_density_step_equals_bucket_step(ctx, dtype):
    wl = W.small_polar(4, 3000)
    rows = R.Rows.from_workload(wl, DEV)
    v0, dv = dev(wl.v0), dev(wl.dv, dtype)
    bump = wl.meta["bump"]
    for steps, dvv in ((1, dv), (5, dv), (6, None)):
        ref = dev(wl.q0, dtype)
        ctx.set_mesh_density(None)
        ctx.set_schedule(4)          # the general kernel the index variant belongs to
        ctx.ram_step(rows, ref, v0, dvv, wl.dt, 5, steps, R.RAM_SUM_DIRECT)
        ctx.set_schedule(0)
        for params in (bump, (bump[0], bump[1], 0.5 * bump[2])):   # right, then wrong c
            ctx.set_mesh_density(params, -math.pi, math.pi)
            q = dev(wl.q0, dtype)
            ctx.ram_step(rows, q, v0, dvv, wl.dt, 5, steps, R.RAM_SUM_DIRECT)
            torch.cuda.synchronize()
            err = rel_l1(q.cpu().numpy().astype(np.float64), ref.cpu().numpy().astype(np.float64))
            assert err <= (1e-15 if dtype == torch.float64 else 1e-7), (steps, params, err)
    if dtype == torch.float64:
        ctx.set_mesh_density(bump, -math.pi, math.pi)
        q = dev(wl.q0)
        ctx.ram_step(rows, q, v0, dv, wl.dt, 5, 3, R.RAM_SUM_DIRECT)
        want = oracle.step(oracle.Rows.from_workload(wl), wl.q0, wl.v0, wl.dv, wl.dt, 5, 3)
        got = q.cpu().numpy()
        assert np.sum(np.abs(got - want)) / np.sum(np.abs(want)) <= 1e-12


def test_density_step_full_size(ctx):
    wl = W.cfg5()
    rows = R.Rows.from_workload(wl, DEV)
    v0 = dev(wl.v0)
    dv = dev(wl.dv.astype(np.float32), torch.float32)
    q0 = dev(wl.q0.astype(np.float32), torch.float32)
    ref = q0.clone()
    ctx.set_schedule(4)
    ctx.ram_step(rows, ref, v0, dv, wl.dt, 5, 2, R.RAM_SUM_DIRECT)
    ctx.set_schedule(0)
    ctx.set_mesh_density(wl.meta["bump"], -math.pi, math.pi)
    q = q0.clone()
    ctx.ram_step(rows, q, v0, dv, wl.dt, 5, 2, R.RAM_SUM_DIRECT)
    torch.cuda.synchronize()
    err = rel_l1(q.cpu().numpy().astype(np.float64), ref.cpu().numpy().astype(np.float64))
    assert err <= 1e-7, err


def test_density_rejects_bad_parameters(ctx):
    for bump, lo, hi in (((0.3, 0.2, 9.0), -math.pi, math.pi),     # a > b
                         ((0.2, 0.3, -2.0), -math.pi, math.pi),    # c <= -1
                         ((0.2, 4.0, 9.0), -math.pi, math.pi)):    # b beyond the period
        with pytest.raises(R.RamError):
            ctx.set_mesh_density(bump, lo, hi)
