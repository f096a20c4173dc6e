"""Launch schedules of the shared-mesh direct-sum step kernel (ram_set_schedule)
and the autotuner that picks one.

* every schedule (0: the FP32 streaming kernel, or the general kernel with
  2..5 shifted nodes per thread) matches the FP64 oracle to
  1e-12 (shift, fused step, several steps, recorded trajectory) and the other
  schedules to rounding (each variant is compiled on its own, so multiply-add
  fusion may differ): 1e-15 relative L1 in FP64, 1e-7 in FP32, including the
  2048 x 16384 disk in FP32; within one schedule the recorded trajectory is
  the step's bit for bit;
* the schedule API rejects other values, 0 (the default) restores it;
* the autotuner times every candidate, leaves the fastest set, and reads a
  cached choice back.
"""
import json

import numpy as np
import pytest
import torch

import oracle
from parity import CELL_F32, CELL_F32_ADJ, CELL_F64, assert_parity
from paper_2305_05362_amd import _lib as R
from paper_2305_05362_amd import tune
from paper_2305_05362_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
ITEMS = (0, 2, 3, 4, 5)


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=dtype, device=DEV)


def rel_l1(a, b):
    return float(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))


@pytest.fixture
def ctx():
    c = R.context(0)
    yield c
    c.set_schedule(0)


def test_schedule_api(ctx):
    assert ctx.get_schedule() == 0
    for k in ITEMS:
        ctx.set_schedule(k)
        assert ctx.get_schedule() == k
    ctx.set_schedule(0)
    assert ctx.get_schedule() == 0
    for bad in (1, 6, -1):
        with pytest.raises(R.RamError):
            ctx.set_schedule(bad)
    assert ctx.get_schedule() == 0


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_schedules_agree_and_match_oracle(ctx, dtype):
    wl = W.small_polar(3, 3500)
    rows = R.Rows.from_workload(wl, DEV)
    orows = oracle.Rows.from_workload(wl)
    v0, dv = dev(wl.v0), dev(wl.dv, dtype)
    outs = {}
    for k in ITEMS:
        ctx.set_schedule(k)
        q = dev(wl.q0, dtype)
        ctx.ram_step(rows, q, v0, dv, wl.dt, 5, 3, R.RAM_SUM_DIRECT)
        h = torch.empty_like(q)
        ctx.ram_shift(rows, dev(wl.q0, dtype), h, v0, wl.dt, 5, R.RAM_SUM_DIRECT)
        traj = torch.empty((3, wl.n_cells), dtype=dtype, device=DEV)
        half = torch.empty((2, wl.n_cells), dtype=dtype, device=DEV)
        traj[0] = dev(wl.q0, dtype)
        ctx.ram_step_record(rows, traj, half, v0, dv, wl.dt, 5, 2, R.RAM_SUM_DIRECT)
        torch.cuda.synchronize()
        outs[k] = (q.clone(), h.clone(), traj.clone(), half.clone())
    # schedules of the general kernel agree to rounding; in FP32 the streaming
    # kernel (schedule 0) forms a uniform run's stencil weights once in FP64
    # where the general kernel forms them per tile in FP32, so it is held to
    # the oracle instead (below)
    tol = 1e-15 if dtype == torch.float64 else 1e-7
    for k in ITEMS:
        if k == 0 and dtype == torch.float32:
            continue
        for a, b in zip(outs[k], outs[4]):
            err = rel_l1(a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64))
            assert err <= tol, (k, err)
        # the recorded trajectory's second state is the 2-step result of the
        # same schedule (ram_step over 3 steps is checked against the oracle)
    if dtype == torch.float32:
        q32 = wl.q0.astype(np.float32).astype(np.float64)
        dv32 = wl.dv.astype(np.float32).astype(np.float64)
        ref3 = oracle.step(orows, q32, wl.v0, dv32, wl.dt, 5, 3)
        refs = oracle.shift(orows, q32, wl.v0, wl.dt, 5)
        for k in ITEMS:
            assert_parity(outs[k][0].cpu().numpy(), ref3, 1e-6, CELL_F32, what=f"step {k}")
            assert_parity(outs[k][1].cpu().numpy(), refs, 1e-6, CELL_F32, what=f"shift {k}")
    if dtype == torch.float64:
        ref3 = oracle.step(orows, wl.q0, wl.v0, wl.dv, wl.dt, 5, 3)
        ref2 = oracle.step(orows, wl.q0, wl.v0, wl.dv, wl.dt, 5, 2)
        refs = oracle.shift(orows, wl.q0, wl.v0, wl.dt, 5)
        for k in ITEMS:
            assert_parity(outs[k][0].cpu().numpy(), ref3, 1e-12, CELL_F64, what=str(k))
            assert_parity(outs[k][1].cpu().numpy(), refs, 1e-12, CELL_F64, what=str(k))
            assert_parity(outs[k][2][2].cpu().numpy(), ref2, 1e-12, CELL_F64, what=str(k))


def test_record_is_step_within_a_schedule(ctx):
    wl = W.small_polar(3, 3500)
    rows = R.Rows.from_workload(wl, DEV)
    v0, dv = dev(wl.v0), dev(wl.dv, torch.float32)
    for k in (0, 2, 5):
        ctx.set_schedule(k)
        traj = torch.empty((3, wl.n_cells), dtype=torch.float32, device=DEV)
        half = torch.empty((2, wl.n_cells), dtype=torch.float32, device=DEV)
        traj[0] = dev(wl.q0, torch.float32)
        ctx.ram_step_record(rows, traj, half, v0, dv, wl.dt, 5, 2, R.RAM_SUM_DIRECT)
        q = dev(wl.q0, torch.float32)
        for i in range(2):
            ctx.ram_step(rows, q, v0, dv, wl.dt, 5, 1, R.RAM_SUM_DIRECT)
            torch.cuda.synchronize()
            assert torch.equal(q, traj[i + 1]), (k, i)


def test_schedules_agree_full_size(ctx):
    wl = W.cfg5()
    rows = R.Rows.from_workload(wl, DEV)
    v0 = dev(wl.v0)
    dv = dev(wl.dv.astype(np.float32), torch.float32)
    q0 = dev(wl.q0.astype(np.float32), torch.float32)
    got = {}
    for k in (4, 5, 3, 0):
        ctx.set_schedule(k)
        q = q0.clone()
        ctx.ram_step(rows, q, v0, dv, wl.dt, 5, 2, R.RAM_SUM_DIRECT)
        torch.cuda.synchronize()
        got[k] = q
    base = got[4].cpu().numpy().astype(np.float64)
    for k in (5, 3):
        assert rel_l1(got[k].cpu().numpy().astype(np.float64), base) <= 1e-7, k
    # the streaming kernel: FP64-formed uniform weights, so within FP32
    # rounding of the others rather than bit-near
    assert rel_l1(got[0].cpu().numpy().astype(np.float64), base) <= 1e-6


def test_autotuner_picks_and_caches(ctx, tmp_path):
    wl = W.small_polar(16, 4096)
    rows = R.Rows.from_workload(wl, DEV)
    q = dev(wl.q0, torch.float32)
    dv = dev(wl.dv, torch.float32)
    v0 = dev(wl.v0)
    cache = str(tmp_path / "sched.json")
    best, us, cached = tune.tuned_schedule(ctx, rows, q, v0, dv, wl.dt, 5,
                                           cache_path=cache, steps=8, reps=2)
    assert not cached and best in ITEMS and sorted(us) == list(ITEMS)
    assert us[best] == min(us.values()) and ctx.get_schedule() == best
    ctx.set_schedule(0)
    best2, us2, cached2 = tune.tuned_schedule(ctx, rows, q, v0, dv, wl.dt, 5, cache_path=cache)
    assert cached2 and best2 == best and ctx.get_schedule() == best
    with open(cache) as fh:
        assert list(json.load(fh).values())[0]["items"] == best
