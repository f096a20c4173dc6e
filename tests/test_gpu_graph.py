"""Multi-step calls replay a captured graph of their step loop.

ram_step with n_steps >= 4 captures its ping-pong loop once and replays it
while the arguments stay the same.  Every replay must equal, bit for bit, the
same steps issued one call at a time (which are never captured), with the
program's own eager work and synchronisations between the replays; changing
an argument (dt, the state buffer) must re-capture.
"""
import numpy as np
import pytest
import torch

from paper_2305_05362_amd import _lib as R
from paper_2305_05362_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=dtype, device=DEV)


def _eager(rows, q0, v0, dv, dt, order, steps, scan):
    q = q0.clone()
    for _ in range(steps):
        R.ram_step(rows, q, v0, dv, dt, order, 1, scan)
    return q


@pytest.mark.parametrize("dtype,scan", [(torch.float64, R.RAM_SCAN_F64),
                                        (torch.float32, R.RAM_SCAN_F32_TWOSUM),
                                        (torch.float32, R.RAM_SUM_DIRECT)])
@pytest.mark.parametrize("kind", ["polar", "ragged"])
@pytest.mark.parametrize("steps", [5, 8])
def test_graph_replays_match_eager(kind, steps, dtype, scan):
    wl = W.small_polar(5, 1500) if kind == "polar" else W.small_ragged(9, 6, 2100, seed=3)
    rows = R.Rows.from_workload(wl, DEV)
    q0 = dev(wl.q0, dtype)
    v0 = dev(wl.v0)
    dv = dev(wl.dv, dtype)
    ref = _eager(rows, q0, v0, dv, wl.dt, 5, steps, scan)
    q = q0.clone()
    scratch = torch.empty_like(q0)
    for rep in range(3):
        q.copy_(q0)
        R.ram_step(rows, q, v0, dv, wl.dt, 5, steps, scan)      # replayed after rep 0
        torch.cuda.synchronize()
        assert torch.equal(q, ref), rep
        # eager work of the program between replays
        R.ram_shift(rows, q0, scratch, v0, wl.dt, 5, scan)
        scratch.mul_(0.5)
        torch.cuda.synchronize()
    # a different dt re-captures
    ref2 = _eager(rows, q0, v0, dv, 0.5 * wl.dt, 5, steps, scan)
    q.copy_(q0)
    R.ram_step(rows, q, v0, dv, 0.5 * wl.dt, 5, steps, scan)
    torch.cuda.synchronize()
    assert torch.equal(q, ref2)
    # another state buffer re-captures too
    q2 = q0.clone()
    R.ram_step(rows, q2, v0, dv, wl.dt, 5, steps, scan)
    torch.cuda.synchronize()
    assert torch.equal(q2, ref)
