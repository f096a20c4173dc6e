"""FP64 results do not depend on the run: the same backward pass twice in one
process gives bit-equal gradients.

The adjoint kernels add nothing in an order set by the hardware: each tile's
v0bar term goes to a per-tile slot and a second kernel sums a row's slots in
tile order; the shared-mesh kernel's Cbar scatter runs in ordered passes for
an FP64 state; window cells shared by two neighbouring tiles take exactly two
terms onto a zero (the same sum in either order).  Checked on shared meshes
(polar rows, several tiles a row) and per-row ragged meshes, for the one-step
adjoint with every gradient (Q, dv, v0), the limited (PPM and PLM) shift
adjoint with v0bar, and a checkpointed autograd rollout.
"""
import numpy as np
import pytest
import torch

from paper_2305_05362_amd import _lib as R
from paper_2305_05362_amd import workloads as W
from paper_2305_05362_amd.autograd import rollout

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=dtype, device=DEV)


CASES = {
    "polar": lambda: W.small_polar(48, 4096, order=5),
    "ragged": lambda: W.small_ragged(40, 8, 2600, seed=47, order=5),
}


def _state(wl):
    rows = R.Rows.from_workload(wl, DEV)
    q0, v0, dv = dev(wl.q0), dev(wl.v0), dev(wl.dv)
    rng = np.random.default_rng(5)
    qbar = dev(rng.standard_normal(wl.n_cells))
    return rows, q0, v0, dv, qbar


@pytest.mark.parametrize("kind", list(CASES))
def test_step_adjoint_bitwise_repeatable(kind):
    wl = CASES[kind]()
    rows, q0, v0, dv, qbar = _state(wl)
    half = torch.empty_like(q0)
    R.ram_shift(rows, q0, half, v0, wl.dt, wl.order, R.RAM_SCAN_F64)
    outs = []
    for _ in range(2):
        qb_in = torch.full_like(q0, float("nan"))
        dvb = torch.zeros_like(dv)
        v0b = torch.zeros_like(v0)
        R.context(0).ram_step_adjoint(rows, q0, half, dv, qbar, qb_in, v0, wl.dt, wl.order,
                                      dvb, v0b)
        torch.cuda.synchronize()
        outs.append((qb_in, dvb, v0b))
    for a, b, what in zip(outs[0], outs[1], ("qbar", "dvbar", "v0bar")):
        assert torch.equal(a, b), (kind, what)
    assert bool(torch.isfinite(outs[0][0]).all())
    assert float(outs[0][2].abs().max()) > 0.0


@pytest.mark.parametrize("kind", list(CASES))
@pytest.mark.parametrize("recon", [R.RAM_RECON_PPM, R.RAM_RECON_PLM])
def test_limited_adjoint_bitwise_repeatable(kind, recon):
    wl = CASES[kind]()
    rows, q0, v0, _, qbar = _state(wl)
    outs = []
    for _ in range(2):
        qb_in = torch.full_like(q0, float("nan"))
        v0b = torch.zeros_like(v0)
        R.context(0).ram_shift_limited_adjoint(rows, q0, qbar, qb_in, v0, wl.dt, recon, v0b)
        torch.cuda.synchronize()
        outs.append((qb_in, v0b))
    assert torch.equal(outs[0][0], outs[1][0]), (kind, "qbar")
    assert torch.equal(outs[0][1], outs[1][1]), (kind, "v0bar")


@pytest.mark.parametrize("kind", list(CASES))
def test_rollout_gradients_bitwise_repeatable(kind):
    wl = CASES[kind]()
    rows, q0, v0, dv, qbar = _state(wl)
    grads = []
    for _ in range(2):
        a = q0.clone().requires_grad_(True)
        b = dv.clone().requires_grad_(True)
        c = v0.clone().requires_grad_(True)
        qT = rollout(a, rows, c, b, wl.dt, wl.order, 12, 4, R.RAM_SCAN_F64)
        torch.sum(qT * qbar).backward()
        torch.cuda.synchronize()
        grads.append((a.grad, b.grad, c.grad))
    for g0, g1, what in zip(grads[0], grads[1], ("q0", "dv", "v0")):
        assert torch.equal(g0, g1), (kind, what)
