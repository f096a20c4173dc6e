"""The differentiable rollout with the limited (PLM / PPM) shift.

* ram_step_limited_record: every recorded state equals ram_step_limited's bit
  for bit (shared mesh: the fused kernel; per-row meshes: shift kernel, then
  residual kernel), and the recorded post-shift states are the shift's;
* rollout(..., recon=...) gradients w.r.t. Q0, dv and v0 against the FP64
  oracle's reverse pass (forward keeping every state, then the residual
  adjoint and the limited shift adjoint per step), with checkpoints every 7
  steps and with every state kept, relative L1 <= 1e-9;
* central differences (FP64, eps = 1e-6) on Q0 and dv coordinates, a
  coordinate whose interval holds a limiter switch (differences at eps and
  eps/4 disagree) replaced by the next draw, norm-wise <= 1e-5.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2305_05362_amd import _lib as R
from paper_2305_05362_amd import workloads as W
from paper_2305_05362_amd.autograd import rollout

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
RECONS = [R.RAM_RECON_PLM, R.RAM_RECON_PPM]


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=dtype, device=DEV)


def rel_l1(a, b):
    return float(np.sum(np.abs(a - b)) / np.sum(np.abs(b)))


@pytest.mark.parametrize("recon", RECONS)
@pytest.mark.parametrize("kind", ["polar", "ragged"])
def test_limited_record_matches_step(kind, recon):
    wl = W.small_polar(3, 3500) if kind == "polar" else W.small_ragged(12, 6, 2600, seed=31)
    rows = R.Rows.from_workload(wl, DEV)
    k = 4
    traj = torch.empty((k + 1, wl.n_cells), dtype=torch.float64, device=DEV)
    half = torch.empty((k, wl.n_cells), dtype=torch.float64, device=DEV)
    traj[0] = dev(wl.q0)
    v0, dv = dev(wl.v0), dev(wl.dv)
    R.context(0).ram_step_limited_record(rows, traj, half, v0, dv, wl.dt, recon, k)
    q = dev(wl.q0)
    for i in range(k):
        R.ram_step_limited(rows, q, v0, dv, wl.dt, recon, 1)
        torch.cuda.synchronize()
        assert torch.equal(q, traj[i + 1]), i
        h = torch.empty_like(q)
        R.ram_shift_limited(rows, traj[i], h, v0, wl.dt, recon)
        torch.cuda.synchronize()
        assert torch.equal(h, half[i]), i


def _oracle_grad(wl, steps, w, recon):
    rows = oracle.Rows.from_workload(wl)
    q = wl.q0.reshape(-1).astype(np.float64)
    pre_shift, pre_res = [], []
    for _ in range(steps):
        pre_shift.append(q)
        h = oracle.shift_recon(rows, q, wl.v0, wl.dt, recon)
        pre_res.append(h)
        q = oracle.residual(rows, h, wl.dv, wl.dt)
    qbar = 2.0 * q * w
    dvbar = np.zeros_like(qbar)
    v0bar = np.zeros(wl.n_rows)
    for i in range(steps - 1, -1, -1):
        qbar, dvb = oracle.residual_adjoint(rows, pre_res[i], wl.dv, qbar, wl.dt)
        dvbar += dvb
        qbar, vb = oracle.shift_recon_adjoint(rows, pre_shift[i], qbar, wl.v0, wl.dt, recon)
        v0bar += vb
    return qbar, dvbar, v0bar


def _gpu_grad(wl, rows, steps, ckpt, w, recon):
    q0 = dev(wl.q0).requires_grad_(True)
    dv = dev(wl.dv).requires_grad_(True)
    v0 = dev(wl.v0).requires_grad_(True)
    out = rollout(q0, rows, v0, dv, wl.dt, 5, steps, ckpt, recon=recon)
    loss = (out * out * dev(w)).sum()
    loss.backward()
    torch.cuda.synchronize()
    return (q0.grad.cpu().numpy(), dv.grad.cpu().numpy(), v0.grad.cpu().numpy(),
            float(loss))


@pytest.mark.parametrize("recon", RECONS)
def test_limited_rollout_gradient_matches_oracle(recon):
    wl = W.small_polar(24, 1024, cfg=4)
    rows = R.Rows.from_workload(wl, DEV)
    rng = np.random.default_rng(3)
    w = rng.uniform(0.5, 1.5, wl.n_cells)
    steps = 20
    ref = _oracle_grad(wl, steps, w, recon)
    for ckpt in (7, 0):
        got = _gpu_grad(wl, rows, steps, ckpt, w, recon)
        assert rel_l1(got[0], ref[0]) <= 1e-9, ckpt
        assert rel_l1(got[1], ref[1]) <= 1e-9, ckpt
        assert np.max(np.abs(got[2] - ref[2])) <= 1e-8 * np.max(np.abs(ref[2])), ckpt


@pytest.mark.parametrize("recon", RECONS)
def test_limited_rollout_gradient_fd(recon):
    wl = W.small_polar(16, 512, cfg=4)
    rows = R.Rows.from_workload(wl, DEV)
    rng = np.random.default_rng(9)
    w = rng.uniform(0.5, 1.5, wl.n_cells)
    steps = 15
    gq, gdv, _, _ = _gpu_grad(wl, rows, steps, 5, w, recon)
    wt = dev(w)
    v0 = dev(wl.v0)

    def loss(q0, dv):
        q = q0.clone()
        R.ram_step_limited(rows, q, v0, dv, wl.dt, recon, steps)
        return float((q * q * wt).sum())

    q0, dv0 = dev(wl.q0), dev(wl.dv)

    def fd(kind, idx, eps):
        d = torch.zeros(wl.n_cells, dtype=torch.float64, device=DEV)
        d[idx] = eps
        if kind == "q":
            return (loss(q0 + d, dv0) - loss(q0 - d, dv0)) / (2 * eps)
        return (loss(q0, dv0 + d) - loss(q0, dv0 - d)) / (2 * eps)

    ad, fdv, replaced = [], [], 0
    q_pool = rng.permutation(np.where(np.abs(wl.q0.reshape(-1) - 1.0) > 1e-2)[0])
    dv_pool = rng.permutation(np.where(np.abs(wl.dv.reshape(-1)) > 1e-3)[0])
    for kind, pool, g, want in (("q", q_pool, gq, 12), ("dv", dv_pool, gdv, 6)):
        floor = 1e-3 * float(np.max(np.abs(g)))
        got = 0
        for tries, idx in enumerate(pool):
            assert tries < 20 * want, f"too many {kind} coordinates next to kinks"
            f1, f2 = fd(kind, idx, 1e-6), fd(kind, idx, 2.5e-7)
            if abs(f1 - f2) > 1e-6 * max(abs(f2), floor):
                replaced += 1
                continue
            ad.append(float(g[idx]))
            fdv.append(f1)
            got += 1
            if got == want:
                break
    ad, fdv = np.array(ad), np.array(fdv)
    rel = np.linalg.norm(ad - fdv) / np.linalg.norm(fdv)
    print(f"recon {recon}: FD norm-wise rel {rel:.3e}, {replaced} replaced")
    assert len(ad) == 18 and rel <= 1e-5
