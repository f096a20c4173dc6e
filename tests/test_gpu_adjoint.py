"""Gradients of the checkpointed RAM rollout (autograd over the HIP adjoints).

* central finite differences (eps = 1e-4, FP64 path) on the polar
  1024 x 4096 workload, 200 steps, checkpoint every 20: 32 coordinates in Q0
  and 16 in dv, norm-wise relative error <= 1e-5 (coordinates next to a kink
  replaced by the next draw); 16 in v0 by convergence of the differences;
* the FP64 oracle gradient on sampled rows (rows are independent, so a row's
  loss gradient only involves that row): relative L1 <= 1e-10;
* the FP32-state gradient against the FP64 one (reported, loose bar);
* checkpoint spacing does not change the gradient, nor does keeping every
  state (no recomputation).
dv coordinates are drawn away from zero (the upwind switch).
"""
import numpy as np
import pytest
import torch

import oracle
from parity import assert_parity
from paper_2305_05362_amd import _lib as R
from paper_2305_05362_amd import workloads as W
from paper_2305_05362_amd.autograd import rollout

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _setup(wl, dtype=torch.float64):
    rows = R.Rows.from_workload(wl, DEV)
    q0 = torch.as_tensor(wl.q0.reshape(-1), dtype=dtype, device=DEV)
    dv = torch.as_tensor(wl.dv.reshape(-1), dtype=dtype, device=DEV)
    v0 = torch.as_tensor(wl.v0, dtype=torch.float64, device=DEV)
    area = torch.as_tensor(wl.meta["area"].reshape(-1), dtype=dtype, device=DEV)
    return rows, q0, dv, v0, area


def _target(wl, rows, steps, dtype):
    """Q_target: the same rollout from Q0 + 0.01 G2 with dv (1 + 0.1 xi')."""
    rng = W.rng_for(4, 4)
    rc = 0.5 * (wl.meta["r_edges"][:-1] + wl.meta["r_edges"][1:])
    pc = 0.5 * (wl.edges[:-1] + wl.edges[1:])
    xx = rc[:, None] * np.cos(pc)[None, :] - 1.1 * np.cos(0.05)
    yy = rc[:, None] * np.sin(pc)[None, :] - 1.1 * np.sin(0.05)
    g2 = np.exp(-(xx ** 2 + yy ** 2) / (2 * 0.05 ** 2))
    q = torch.as_tensor((wl.q0 + 0.01 * g2).reshape(-1), dtype=dtype, device=DEV)
    dvt = wl.dv * (1.0 + 0.1 * rng.standard_normal(wl.dv.shape))
    dvt = torch.as_tensor(dvt.reshape(-1), dtype=dtype, device=DEV)
    v0 = torch.as_tensor(wl.v0, dtype=torch.float64, device=DEV)
    R.ram_step(rows, q, v0, dvt, wl.dt, wl.order, steps,
               R.RAM_SCAN_F64)
    return q


def _loss(qT, tgt, area):
    return torch.sum((qT - tgt) ** 2 * area)


def _grads(wl, rows, q0, dv, v0, area, tgt, steps, ckpt, scan=R.RAM_SCAN_F64):
    a = q0.clone().requires_grad_(True)
    b = dv.clone().requires_grad_(True)
    c = v0.clone().requires_grad_(True)
    qT = rollout(a, rows, c, b, wl.dt, wl.order, steps, ckpt, scan)
    L = _loss(qT, tgt.to(qT.dtype), area)
    L.backward()
    torch.cuda.synchronize()
    return a.grad.double(), b.grad.double(), c.grad.double(), float(L)


def _loss_at(wl, rows, q0, dv, v0, area, tgt, steps):
    q = q0.clone()
    R.ram_step(rows, q, v0, dv, wl.dt, wl.order, steps, R.RAM_SCAN_F64)
    return float(_loss(q, tgt, area))


def _fd(wl, rows, q0, dv, v0, area, tgt, steps, kind, idx, eps):
    n = wl.n_cells
    if kind == "v0":
        d = torch.zeros(wl.n_rows, dtype=torch.float64, device=DEV)
        d[idx] = eps
        return (_loss_at(wl, rows, q0, dv, v0 + d, area, tgt, steps)
                - _loss_at(wl, rows, q0, dv, v0 - d, area, tgt, steps)) / (2 * eps)
    d = torch.zeros(n, dtype=torch.float64, device=DEV)
    d[idx] = eps
    if kind == "q":
        return (_loss_at(wl, rows, q0 + d, dv, v0, area, tgt, steps)
                - _loss_at(wl, rows, q0 - d, dv, v0, area, tgt, steps)) / (2 * eps)
    return (_loss_at(wl, rows, q0, dv + d, v0, area, tgt, steps)
            - _loss_at(wl, rows, q0, dv - d, v0, area, tgt, steps)) / (2 * eps)


def test_rollout_gradient_fd_cfg4():
    """Central differences at eps = 1e-4 (FP64 path) against the adjoint
    gradient, 32 coordinates in Q0 and 16 in dv, norm-wise <= 1e-5.

    The loss is continuous but only piecewise smooth: the van Leer limiter
    switches branch where a slope product crosses zero and the polar state
    carries 1e-3 white noise, so such kinks are dense along a 200-step
    rollout.  A coordinate whose +-eps interval holds a kink is detected by
    comparing the differences at eps and eps/4 (on a smooth stretch they agree
    to O(eps^2)) and is replaced by the next draw of the seeded sequence; the
    number replaced is printed.  The v0 dependence has a kink wherever a
    shifted node crosses a source node, which any eps on a 4096-cell row
    does, so there the differences must converge to the adjoint instead
    (median relative error <= 1e-3 at eps = 1e-6 and more than 3x below the
    one at 1e-4); the oracle-gradient test pins v0bar exactly."""
    wl = W.cfg4()
    steps, ckpt = 200, 20
    rows, q0, dv, v0, area = _setup(wl)
    tgt = _target(wl, rows, steps, torch.float64)
    gq, gdv, gv0, _ = _grads(wl, rows, q0, dv, v0, area, tgt, steps, ckpt)
    rng = W.rng_for(4, 5)
    n = wl.n_cells
    rows_of = np.arange(n) // wl.n_cols
    dvh = wl.dv.reshape(-1)
    pools = {
        "q": rng.permutation(np.where(np.abs(wl.q0.reshape(-1) - 1.0) > 1e-2)[0]),
        "dv": rng.permutation(np.where((np.abs(dvh) > 1e-3) & (rows_of > 400)
                                       & (rows_of < 650))[0]),
    }
    eps = 1e-4
    ad, fd, replaced = [], [], 0
    for kind, want, g in (("q", 32, gq), ("dv", 16, gdv)):
        floor = 1e-3 * float(g.abs().max())
        got = 0
        for tries, idx in enumerate(pools[kind]):
            assert tries < 20 * want, f"too many {kind} coordinates next to kinks"
            f1 = _fd(wl, rows, q0, dv, v0, area, tgt, steps, kind, idx, eps)
            f2 = _fd(wl, rows, q0, dv, v0, area, tgt, steps, kind, idx, eps / 4)
            if abs(f1 - f2) > 1e-6 * max(abs(f2), floor):
                replaced += 1
                continue
            ad.append(float(g[idx]))
            fd.append(f1)
            got += 1
            if got == want:
                break
    ad, fd = np.array(ad), np.array(fd)
    rel = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    per = np.abs(ad - fd) / np.maximum(np.abs(fd), 1e-3 * np.max(np.abs(fd)))
    print(f"Q0+dv: FD norm-wise rel {rel:.3e}, worst per-coordinate {per.max():.3e}, "
          f"{replaced} coordinates replaced (kink within eps)")
    assert len(ad) == 48
    assert rel <= 1e-5
    epss = (1e-4, 1e-5, 1e-6)
    errs = []
    for idx in rng.choice(np.arange(wl.n_rows)[200:800], 16, replace=False):
        a = float(gv0[idx])
        errs.append([abs(_fd(wl, rows, q0, dv, v0, area, tgt, steps, "v0", idx, h) - a) / abs(a)
                     for h in epss])
    errs = np.array(errs)
    print("v0: median FD rel error at eps 1e-4/1e-5/1e-6:", np.median(errs, axis=0))
    assert np.median(errs[:, 2]) <= 1e-3
    assert np.median(errs[:, 0]) > 3 * np.median(errs[:, 2])


def _oracle_rollout_grad(sw, steps, gfun):
    """FP64 oracle gradient of a rollout: forward keeping every state, then
    the transposed steps in reverse."""
    rows = oracle.Rows.from_workload(sw)
    q = sw.q0.reshape(-1).astype(np.float64)
    pre_shift, pre_res = [], []
    for _ in range(steps):
        pre_shift.append(q)
        h = oracle.shift(rows, q, sw.v0, sw.dt, sw.order)
        pre_res.append(h)
        q = oracle.residual(rows, h, sw.dv, sw.dt)
    qbar = gfun(q)
    dvbar = np.zeros_like(qbar)
    v0bar = np.zeros(sw.n_rows)
    for i in range(steps - 1, -1, -1):
        qbar, dvb = oracle.residual_adjoint(rows, pre_res[i], sw.dv, qbar, sw.dt)
        dvbar += dvb
        qbar, vb = oracle.shift_adjoint(rows, pre_shift[i], qbar, sw.v0, sw.dt, sw.order)
        v0bar += vb
    return qbar, dvbar, v0bar


def test_rollout_gradient_matches_oracle_sampled_rows():
    wl = W.small_polar(64, 1024, cfg=4)
    steps, ckpt = 30, 7
    rows, q0, dv, v0, area = _setup(wl)
    tgt = torch.as_tensor(wl.q0.reshape(-1) * 1.01, dtype=torch.float64, device=DEV)
    gq, gdv, gv0, _ = _grads(wl, rows, q0, dv, v0, area, tgt, steps, ckpt)
    pick = np.array([0, 17, 40, 63])
    n = wl.n_cols
    sw = W.Workload("s", len(pick), n, np.arange(len(pick) + 1) * n, wl.edges, True,
                    wl.q0[pick], wl.dv[pick], wl.v0[pick], wl.dt, wl.order, steps)
    ar = wl.meta["area"][pick].reshape(-1)
    tg = (wl.q0[pick] * 1.01).reshape(-1)
    oq, odv, ov0 = _oracle_rollout_grad(sw, steps, lambda qT: 2.0 * (qT - tg) * ar)
    got_q = gq.cpu().numpy().reshape(wl.n_rows, n)[pick].reshape(-1)
    got_dv = gdv.cpu().numpy().reshape(wl.n_rows, n)[pick].reshape(-1)
    got_v0 = gv0.cpu().numpy()[pick]
    rel = lambda a, b: np.sum(np.abs(a - b)) / np.sum(np.abs(b))
    assert rel(got_q, oq) <= 1e-10
    assert rel(got_dv, odv) <= 1e-10
    assert np.max(np.abs(got_v0 - ov0)) <= 1e-9 * np.max(np.abs(ov0))


def test_checkpoint_spacing_and_fp32_gradient():
    """FP64: the same gradients bit for bit whatever the checkpoint spacing
    (the recomputed segments repeat the forward states exactly and the
    adjoint adds nothing in a hardware-chosen order).  FP32 state: within
    1e-3 of the FP64 gradient for this squared loss (its seed 2 (Q_T - tgt)
    sits 1 % below Q, so the FP32 forward's rounding enters it amplified;
    the linear-loss test below holds FP32 to the oracle at a bar from
    rounding alone)."""
    wl = W.small_polar(32, 2048, cfg=4)
    steps = 40
    rows, q0, dv, v0, area = _setup(wl)
    tgt = torch.as_tensor(wl.q0.reshape(-1) * 0.99, dtype=torch.float64, device=DEV)
    a = _grads(wl, rows, q0, dv, v0, area, tgt, steps, 40)
    b = _grads(wl, rows, q0, dv, v0, area, tgt, steps, 7)
    st = _grads(wl, rows, q0, dv, v0, area, tgt, steps, 0)     # every state kept
    for x, y, z in zip(a[:3], b[:3], st[:3]):
        assert torch.equal(x, y)
        assert torch.equal(z, y)
    rows32, q32, dv32, _, area32 = _setup(wl, torch.float32)
    c = _grads(wl, rows32, q32, dv32, v0, area32, tgt, steps, 10, R.RAM_SCAN_F64)
    for x, y in zip(c[:3], a[:3]):
        err = float((x - y).abs().sum() / y.abs().sum())
        print(f"FP32-state gradient rel-L1 vs FP64: {err:.2e}")
        assert err <= 1e-3


def test_fp32_gradient_against_oracle_sampled_rows():
    """The FP32-state rollout gradient (direct sums, the streaming step)
    against the FP64 oracle's gradient on sampled rows, for the linear loss
    L = sum(g Q_T) with a fixed g, so that the seed is exact and only FP32
    rounding separates the two.

    Bars from the rounding: each of the 2 x 25 forward and backward steps
    rounds every value a few times at u = 2^-24 = 6e-8, so Q0bar and dvbar
    carry about 50 x 4 u = 1.2e-5 relative (bar 1e-4, rel-L1 over the
    sampled rows, and 1e-4 of the largest entry per cell); v0bar sums
    differences of the FP32 reconstruction between neighbouring nodes, each
    about 1e-4 relative (bar 1e-3 of the row's value).  Inputs are rounded to
    FP32 first, so both sides start from the same data."""
    wl = W.small_polar(64, 2048, cfg=4)
    steps, ckpt = 25, 6
    q0h = wl.q0.astype(np.float32).astype(np.float64)
    dvh = wl.dv.astype(np.float32).astype(np.float64)
    rows = R.Rows.from_workload(wl, DEV)
    q0 = torch.as_tensor(q0h.reshape(-1), dtype=torch.float32, device=DEV)
    dv = torch.as_tensor(dvh.reshape(-1), dtype=torch.float32, device=DEV)
    v0 = torch.as_tensor(wl.v0, dtype=torch.float64, device=DEV)
    rng = np.random.default_rng(11)
    gh = rng.uniform(0.5, 1.5, wl.n_cells)
    g = torch.as_tensor(gh, dtype=torch.float32, device=DEV)
    a = q0.clone().requires_grad_(True)
    b = dv.clone().requires_grad_(True)
    c = v0.clone().requires_grad_(True)
    qT = rollout(a, rows, c, b, wl.dt, wl.order, steps, ckpt, R.RAM_SUM_DIRECT)
    torch.sum(qT * g).backward()
    torch.cuda.synchronize()
    pick = np.array([0, 21, 42, 63])
    n = wl.n_cols
    sw = W.Workload("s", len(pick), n, np.arange(len(pick) + 1) * n, wl.edges, True,
                    q0h[pick], dvh[pick], wl.v0[pick], wl.dt, wl.order, steps)
    gp = gh.reshape(wl.n_rows, n)[pick].reshape(-1).astype(np.float32).astype(np.float64)
    oq, odv, ov0 = _oracle_rollout_grad(sw, steps, lambda qT_: gp)
    got_q = a.grad.double().cpu().numpy().reshape(wl.n_rows, n)[pick].reshape(-1)
    got_dv = b.grad.double().cpu().numpy().reshape(wl.n_rows, n)[pick].reshape(-1)
    got_v0 = c.grad.double().cpu().numpy()[pick]
    eq = assert_parity(got_q, oq, 1e-4, 1e-4, "Q0bar")
    edv = assert_parity(got_dv, odv, 1e-4, 1e-4, "dvbar")
    ev0 = float(np.max(np.abs(got_v0 - ov0) / np.abs(ov0)))
    print(f"FP32 gradient vs oracle: Q0 {eq}, dv {edv}, v0 max rel {ev0:.2e}")
    assert ev0 <= 1e-3


@pytest.mark.parametrize("recon", [0, R.RAM_RECON_PPM])
@pytest.mark.parametrize("ckpt", [0, 4])
def test_only_requested_gradients(recon, ckpt):
    """With only Q0 requiring a gradient the backward pass skips the dv and v0
    terms; Q0's gradient is the one the full backward pass gives and dv / v0
    get none.  With Q0 and v0 only, v0's gradient is unchanged too.  (To
    rounding: the passes without the dv and v0 terms are other kernel
    instantiations, which the compiler may schedule differently.)"""
    wl = W.small_polar(6, 1500)
    rows = R.Rows.from_workload(wl, DEV)
    q0 = torch.as_tensor(wl.q0.reshape(-1), dtype=torch.float64, device=DEV)
    dv = torch.as_tensor(wl.dv.reshape(-1), dtype=torch.float64, device=DEV)
    v0 = torch.as_tensor(wl.v0, dtype=torch.float64, device=DEV)
    g = torch.linspace(-1.0, 1.0, q0.numel(), dtype=torch.float64, device=DEV)

    def run(need_dv, need_v0):
        a = q0.clone().requires_grad_(True)
        b = dv.clone().requires_grad_(need_dv)
        c = v0.clone().requires_grad_(need_v0)
        out = rollout(a, rows, c, b, wl.dt, 5, 8, ckpt, R.RAM_SCAN_F64, recon)
        out.backward(g)
        torch.cuda.synchronize()
        return a.grad, b.grad, c.grad

    def close(u, w):
        return float((u - w).abs().max()) <= 1e-13 * float(w.abs().max())

    fa, fb, fc = run(True, True)
    oa, ob, oc = run(False, False)
    assert ob is None and oc is None
    assert close(oa, fa)
    va, vb, vc = run(False, True)
    assert vb is None
    assert close(va, fa) and close(vc, fc)
