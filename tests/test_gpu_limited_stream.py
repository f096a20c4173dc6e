"""The streaming limited adjoint (FP32 state, shared mesh, rows of a multiple
of four cells: k_ladj on the tile plan of the reconstruction's stencil width)
against the FP64 oracle's transposed Jacobian of the limited shift (Section
3.1's PLM and PPM reconstructions, each limiter differentiated on the branch
it takes), and composed with the residual's transpose (ram_step_limited_adjoint);
the general kernels (schedule 4) on the same inputs and bars.

Bars.  The shift's transpose alone: those of test_gpu_limited_adjoint.py's
FP32 case (rel-L1 1e-6, per cell CELL_F32, v0bar 1e-10 of the largest): the
Jacobian rows are FP64 at FP64 positions, so only the final rounding to FP32
and the FP64 accumulation order differ from the oracle.  With the residual:
those of the FP32 step adjoint (rel-L1 1e-5, per cell CELL_F32_ADJ), the
residual's transpose running in FP32, and v0bar within 1e-5 of its largest
entry (the FP32 rounding of Qbar^{n+1/2}, about 1e-7 of it, enters v0bar's
sum of signed terms).

Cases: the refined polar mesh (uniform-run and searching tiles), PLM and PPM,
shifts of under a cell up to many periods either way; rows of 264 and 300
cells; a coarse half next to a 20x finer half (windows beyond the LDS, taken
in chunks); the 2048 x 16384 disk on sampled rows; and the fused call's
fallback (per-row meshes, FP64) equal to the two calls it composes.
"""
import numpy as np
import pytest
import torch

import oracle
from parity import CELL_F32, CELL_F32_ADJ, assert_parity
from paper_2305_05362_amd import _lib as R
from paper_2305_05362_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
RECONS = [R.RAM_RECON_PLM, R.RAM_RECON_PPM]


def f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def t32(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=dtype, device=DEV)


@pytest.fixture
def ctx():
    c = R.context(0)
    c.set_schedule(0)
    yield c
    c.set_schedule(0)


def _shift_case(ctx, wl, recon, sched, seed=11, what=""):
    ctx.set_schedule(sched)
    rng = np.random.default_rng(seed)
    q = f32(wl.q0.reshape(-1))
    qb = f32(rng.standard_normal(wl.n_cells))
    rows = R.Rows.from_workload(wl, DEV)
    out = torch.empty(wl.n_cells, dtype=torch.float32, device=DEV)
    v0b = torch.zeros(wl.n_rows, dtype=torch.float64, device=DEV)
    v0 = t32(wl.v0, torch.float64)
    ctx.ram_shift_limited_adjoint(rows, t32(q), t32(qb), out, v0, wl.dt, recon, v0b)
    torch.cuda.synchronize()
    got, gv = out.cpu().numpy().astype(np.float64), v0b.cpu().numpy()
    ref, rv = oracle.shift_recon_adjoint(oracle.Rows.from_workload(wl), q, qb, wl.v0, wl.dt,
                                         recon)
    e, c = assert_parity(got, ref, 1e-6, CELL_F32, what)
    ev = np.max(np.abs(gv - rv)) / np.max(np.abs(rv))
    print(f"{what}: qbar rel-L1 {e:.2e} cell {c:.2e}, v0bar {ev:.2e}")
    assert ev <= 1e-10, what


def _polar(recon):
    wl = W.small_polar(12, 4096, order=5)
    n = wl.n_cols
    wl.v0[:] = wl.v0 * np.array([1.0, -1.0, 7.3, -11.9, 0.02, -0.05,
                                 n * 0.37, -n * 0.81, 1.0, -2.0, 3.0, -4.0])
    return wl


@pytest.mark.parametrize("sched", [0, 4])
@pytest.mark.parametrize("recon", RECONS)
def test_stream_limited_shift_adjoint(ctx, recon, sched):
    _shift_case(ctx, _polar(recon), recon, sched, what=f"recon {recon} sched {sched}")


@pytest.mark.parametrize("n", [264, 300])
@pytest.mark.parametrize("recon", RECONS)
def test_stream_limited_short_rows(ctx, recon, n):
    rng = np.random.default_rng(n + recon)
    e = W.stretched_edges(n, 8.0, rng)
    q = 1.0 + 0.2 * rng.standard_normal((4, n))
    v0 = np.array([0.3, -17.2, n + 0.6, -1.7 * n]) / n
    wl = W.Workload("short", 4, n, np.arange(5) * n, e, True, q, None, v0, 1.0, 5, 1)
    _shift_case(ctx, wl, recon, 0, what=f"n={n} recon {recon}")


@pytest.mark.parametrize("recon", RECONS)
def test_stream_limited_refinement_jump(ctx, recon):
    # shifted by about half the period, coarse tiles land on the 20x finer
    # half: windows of thousands of cells, taken in chunks
    coarse = np.linspace(0.0, 0.5, 257)
    fine = np.linspace(0.5, 1.0, 256 * 20 + 1)[1:]
    e = np.concatenate([coarse, fine])
    n = len(e) - 1
    rng = np.random.default_rng(5)
    q = 1.0 + 0.2 * rng.standard_normal((3, n))
    wl = W.Workload("jump", 3, n, np.arange(4) * n, e, True, q, None,
                    np.array([-0.5, -0.37, 0.41]), 1.0, 5, 1)
    _shift_case(ctx, wl, recon, 0, what=f"jump recon {recon}")


@pytest.mark.parametrize("sched", [0, 4])
@pytest.mark.parametrize("recon", RECONS)
def test_stream_limited_step_adjoint(ctx, recon, sched):
    ctx.set_schedule(sched)
    wl = _polar(recon)
    orows = oracle.Rows.from_workload(wl)
    rng = np.random.default_rng(13)
    qf = f32(wl.q0.reshape(-1))
    qh = f32(oracle.shift_recon(orows, qf, wl.v0, wl.dt, recon))
    dv = f32(wl.dv.reshape(-1))
    rbar = f32(rng.standard_normal(wl.n_cells))
    rows = R.Rows.from_workload(wl, DEV)
    out = torch.empty(wl.n_cells, dtype=torch.float32, device=DEV)
    dvb = torch.zeros(wl.n_cells, dtype=torch.float32, device=DEV)
    v0b = torch.zeros(wl.n_rows, dtype=torch.float64, device=DEV)
    ctx.ram_step_limited_adjoint(rows, t32(qf), t32(qh), t32(dv), t32(rbar), out,
                                 t32(wl.v0, torch.float64), wl.dt, recon, dvb, v0b)
    torch.cuda.synchronize()
    rq, rdvb = oracle.residual_adjoint(orows, qh, dv, rbar, wl.dt)
    ref, rv = oracle.shift_recon_adjoint(orows, qf, rq, wl.v0, wl.dt, recon)
    got = out.cpu().numpy().astype(np.float64)
    e0, c0 = assert_parity(got, ref, 1e-5, CELL_F32_ADJ, "qbar")
    e1, c1 = assert_parity(dvb.cpu().numpy().astype(np.float64), rdvb, 1e-5, CELL_F32_ADJ,
                           "dvbar")
    ev = np.max(np.abs(v0b.cpu().numpy() - rv)) / np.max(np.abs(rv))
    print(f"recon {recon} sched {sched}: qbar {e0:.2e}/{c0:.2e}, dvbar {e1:.2e}/{c1:.2e}, "
          f"v0bar {ev:.2e}")
    assert ev <= 1e-5


@pytest.mark.parametrize("recon", RECONS)
def test_stream_limited_cfg5_sampled_rows(ctx, recon):
    wl = W.cfg5()
    rows = R.Rows.from_workload(wl, DEV)
    rng = np.random.default_rng(3)
    q = f32(wl.q0.reshape(-1))
    qb = f32(rng.standard_normal(wl.n_cells))
    out = torch.empty(wl.n_cells, dtype=torch.float32, device=DEV)
    v0b = torch.zeros(wl.n_rows, dtype=torch.float64, device=DEV)
    ctx.ram_shift_limited_adjoint(rows, t32(q), t32(qb), out, t32(wl.v0, torch.float64),
                                  wl.dt, recon, v0b)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64).reshape(wl.n_rows, -1)
    gv = v0b.cpu().numpy()
    n = wl.n_cols
    pick = (0, 1020, 1024, 1031, 2047)
    one = oracle.Rows.single(wl.edges)
    rvs = []
    for r in pick:
        s = slice(r * n, (r + 1) * n)
        ref, rv = oracle.shift_recon_adjoint(one, q[s], qb[s], wl.v0[r:r + 1], wl.dt, recon)
        assert_parity(got[r], ref, 1e-6, CELL_F32, what=str(r))
        rvs.append(rv[0])
    rvs = np.array(rvs)
    ev = np.max(np.abs(gv[list(pick)] - rvs)) / np.max(np.abs(rvs))
    print(f"cfg5 recon {recon}: v0bar {ev:.2e}")
    assert ev <= 1e-10


@pytest.mark.parametrize("kind,dtype", [("ragged", torch.float32), ("polar", torch.float64)])
def test_fused_limited_fallback_equals_two_calls(ctx, kind, dtype):
    wl = (W.small_ragged(16, 8, 2600, seed=53) if kind == "ragged"
          else W.small_polar(6, 2048))
    recon = R.RAM_RECON_PPM
    rows = R.Rows.from_workload(wl, DEV)
    rng = np.random.default_rng(17)
    qf, qh = t32(wl.q0, dtype), t32(wl.q0 * 1.01, dtype)
    dv = t32(wl.dv, dtype)
    rbar = t32(rng.standard_normal(wl.n_cells), dtype)
    v0 = t32(wl.v0, torch.float64)
    out1 = torch.empty_like(rbar)
    dvb1 = torch.zeros_like(dv)
    v0b1 = torch.zeros_like(v0)
    ctx.ram_step_limited_adjoint(rows, qf, qh, dv, rbar, out1, v0, wl.dt, recon, dvb1, v0b1)
    mid, out2 = torch.empty_like(rbar), torch.empty_like(rbar)
    dvb2 = torch.zeros_like(dv)
    v0b2 = torch.zeros_like(v0)
    ctx.ram_residual_adjoint(rows, qh, dv, rbar, mid, wl.dt, dvb2)
    ctx.ram_shift_limited_adjoint(rows, qf, mid, out2, v0, wl.dt, recon, v0b2)
    torch.cuda.synchronize()
    assert torch.equal(out1, out2) and torch.equal(dvb1, dvb2) and torch.equal(v0b1, v0b2)
