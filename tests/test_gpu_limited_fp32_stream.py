"""The limited (PLM / PPM) FP32 step on a shared mesh at the default schedule
(k_step_uni_lim for the uniform-run tiles, k_step_gen_lim for the rest:
windows of up to 400 cells tabulated in LDS, wider ones integrated from
global memory) against the FP64 oracle run on the same FP32 inputs, at the
FP32 bars (relative L1 1e-6, per cell CELL_F32; Section 3.1's limited
shift, then the residual step):

* a coarse half beside a 2x finer half (searching windows of about 520
  cells: the global path) and a 20x finer half (thousands), shift and step;
* a mesh of a coarse and a 1.3x finer uniform half (windows of about 330
  cells: the LDS path, besides the uniform-run tiles);
* rows of 8, 13, 264 and 300 cells (windows that wrap the row, no uniform
  tile) and of 1001 cells (no 16-byte loads or stores);
* the recorded trajectory's half steps (the limited shift alone) and steps.
"""
import numpy as np
import pytest
import torch

import oracle
from parity import CELL_F32, assert_parity
from paper_2305_05362_amd import _lib as R
from paper_2305_05362_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
RECONS = [R.RAM_RECON_PLM, R.RAM_RECON_PPM]


def f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def t32(a):
    return torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=torch.float32, device=DEV)


@pytest.fixture(autouse=True)
def default_schedule():
    c = R.context(0)
    c.set_schedule(0)
    yield
    c.set_schedule(0)


def _wl(edges, v0, seed, with_dv):
    n = len(edges) - 1
    v0 = np.asarray(v0, dtype=np.float64)
    rng = np.random.default_rng(seed)
    xc = 0.5 * (edges[:-1] + edges[1:])
    q = 1.0 + 0.3 * np.sin(2 * np.pi * xc)[None, :] + 0.2 * rng.standard_normal((len(v0), n))
    dv = (0.2 * np.diff(edges).min() * rng.uniform(-1, 1, (len(v0), n))) if with_dv else None
    return W.Workload("lim32", len(v0), n, np.arange(len(v0) + 1) * n, edges, True, f32(q),
                      None if dv is None else f32(dv), v0, 1.0, 5, 1)


def _check(wl, recon, steps, with_dv, what):
    rows = R.Rows.from_workload(wl, DEV)
    q = t32(wl.q0)
    v0 = torch.as_tensor(wl.v0, dtype=torch.float64, device=DEV)
    R.context(0).ram_step_limited(rows, q, v0, t32(wl.dv) if with_dv else None, wl.dt, recon,
                                  steps)
    torch.cuda.synchronize()
    ref = oracle.step_recon(oracle.Rows.from_workload(wl), wl.q0, wl.v0,
                            wl.dv if with_dv else None, wl.dt, recon, steps)
    e1, ec = assert_parity(q.cpu().numpy().astype(np.float64), ref, 1e-6, CELL_F32, what)
    print(f"{what}: rel-L1 {e1:.2e}, max cell {ec:.2e}")


def _halves(ratio):
    coarse = np.linspace(0.0, 0.5, 257)
    fine = np.linspace(0.5, 1.0, int(256 * ratio) + 1)[1:]
    return np.concatenate([coarse, fine])


@pytest.mark.parametrize("ratio", [1.3, 2, 20])
@pytest.mark.parametrize("recon", RECONS)
def test_refined_halves(recon, ratio):
    e = _halves(ratio)
    for with_dv in (False, True):
        _check(_wl(e, [-0.5, -0.37, 0.41, 0.013], 3, with_dv), recon, 1, with_dv,
               f"x{ratio} recon {recon} dv={with_dv}")


@pytest.mark.parametrize("n", [8, 13, 264, 300, 1001])
@pytest.mark.parametrize("recon", RECONS)
def test_short_and_odd_rows(recon, n):
    rng = np.random.default_rng(n + recon)
    e = W.stretched_edges(n, 8.0, rng)
    v0 = np.array([0.3, -17.2, n + 0.6, -1.7 * n]) / n
    for with_dv in (False, True):
        _check(_wl(e, v0, n, with_dv), recon, 1, with_dv, f"n={n} recon {recon} dv={with_dv}")


@pytest.mark.parametrize("recon", RECONS)
def test_recorded_half_steps(recon):
    wl = W.small_polar(8, 4096, order=5)
    q0 = f32(wl.q0.reshape(-1))
    dv = f32(wl.dv.reshape(-1))
    rows = R.Rows.from_workload(wl, DEV)
    k = 3
    traj = torch.empty((k + 1, wl.n_cells), dtype=torch.float32, device=DEV)
    half = torch.empty((k, wl.n_cells), dtype=torch.float32, device=DEV)
    traj[0] = t32(q0)
    v0 = torch.as_tensor(wl.v0, dtype=torch.float64, device=DEV)
    R.context(0).ram_step_limited_record(rows, traj, half, v0, t32(dv), wl.dt, recon, k)
    torch.cuda.synchronize()
    orows = oracle.Rows.from_workload(wl)
    for s in range(k):
        # each half step from the GPU's own state of that step (the FP32
        # rounding of the steps before is not the object here)
        qs = traj[s].cpu().numpy().astype(np.float64)
        qh = oracle.shift_recon(orows, qs, wl.v0, wl.dt, recon)
        assert_parity(half[s].cpu().numpy().astype(np.float64), qh, 1e-6, CELL_F32,
                      f"half step {s}")
        qn = oracle.step_recon(orows, qs, wl.v0, dv, wl.dt, recon, 1)
        assert_parity(traj[s + 1].cpu().numpy().astype(np.float64), qn, 1e-6, CELL_F32,
                      f"step {s}")
