"""Per-row checks on the GPU (ram_row_norms) against numpy in FP64: row mass
sum Q dx, the dx-weighted L1 distance to a reference, and max |Q|, on a shared
mesh, per-row ragged meshes, FP64 and FP32 states; and the conservation check
the mass serves, on the 2048 x 16384 disk after several steps."""
import numpy as np
import pytest
import torch

from paper_2305_05362_amd import _lib as R
from paper_2305_05362_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _dx_per_cell(wl):
    if wl.edges_shared:
        return np.tile(np.diff(wl.edges), wl.n_rows)
    return np.concatenate([np.diff(wl.row_edges(r)) for r in range(wl.n_rows)])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kind", ["polar", "ragged"])
def test_row_norms_match_numpy(kind, dtype):
    wl = W.small_polar(5, 3000) if kind == "polar" else W.small_ragged(40, 6, 2500, seed=3)
    rows = R.Rows.from_workload(wl, DEV)
    rng = np.random.default_rng(1)
    q = wl.q0.reshape(-1)
    ref = q + 0.01 * rng.standard_normal(q.shape)
    qd = torch.as_tensor(q, dtype=dtype, device=DEV)
    rd = torch.as_tensor(ref, dtype=dtype, device=DEV)
    out = R.ram_row_norms(rows, qd, rd).cpu().numpy()
    nor = R.ram_row_norms(rows, qd).cpu().numpy()
    torch.cuda.synchronize()
    qh = qd.cpu().numpy().astype(np.float64)
    rh = rd.cpu().numpy().astype(np.float64)
    dx = _dx_per_cell(wl)
    for r in range(wl.n_rows):
        sl = slice(wl.row_ptr[r], wl.row_ptr[r + 1])
        m = np.sum(qh[sl] * dx[sl])
        d = np.sum(np.abs(qh[sl] - rh[sl]) * dx[sl])
        assert abs(out[r, 0] - m) <= 1e-13 * np.sum(np.abs(qh[sl] * dx[sl])), r
        assert abs(out[r, 1] - d) <= 1e-13 * d, r
        assert out[r, 2] == np.max(np.abs(qh[sl])), r
        assert nor[r, 1] == 0.0 and nor[r, 0] == out[r, 0]


def test_row_mass_conserved_full_size():
    wl = W.cfg5()
    rows = R.Rows.from_workload(wl, DEV)
    q = torch.as_tensor(wl.q0.reshape(-1), dtype=torch.float64, device=DEV)
    m0 = R.ram_row_norms(rows, q)[:, 0].clone()
    R.ram_step(rows, q, torch.as_tensor(wl.v0, device=DEV),
               torch.as_tensor(wl.dv.reshape(-1), device=DEV), wl.dt, 5, 5)
    m1 = R.ram_row_norms(rows, q)[:, 0]
    torch.cuda.synchronize()
    rel = ((m1 - m0).abs() / m0.abs()).max().item()
    assert rel <= 1e-13, rel
