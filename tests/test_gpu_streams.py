"""One context's calls issued alternately on two streams with no
synchronisation between them.

The calls share the context's device scratch (mesh tables, tile plan,
ping-pong state), rewritten by every call; ram_set_stream hands the context
from one stream to the other with an event, so each call still sees its own
tables.  The results must equal those of the same calls made one after the
other on one stream, bit for bit: a call that read another's tables would be
off by far more than rounding (a different mesh).
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


@pytest.fixture
def ctx():
    c = R.context(0)
    c.set_schedule(0)
    yield c
    c.set_schedule(0)


def _cases():
    a = W.small_polar(128, 4096, order=5)              # one shared mesh
    b = W.small_ragged(96, 8, 3000, seed=45, order=5)  # per-row meshes
    out = []
    for wl in (a, b):
        rows = R.Rows.from_workload(wl, DEV)
        out.append((wl, rows, dev(wl.q0), dev(wl.v0),
                    dev(wl.dv) if wl.dv is not None else None))
    return out


@pytest.mark.parametrize("what", ["shift", "step"])
def test_two_streams_equal_one_stream(ctx, what):
    cases = _cases()

    def call(case, q, out):
        wl, rows, _, v0, dv = case
        if what == "shift":
            ctx.ram_shift(rows, q, out, v0, wl.dt, wl.order, R.RAM_SCAN_F64)
        else:                                  # a captured multi-step loop, in place
            out.copy_(q)
            ctx.ram_step(rows, out, v0, dv if dv is not None else torch.zeros_like(q),
                         wl.dt, wl.order, 6, R.RAM_SCAN_F64)

    # one stream, one call after the other (this also sizes the scratch, so
    # that no reallocation synchronises the streams below)
    ref = []
    for case in cases:
        o = torch.empty_like(case[2])
        call(case, case[2], o)
        ref.append(o)
    torch.cuda.synchronize()

    n = 8
    outs = [torch.full_like(cases[k % 2][2], float("nan")) for k in range(n)]
    s = [torch.cuda.Stream(device=DEV), torch.cuda.Stream(device=DEV)]
    cur = torch.cuda.current_stream(DEV)
    for st in s:
        st.wait_stream(cur)                    # inputs and outputs are ready
    for k in range(n):
        with torch.cuda.stream(s[k % 2]):
            call(cases[k % 2], cases[k % 2][2], outs[k])
    torch.cuda.synchronize()
    for k in range(n):
        assert torch.equal(outs[k], ref[k % 2]), (what, k)
