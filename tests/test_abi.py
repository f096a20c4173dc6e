"""Host-side checks of the C ABI (no GPU needed).

* libram.so loads and exports every function include/ram.h declares;
* argument errors are reported with the documented status before the library
  touches a device (a null context is only reported after the arguments).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ram.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ram_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2305_05362_amd import _lib
    return _lib.load_library()


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("ram_shift", "ram_residual", "ram_step", "ram_shift_adjoint",
                 "ram_residual_adjoint", "ram_create", "ram_destroy",
                 "ram_validate", "ram_status_string", "ram_last_error"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    assert lib.ram_status_string(0) == b"ok"
    assert lib.ram_status_string(-2) == b"unsupported configuration"
    assert lib.ram_version().startswith(b"ram-mi355x")


def _layout(n_rows=2, n_cols=16, shared=1):
    from paper_2305_05362_amd._lib import Layout
    return Layout(n_rows, n_cols, None, 0, shared)


def test_argument_errors_without_device(lib):
    from paper_2305_05362_amd import _lib as R
    L = _layout()
    fake = ctypes.c_void_p(0x1000)     # never dereferenced: checks fail first
    # even order
    st = lib.ram_shift(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F64, fake,
                       ctypes.c_void_p(0x2000), fake, fake, 0.1, 2)
    assert st == R.RAM_E_UNSUPPORTED and b"order" in lib.ram_last_error()
    # FP64 state with an FP32 scan
    st = lib.ram_shift(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F32, fake,
                       ctypes.c_void_p(0x2000), fake, fake, 0.1, 5)
    assert st == R.RAM_E_UNSUPPORTED
    # aliasing input and output
    st = lib.ram_shift(None, ctypes.byref(L), R.RAM_F32, R.RAM_SCAN_F64, fake,
                       fake, fake, fake, 0.1, 5)
    assert st == R.RAM_E_INVALID_ARG and b"alias" in lib.ram_last_error()
    # non-finite dt
    st = lib.ram_residual(None, ctypes.byref(L), R.RAM_F64, fake,
                          ctypes.c_void_p(0x2000), fake, fake, float("nan"))
    assert st == R.RAM_E_INVALID_ARG and b"dt" in lib.ram_last_error()
    # rows shorter than the stencil
    L2 = _layout(1, 4)
    st = lib.ram_step(None, ctypes.byref(L2), R.RAM_F64, R.RAM_SCAN_F64, fake,
                      fake, fake, None, 0.1, 5, 3)
    assert st == R.RAM_E_INVALID_ARG
    # ragged layout without row_ptr
    from paper_2305_05362_amd._lib import Layout
    L3 = Layout(3, 0, None, 100, 0)
    st = lib.ram_residual(None, ctypes.byref(L3), R.RAM_F64, fake,
                          ctypes.c_void_p(0x2000), fake, fake, 0.1)
    assert st == R.RAM_E_INVALID_ARG and b"row_ptr" in lib.ram_last_error()
    # shared edges need uniform rows
    L4 = Layout(3, 0, 0x3000, 100, 1)
    st = lib.ram_residual(None, ctypes.byref(L4), R.RAM_F64, fake,
                          ctypes.c_void_p(0x2000), fake, fake, 0.1)
    assert st == R.RAM_E_INVALID_ARG
    # null adjoint outputs
    st = lib.ram_shift_adjoint(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F64,
                               None, fake, None, fake, fake, 0.1, 5, None)
    assert st == R.RAM_E_INVALID_ARG
    # v0bar without the forward state
    st = lib.ram_shift_adjoint(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F64,
                               None, fake, ctypes.c_void_p(0x2000), fake, fake,
                               0.1, 5, ctypes.c_void_p(0x4000))
    assert st == R.RAM_E_INVALID_ARG and b"q_fwd" in lib.ram_last_error()
    # valid arguments, null context: reported last
    st = lib.ram_shift(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F64, fake,
                       ctypes.c_void_p(0x2000), fake, fake, 0.1, 5)
    assert st == R.RAM_E_INVALID_ARG and b"context" in lib.ram_last_error()


def test_record_and_step_adjoint_argument_errors(lib):
    from paper_2305_05362_amd import _lib as R
    L = _layout()
    a, b, c, d = (ctypes.c_void_p(0x1000 * i) for i in (1, 2, 3, 4))
    # a step with a residual must record the post-shift states
    st = lib.ram_step_record(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F64, a, None,
                             b, c, d, 0.1, 5, 4)
    assert st == R.RAM_E_INVALID_ARG and b"q_half" in lib.ram_last_error()
    st = lib.ram_step_record(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F64, a, None,
                             b, c, None, 0.1, 5, -1)
    assert st == R.RAM_E_INVALID_ARG and b"n_steps" in lib.ram_last_error()
    # adjoint: dvbar without dv, v0bar without q_fwd, aliasing output
    st = lib.ram_step_adjoint(None, ctypes.byref(L), R.RAM_F64, a, None, None, b,
                              c, d, d, 0.1, 5, ctypes.c_void_p(0x9000), None)
    assert st == R.RAM_E_INVALID_ARG and b"dvbar" in lib.ram_last_error()
    st = lib.ram_step_adjoint(None, ctypes.byref(L), R.RAM_F64, None, None, None, b,
                              c, d, d, 0.1, 5, None, ctypes.c_void_p(0x9000))
    assert st == R.RAM_E_INVALID_ARG and b"q_fwd" in lib.ram_last_error()
    st = lib.ram_step_adjoint(None, ctypes.byref(L), R.RAM_F64, a, b, d, c,
                              b, d, d, 0.1, 5, None, None)
    assert st == R.RAM_E_INVALID_ARG and b"alias" in lib.ram_last_error()
    # valid arguments, null context
    st = lib.ram_step_adjoint(None, ctypes.byref(L), R.RAM_F64, a, b, d, c,
                              ctypes.c_void_p(0x7000), d, d, 0.1, 5, None, None)
    assert st == R.RAM_E_INVALID_ARG and b"context" in lib.ram_last_error()


def test_step_adjoint_steps_argument_errors(lib):
    from paper_2305_05362_amd import _lib as R
    L = _layout()                            # 2 x 16 cells: 256 bytes a state in FP64
    traj, half, dv, qb, wk, e, v0 = (ctypes.c_void_p(0x100000 * i) for i in range(1, 8))
    I64 = ctypes.c_int64

    def call(*, q_traj=traj, q_half=half, dvp=dv, qbar=qb, work=wk, n=4, dvbar=None):
        return lib.ram_step_adjoint_steps(None, ctypes.byref(L), R.RAM_F64, q_traj, q_half,
                                          dvp, qbar, work, e, v0, 0.1, 5, I64(n), dvbar, None)
    assert call(work=None) == R.RAM_E_INVALID_ARG and b"qbar_work" in lib.ram_last_error()
    assert call(q_half=None) == R.RAM_E_INVALID_ARG and b"q_half" in lib.ram_last_error()
    st = call(dvp=None, q_half=None, dvbar=ctypes.c_void_p(0x900000))
    assert st == R.RAM_E_INVALID_ARG and b"dvbar" in lib.ram_last_error()
    assert call(n=-1) == R.RAM_E_INVALID_ARG and b"n_steps" in lib.ram_last_error()
    # the workspace inside the trajectory, the gradient on the workspace
    st = call(work=ctypes.c_void_p(0x100000 + 3 * 256))
    assert st == R.RAM_E_INVALID_ARG and b"overlap" in lib.ram_last_error()
    st = call(qbar=ctypes.c_void_p(0x500000 + 100))
    assert st == R.RAM_E_INVALID_ARG and b"overlap" in lib.ram_last_error()
    # the workspace past the trajectory's n_steps states is free
    st = call(work=ctypes.c_void_p(0x100000 + 4 * 256))
    assert st == R.RAM_E_INVALID_ARG and b"context" in lib.ram_last_error()
    # no steps: nothing to do, before the context is needed
    assert call(n=0) == R.RAM_OK


def test_limited_argument_errors(lib):
    from paper_2305_05362_amd import _lib as R
    L = _layout()
    a, b, c, d = (ctypes.c_void_p(0x1000 * i) for i in (1, 2, 3, 4))
    # unknown reconstruction
    st = lib.ram_shift_limited(None, ctypes.byref(L), R.RAM_F64, 0, a, b, c, d, 0.1)
    assert st == R.RAM_E_UNSUPPORTED and b"recon" in lib.ram_last_error()
    st = lib.ram_step_limited(None, ctypes.byref(L), R.RAM_F32, 3, a, c, d, None, 0.1, 2)
    assert st == R.RAM_E_UNSUPPORTED and b"recon" in lib.ram_last_error()
    # rows shorter than the PPM stencil (5 cells) plus one
    short = _layout(n_cols=5)
    st = lib.ram_shift_limited(None, ctypes.byref(short), R.RAM_F64, R.RAM_RECON_PPM,
                               a, b, c, d, 0.1)
    assert st == R.RAM_E_INVALID_ARG and b"at least 6" in lib.ram_last_error()
    # aliasing, non-finite dt, negative steps
    st = lib.ram_shift_limited(None, ctypes.byref(L), R.RAM_F64, R.RAM_RECON_PLM,
                               a, a, c, d, 0.1)
    assert st == R.RAM_E_INVALID_ARG and b"alias" in lib.ram_last_error()
    st = lib.ram_shift_limited(None, ctypes.byref(L), R.RAM_F64, R.RAM_RECON_PLM,
                               a, b, c, d, float("nan"))
    assert st == R.RAM_E_INVALID_ARG and b"dt" in lib.ram_last_error()
    st = lib.ram_step_limited(None, ctypes.byref(L), R.RAM_F64, R.RAM_RECON_PPM,
                              a, c, d, None, 0.1, -1)
    assert st == R.RAM_E_INVALID_ARG and b"n_steps" in lib.ram_last_error()
    # zero steps succeed without a context; valid arguments then need one
    st = lib.ram_step_limited(None, ctypes.byref(L), R.RAM_F64, R.RAM_RECON_PPM,
                              a, c, d, None, 0.1, 0)
    assert st == R.RAM_OK
    st = lib.ram_shift_limited(None, ctypes.byref(L), R.RAM_F64, R.RAM_RECON_PPM,
                               a, b, c, d, 0.1)
    assert st == R.RAM_E_INVALID_ARG and b"context" in lib.ram_last_error()


def test_row_norms_argument_errors(lib):
    from paper_2305_05362_amd import _lib as R
    L = _layout()
    a, c, d = (ctypes.c_void_p(0x1000 * i) for i in (1, 3, 4))
    st = lib.ram_row_norms(None, ctypes.byref(L), R.RAM_F32, None, None, c, d)
    assert st == R.RAM_E_INVALID_ARG and b"null q" in lib.ram_last_error()
    st = lib.ram_row_norms(None, ctypes.byref(L), 7, a, None, c, d)
    assert st == R.RAM_E_UNSUPPORTED
    st = lib.ram_row_norms(None, ctypes.byref(L), R.RAM_F32, a, None, c, d)
    assert st == R.RAM_E_INVALID_ARG and b"context" in lib.ram_last_error()


def test_schedule_argument_errors(lib):
    from paper_2305_05362_amd import _lib as R
    sc = R.Schedule(3)
    st = lib.ram_set_schedule(None, ctypes.byref(sc))
    assert st == R.RAM_E_INVALID_ARG and b"context" in lib.ram_last_error()
    st = lib.ram_get_schedule(None, ctypes.byref(sc))
    assert st == R.RAM_E_INVALID_ARG


def test_limited_adjoint_argument_errors(lib):
    from paper_2305_05362_amd import _lib as R
    L = _layout()
    a, b, c, d, e = (ctypes.c_void_p(0x1000 * i) for i in (1, 2, 3, 4, 5))
    # the forward state is required (the map is nonlinear)
    st = lib.ram_shift_limited_adjoint(None, ctypes.byref(L), R.RAM_F64, R.RAM_RECON_PPM,
                                       None, b, c, d, e, 0.1, None)
    assert st == R.RAM_E_INVALID_ARG and b"q_fwd" in lib.ram_last_error()
    st = lib.ram_shift_limited_adjoint(None, ctypes.byref(L), R.RAM_F64, R.RAM_RECON_PPM,
                                       a, b, a, d, e, 0.1, None)
    assert st == R.RAM_E_INVALID_ARG and b"alias" in lib.ram_last_error()
    st = lib.ram_shift_limited_adjoint(None, ctypes.byref(L), R.RAM_F64, 9,
                                       a, b, c, d, e, 0.1, None)
    assert st == R.RAM_E_UNSUPPORTED
    st = lib.ram_shift_limited_adjoint(None, ctypes.byref(L), R.RAM_F32, R.RAM_RECON_PLM,
                                       a, b, c, d, e, 0.1, None)
    assert st == R.RAM_E_INVALID_ARG and b"context" in lib.ram_last_error()


def test_mesh_density_argument_errors(lib):
    from paper_2305_05362_amd import _lib as R
    d = R.MeshDensity(R.RAM_DENSITY_PERIODIC_BUMP, -3.14, 3.14, 0.2, 0.3, 9.0)
    st = lib.ram_set_mesh_density(None, ctypes.byref(d))
    assert st == R.RAM_E_INVALID_ARG and b"context" in lib.ram_last_error()
    st = lib.ram_mesh_density_cells(None, None, 10, None, 0, None)
    assert st == R.RAM_E_UNSUPPORTED
    st = lib.ram_mesh_density_cells(None, ctypes.byref(d), 0, None, 0, None)
    assert st == R.RAM_E_INVALID_ARG
    st = lib.ram_mesh_density_cells(None, ctypes.byref(d), 10, None, 5, None)
    assert st == R.RAM_E_INVALID_ARG and b"null" in lib.ram_last_error()


def test_radial_and_split_argument_errors(lib):
    from paper_2305_05362_amd import _lib as R
    L = _layout()
    a, b, c, d, e, f = (ctypes.c_void_p(0x1000 * i) for i in (1, 2, 3, 4, 5, 6))
    # ragged rows have no radial columns
    Lr = R.Layout(2, 0, a, 16, 0)
    st = lib.ram_radial_step(None, ctypes.byref(Lr), R.RAM_F64, a, b, c, d, 0.1)
    assert st == R.RAM_E_INVALID_ARG and b"n_cols" in lib.ram_last_error()
    st = lib.ram_radial_step(None, ctypes.byref(L), R.RAM_F64, a, a, c, d, 0.1)
    assert st == R.RAM_E_INVALID_ARG and b"alias" in lib.ram_last_error()
    st = lib.ram_radial_step(None, ctypes.byref(L), R.RAM_F64, a, b, None, d, 0.1)
    assert st == R.RAM_E_INVALID_ARG and b"null" in lib.ram_last_error()
    st = lib.ram_radial_step(None, ctypes.byref(L), R.RAM_F64, a, b, c, d, float("nan"))
    assert st == R.RAM_E_INVALID_ARG and b"dt" in lib.ram_last_error()
    st = lib.ram_radial_step(None, ctypes.byref(L), 5, a, b, c, d, 0.1)
    assert st == R.RAM_E_UNSUPPORTED
    st = lib.ram_radial_step(None, ctypes.byref(L), R.RAM_F32, a, b, c, d, 0.1)
    assert st == R.RAM_E_INVALID_ARG and b"context" in lib.ram_last_error()
    # the split step: row-step and radial checks, then the context
    st = lib.ram_step_split2d(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F64, 0, a, b, c,
                              d, e, f, 0.1, 4, 1)
    assert st == R.RAM_E_UNSUPPORTED and b"order" in lib.ram_last_error()
    st = lib.ram_step_split2d(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F64, 7, a, b, c,
                              d, e, f, 0.1, 5, 1)
    assert st == R.RAM_E_UNSUPPORTED and b"recon" in lib.ram_last_error()
    Lp = _layout(shared=0)
    st = lib.ram_step_split2d(None, ctypes.byref(Lp), R.RAM_F64, R.RAM_SCAN_F64,
                              R.RAM_RECON_PLM, a, b, c, d, e, f, 0.1, 5, 1)
    assert st == R.RAM_E_UNSUPPORTED and b"shared" in lib.ram_last_error()
    st = lib.ram_step_split2d(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F64, 0, a, b, c,
                              d, None, f, 0.1, 5, 1)
    assert st == R.RAM_E_INVALID_ARG and b"null" in lib.ram_last_error()
    st = lib.ram_step_split2d(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F64, 0, a, b, c,
                              d, e, f, 0.1, 5, -1)
    assert st == R.RAM_E_INVALID_ARG and b"n_steps" in lib.ram_last_error()
    st = lib.ram_step_split2d(None, ctypes.byref(L), R.RAM_F32, R.RAM_SUM_DIRECT, 0, a, b, c,
                              d, e, f, 0.1, 5, 1)
    assert st == R.RAM_E_INVALID_ARG and b"context" in lib.ram_last_error()


def test_cell_average_and_point4_argument_errors(lib):
    from paper_2305_05362_amd import _lib as R
    L = _layout()
    a, b, c, d = (ctypes.c_void_p(0x1000 * i) for i in (1, 2, 3, 4))
    st = lib.ram_cell_average(None, ctypes.byref(L), R.RAM_F64, a, b, c, 2)
    assert st == R.RAM_E_INVALID_ARG and b"to_centre" in lib.ram_last_error()
    st = lib.ram_cell_average(None, ctypes.byref(L), R.RAM_F64, a, a, c, 0)
    assert st == R.RAM_E_INVALID_ARG and b"alias" in lib.ram_last_error()
    st = lib.ram_cell_average(None, ctypes.byref(L), R.RAM_F64, None, b, c, 0)
    assert st == R.RAM_E_INVALID_ARG and b"null" in lib.ram_last_error()
    st = lib.ram_cell_average(None, ctypes.byref(L), 9, a, b, c, 0)
    assert st == R.RAM_E_UNSUPPORTED
    st = lib.ram_cell_average(None, ctypes.byref(L), R.RAM_F32, a, b, c, 1)
    assert st == R.RAM_E_INVALID_ARG and b"context" in lib.ram_last_error()
    # the step on centre values: the row step's checks, then the context
    st = lib.ram_step_point4(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F64, 0, a, b, c, d,
                             0.1, 2, 1)
    assert st == R.RAM_E_UNSUPPORTED and b"order" in lib.ram_last_error()
    Lp = _layout(shared=0)
    st = lib.ram_step_point4(None, ctypes.byref(Lp), R.RAM_F64, R.RAM_SCAN_F64,
                             R.RAM_RECON_PPM, a, b, c, d, 0.1, 5, 1)
    assert st == R.RAM_E_UNSUPPORTED and b"shared" in lib.ram_last_error()
    st = lib.ram_step_point4(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F64, 0, a, b, c, d,
                             0.1, 5, -3)
    assert st == R.RAM_E_INVALID_ARG and b"n_steps" in lib.ram_last_error()
    st = lib.ram_step_point4(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F64, 0, None, b, c,
                             d, 0.1, 5, 1)
    assert st == R.RAM_E_INVALID_ARG and b"null q" in lib.ram_last_error()
    st = lib.ram_step_point4(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F64, 0, a, b, c, d,
                             float("inf"), 5, 1)
    assert st == R.RAM_E_INVALID_ARG and b"dt" in lib.ram_last_error()
    st = lib.ram_step_point4(None, ctypes.byref(L), R.RAM_F32, R.RAM_SUM_DIRECT, 0, a, b, c,
                             d, 0.1, 5, 1)
    assert st == R.RAM_E_INVALID_ARG and b"context" in lib.ram_last_error()


def test_layout_errors(lib):
    # an empty batch, negative widths, ragged layouts without offsets or with
    # a shared mesh are refused before any device work, by every entry point
    from paper_2305_05362_amd import _lib as R
    a, b, c = (ctypes.c_void_p(0x1000 * i) for i in (1, 2, 3))
    cases = [(R.Layout(0, 16, None, 0, 1), b"n_rows"),
             (R.Layout(2, -1, None, 0, 1), b"n_cols"),
             (R.Layout(2, 0, None, 10, 0), b"row_ptr"),
             (R.Layout(2, 0, a, 0, 0), b"n_cells"),
             (R.Layout(2, 0, a, 10, 1), b"shared")]
    for L, msg in cases:
        st = lib.ram_step(None, ctypes.byref(L), R.RAM_F64, R.RAM_SCAN_F64, a, b, c, None,
                          0.1, 5, 1)
        assert st == R.RAM_E_INVALID_ARG and msg in lib.ram_last_error(), msg
        st = lib.ram_cell_average(None, ctypes.byref(L), R.RAM_F64, a, b, c, 0)
        assert st == R.RAM_E_INVALID_ARG and msg in lib.ram_last_error(), msg
    st = lib.ram_step(None, None, R.RAM_F64, R.RAM_SCAN_F64, a, b, c, None, 0.1, 5, 1)
    assert st == R.RAM_E_INVALID_ARG and b"layout" in lib.ram_last_error()
