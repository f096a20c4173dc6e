"""ctypes binding of libram.so (the C ABI declared in include/ram.h).

Argument marshalling only: every step of the advection path runs in the HIP
kernels of libram.so.  PyTorch supplies device memory (tensors) and the
stream; the library never sees a torch type.  If the library is missing the
import fails loudly -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libram.so")

RAM_OK = 0
RAM_E_INVALID_ARG = -1
RAM_E_UNSUPPORTED = -2
RAM_E_MESH = -3
RAM_E_CFL = -4
RAM_E_HIP = -5
RAM_E_NOMEM = -6

RAM_F64 = 0
RAM_F32 = 1

RAM_SCAN_F64 = 0
RAM_SCAN_F32_TWOSUM = 1
RAM_SCAN_F32 = 2
RAM_SUM_DIRECT = 3

SCANS = {"f64": RAM_SCAN_F64, "twosum": RAM_SCAN_F32_TWOSUM, "f32": RAM_SCAN_F32,
         "direct": RAM_SUM_DIRECT}

RAM_RECON_PLM = 1
RAM_RECON_PPM = 2

RAM_TILE_WINDOW = 0
RAM_TILE_UNIFORM = 1
RAM_TILE_DIRECT = 2
RECONS = {"plm": RAM_RECON_PLM, "ppm": RAM_RECON_PPM}


class RamError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"RAM error {status}: {message}")
        self.status = status


class Layout(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("n_cells", ctypes.c_int64),
                ("edges_shared", ctypes.c_int32)]


class Schedule(ctypes.Structure):
    _fields_ = [("items_per_thread", ctypes.c_int32)]


RAM_DENSITY_NONE = 0
RAM_DENSITY_PERIODIC_BUMP = 1


class MeshDensity(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("xmin", ctypes.c_double),
                ("xmax", ctypes.c_double), ("a", ctypes.c_double),
                ("b", ctypes.c_double), ("c", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libram.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2305_05362_amd.build` "
            "(the RAM path has no non-HIP implementation)")
    lib = ctypes.CDLL(path)
    P, D, I, I64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int64
    LP = ctypes.POINTER(Layout)
    sig = {
        "ram_create": [ctypes.POINTER(ctypes.c_void_p), I, P],
        "ram_destroy": [P],
        "ram_set_stream": [P, P],
        "ram_sync": [P],
        "ram_shift": [P, LP, I, I, P, P, P, P, D, I],
        "ram_shift_noalloc": [P, LP, I, I, P, P, P, P, D, I],
        "ram_residual": [P, LP, I, P, P, P, P, D],
        "ram_step": [P, LP, I, I, P, P, P, P, D, I, I64],
        "ram_shift_adjoint": [P, LP, I, I, P, P, P, P, P, D, I, P],
        "ram_residual_adjoint": [P, LP, I, P, P, P, P, P, D, P],
        "ram_step_record": [P, LP, I, I, P, P, P, P, P, D, I, I64],
        "ram_step_adjoint": [P, LP, I, P, P, P, P, P, P, P, D, I, P, P],
        "ram_step_adjoint_steps": [P, LP, I, P, P, P, P, P, P, P, D, I, I64, P, P],
        "ram_validate": [P, LP, I, P, P, D],
        "ram_shift_limited": [P, LP, I, I, P, P, P, P, D],
        "ram_step_limited": [P, LP, I, I, P, P, P, P, D, I64],
        "ram_row_norms": [P, LP, I, P, P, P, P],
        "ram_step_tile_paths": [P, LP, P, P, D, I, I, P, I64, ctypes.POINTER(I64)],
        "ram_shift_limited_adjoint": [P, LP, I, I, P, P, P, P, P, D, P],
        "ram_step_limited_adjoint": [P, LP, I, I, P, P, P, P, P, P, P, D, P, P],
        "ram_step_limited_record": [P, LP, I, I, P, P, P, P, P, D, I64],
        "ram_set_schedule": [P, ctypes.POINTER(Schedule)],
        "ram_get_schedule": [P, ctypes.POINTER(Schedule)],
        "ram_set_mesh_density": [P, ctypes.POINTER(MeshDensity)],
        "ram_radial_step": [P, LP, I, P, P, P, P, D],
        "ram_step_split2d": [P, LP, I, I, I, P, P, P, P, P, P, D, I, I64],
        "ram_cell_average": [P, LP, I, P, P, P, I],
        "ram_step_point4": [P, LP, I, I, I, P, P, P, P, D, I, I64],
        "ram_mesh_density_cells": [P, ctypes.POINTER(MeshDensity), I64, P, I64, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.ram_status_string.argtypes = [ctypes.c_int]
    lib.ram_status_string.restype = ctypes.c_char_p
    lib.ram_last_error.argtypes = []
    lib.ram_last_error.restype = ctypes.c_char_p
    lib.ram_version.argtypes = []
    lib.ram_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status: int):
    if status != RAM_OK:
        lib = load_library()
        msg = lib.ram_last_error().decode() or lib.ram_status_string(status).decode()
        raise RamError(status, msg)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return RAM_F64
    if t.dtype == torch.float32:
        return RAM_F32
    raise TypeError(f"state must be float64 or float32, got {t.dtype}")


def _dev_ptr(t: Optional[torch.Tensor], dtype=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return t.data_ptr()


class Rows:
    """Device-side row geometry: node coordinates (FP64) and, for ragged
    batches, the cell offsets ``row_ptr`` (int64, n_rows+1)."""

    def __init__(self, edges: torch.Tensor, n_rows: int, n_cols: int = 0,
                 row_ptr: Optional[torch.Tensor] = None, shared: bool = False,
                 n_cells: Optional[int] = None):
        self.edges = edges
        self.row_ptr = row_ptr
        self.n_rows = int(n_rows)
        self.n_cols = int(n_cols)
        self.shared = bool(shared)
        if self.n_cols > 0:
            self.n_cells = self.n_rows * self.n_cols
        else:
            if row_ptr is None:
                raise ValueError("ragged rows need row_ptr")
            self.n_cells = int(n_cells) if n_cells is not None else int(row_ptr[-1].item())
        _dev_ptr(edges, torch.float64, "edges")
        if row_ptr is not None:
            _dev_ptr(row_ptr, torch.int64, "row_ptr")
        self.layout = Layout(self.n_rows, self.n_cols,
                             row_ptr.data_ptr() if (row_ptr is not None and self.n_cols == 0) else None,
                             self.n_cells, 1 if self.shared else 0)

    @classmethod
    def from_workload(cls, wl, device="cuda") -> "Rows":
        edges = torch.as_tensor(wl.edges, dtype=torch.float64, device=device)
        if wl.n_cols > 0:
            return cls(edges, wl.n_rows, wl.n_cols, None, wl.edges_shared)
        rp = torch.as_tensor(wl.row_ptr, dtype=torch.int64, device=device)
        return cls(edges, wl.n_rows, 0, rp, False, int(wl.row_ptr[-1]))


class Context:
    """One ram_ctx on a device; calls go to torch's current stream."""

    def __init__(self, device: Optional[int] = None):
        lib = load_library()
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        self._lib = lib
        h = ctypes.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        check(lib.ram_create(ctypes.byref(h), self.device, ctypes.c_void_p(stream)))
        self._h = h

    def __del__(self):
        try:
            if getattr(self, "_h", None) and self._h.value:
                self._lib.ram_destroy(self._h)
        except Exception:
            pass

    def _stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(self._lib.ram_set_stream(self._h, ctypes.c_void_p(s)))

    def sync(self):
        check(self._lib.ram_sync(self._h))

    # -- the C ABI, one method per entry point ---------------------------
    def ram_shift(self, rows: Rows, q_in, q_out, v0, dt: float, order: int,
                  scan: int = RAM_SCAN_F64):
        self._stream()
        dt_code = _dtype_code(q_in)
        check(self._lib.ram_shift(
            self._h, ctypes.byref(rows.layout), dt_code, int(scan),
            _dev_ptr(q_in, q_in.dtype, "q_in"), _dev_ptr(q_out, q_in.dtype, "q_out"),
            _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(v0, torch.float64, "v0"), float(dt), int(order)))
        return q_out

    def ram_shift_noalloc(self, rows: Rows, q_in, q_out, v0, dt: float, order: int,
                          scan: int = RAM_SCAN_F64):
        """ram_shift through the entry point that allocates no device memory
        (a static library buffer holds its tables and plan)."""
        self._stream()
        check(self._lib.ram_shift_noalloc(
            self._h, ctypes.byref(rows.layout), _dtype_code(q_in), int(scan),
            _dev_ptr(q_in, q_in.dtype, "q_in"), _dev_ptr(q_out, q_in.dtype, "q_out"),
            _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(v0, torch.float64, "v0"), float(dt), int(order)))
        return q_out

    def set_schedule(self, items_per_thread: int):
        """Shifted nodes per thread of the shared-mesh direct-sum step kernel
        (2..5; 0 = the default)."""
        check(self._lib.ram_set_schedule(self._h, ctypes.byref(Schedule(int(items_per_thread)))))

    def set_mesh_density(self, bump=None, xmin: float = 0.0, xmax: float = 0.0):
        """Periodic-bump mesh density (a, b, c) of the shared mesh on
        [xmin, xmax], or None to switch the closed-form index off."""
        if bump is None:
            check(self._lib.ram_set_mesh_density(self._h, None))
            return
        a, b, c = bump
        d = MeshDensity(RAM_DENSITY_PERIODIC_BUMP, xmin, xmax, a, b, c)
        check(self._lib.ram_set_mesh_density(self._h, ctypes.byref(d)))

    def mesh_density_cells(self, bump, xmin: float, xmax: float, n: int, x):
        """floor(F(x)) of the periodic-bump index for the points x (device
        FP64), int32 on x's device."""
        self._stream()
        a, b, c = bump
        d = MeshDensity(RAM_DENSITY_PERIODIC_BUMP, xmin, xmax, a, b, c)
        out = torch.empty(x.numel(), dtype=torch.int32, device=x.device)
        check(self._lib.ram_mesh_density_cells(self._h, ctypes.byref(d), int(n),
                                               _dev_ptr(x, torch.float64, "x"), x.numel(),
                                               _dev_ptr(out, torch.int32, "cells")))
        return out

    def get_schedule(self) -> int:
        sc = Schedule(0)
        check(self._lib.ram_get_schedule(self._h, ctypes.byref(sc)))
        return int(sc.items_per_thread)

    def ram_shift_limited(self, rows: Rows, q_in, q_out, v0, dt: float, recon: int):
        self._stream()
        check(self._lib.ram_shift_limited(
            self._h, ctypes.byref(rows.layout), _dtype_code(q_in), int(recon),
            _dev_ptr(q_in, q_in.dtype, "q_in"), _dev_ptr(q_out, q_in.dtype, "q_out"),
            _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(v0, torch.float64, "v0"), float(dt)))
        return q_out

    def ram_step_limited(self, rows: Rows, q, v0, dv, dt: float, recon: int,
                         n_steps: int):
        self._stream()
        check(self._lib.ram_step_limited(
            self._h, ctypes.byref(rows.layout), _dtype_code(q), int(recon),
            _dev_ptr(q, q.dtype, "q"), _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(v0, torch.float64, "v0"), _dev_ptr(dv, q.dtype, "dv"),
            float(dt), int(n_steps)))
        return q

    def ram_step_limited_record(self, rows: Rows, q_traj, q_half, v0, dv, dt: float,
                                recon: int, n_steps: int):
        self._stream()
        check(self._lib.ram_step_limited_record(
            self._h, ctypes.byref(rows.layout), _dtype_code(q_traj), int(recon),
            _dev_ptr(q_traj, q_traj.dtype, "q_traj"),
            _dev_ptr(q_half, q_traj.dtype, "q_half"),
            _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(v0, torch.float64, "v0"), _dev_ptr(dv, q_traj.dtype, "dv"),
            float(dt), int(n_steps)))
        return q_traj

    def ram_shift_limited_adjoint(self, rows: Rows, q_fwd, qbar_out, qbar_in, v0,
                                  dt: float, recon: int, v0bar=None):
        self._stream()
        check(self._lib.ram_shift_limited_adjoint(
            self._h, ctypes.byref(rows.layout), _dtype_code(qbar_out), int(recon),
            _dev_ptr(q_fwd, qbar_out.dtype, "q_fwd"),
            _dev_ptr(qbar_out, qbar_out.dtype, "qbar_out"),
            _dev_ptr(qbar_in, qbar_out.dtype, "qbar_in"),
            _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(v0, torch.float64, "v0"), float(dt),
            _dev_ptr(v0bar, torch.float64, "v0bar")))
        return qbar_in

    def ram_step_limited_adjoint(self, rows: Rows, q_fwd, q_half, dv, qbar_out, qbar_in, v0,
                                 dt: float, recon: int, dvbar=None, v0bar=None):
        self._stream()
        t = qbar_out.dtype
        check(self._lib.ram_step_limited_adjoint(
            self._h, ctypes.byref(rows.layout), _dtype_code(qbar_out), int(recon),
            _dev_ptr(q_fwd, t, "q_fwd"), _dev_ptr(q_half, t, "q_half"), _dev_ptr(dv, t, "dv"),
            _dev_ptr(qbar_out, t, "qbar_out"), _dev_ptr(qbar_in, t, "qbar_in"),
            _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(v0, torch.float64, "v0"), float(dt),
            _dev_ptr(dvbar, t, "dvbar"), _dev_ptr(v0bar, torch.float64, "v0bar")))
        return qbar_in

    def ram_radial_step(self, rows: Rows, q_in, q_out, r_edges, u, dt: float):
        self._stream()
        check(self._lib.ram_radial_step(
            self._h, ctypes.byref(rows.layout), _dtype_code(q_in),
            _dev_ptr(q_in, q_in.dtype, "q_in"), _dev_ptr(q_out, q_in.dtype, "q_out"),
            _dev_ptr(r_edges, torch.float64, "r_edges"), _dev_ptr(u, q_in.dtype, "u"),
            float(dt)))
        return q_out

    def ram_step_split2d(self, rows: Rows, q, v0, dv, r_edges, u, dt: float, order: int,
                         n_steps: int, scan: int = RAM_SCAN_F64, recon: int = 0):
        self._stream()
        check(self._lib.ram_step_split2d(
            self._h, ctypes.byref(rows.layout), _dtype_code(q), int(scan), int(recon),
            _dev_ptr(q, q.dtype, "q"), _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(v0, torch.float64, "v0"), _dev_ptr(dv, q.dtype, "dv"),
            _dev_ptr(r_edges, torch.float64, "r_edges"), _dev_ptr(u, q.dtype, "u"),
            float(dt), int(order), int(n_steps)))
        return q

    def ram_cell_average(self, rows: Rows, q_in, q_out, to_centre: bool = False):
        self._stream()
        check(self._lib.ram_cell_average(
            self._h, ctypes.byref(rows.layout), _dtype_code(q_in),
            _dev_ptr(q_in, q_in.dtype, "q_in"), _dev_ptr(q_out, q_in.dtype, "q_out"),
            _dev_ptr(rows.edges, torch.float64, "edges"), int(bool(to_centre))))
        return q_out

    def ram_step_point4(self, rows: Rows, q, v0, dv, dt: float, order: int, n_steps: int,
                        scan: int = RAM_SCAN_F64, recon: int = 0):
        self._stream()
        check(self._lib.ram_step_point4(
            self._h, ctypes.byref(rows.layout), _dtype_code(q), int(scan), int(recon),
            _dev_ptr(q, q.dtype, "q"), _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(v0, torch.float64, "v0"), _dev_ptr(dv, q.dtype, "dv"), float(dt),
            int(order), int(n_steps)))
        return q

    def ram_step_tile_paths(self, rows: Rows, v0, dt: float, order: int, with_residual: bool):
        """Path of every tile of the FP32 direct-sum step (RAM_TILE_*), an
        int32 tensor of n_rows * ceil(n_cols / 256) entries on v0's device."""
        self._stream()
        nt = rows.n_rows * ((rows.n_cols + 255) // 256)
        out = torch.empty(max(nt, 1), dtype=torch.int32, device=v0.device)
        got = ctypes.c_int64(0)
        check(self._lib.ram_step_tile_paths(
            self._h, ctypes.byref(rows.layout), _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(v0, torch.float64, "v0"), float(dt), int(order), int(bool(with_residual)),
            _dev_ptr(out, torch.int32, "paths"), int(out.numel()), ctypes.byref(got)))
        return out[:got.value]

    def ram_row_norms(self, rows: Rows, q, q_ref=None, out=None):
        """Per-row (mass, dx-weighted L1 distance to q_ref, max |q|), FP64
        tensor of shape [n_rows, 3] on q's device."""
        self._stream()
        if out is None:
            out = torch.empty((rows.n_rows, 3), dtype=torch.float64, device=q.device)
        check(self._lib.ram_row_norms(
            self._h, ctypes.byref(rows.layout), _dtype_code(q), _dev_ptr(q, q.dtype, "q"),
            _dev_ptr(q_ref, q.dtype, "q_ref"), _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(out, torch.float64, "out")))
        return out

    def ram_residual(self, rows: Rows, q_in, q_out, dv, dt: float):
        self._stream()
        check(self._lib.ram_residual(
            self._h, ctypes.byref(rows.layout), _dtype_code(q_in),
            _dev_ptr(q_in, q_in.dtype, "q_in"), _dev_ptr(q_out, q_in.dtype, "q_out"),
            _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(dv, q_in.dtype, "dv"), float(dt)))
        return q_out

    def ram_step(self, rows: Rows, q, v0, dv, dt: float, order: int,
                 n_steps: int, scan: int = RAM_SCAN_F64):
        self._stream()
        check(self._lib.ram_step(
            self._h, ctypes.byref(rows.layout), _dtype_code(q), int(scan),
            _dev_ptr(q, q.dtype, "q"), _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(v0, torch.float64, "v0"), _dev_ptr(dv, q.dtype, "dv"),
            float(dt), int(order), int(n_steps)))
        return q

    def ram_shift_adjoint(self, rows: Rows, q_fwd, qbar_out, qbar_in, v0,
                          dt: float, order: int, v0bar=None,
                          scan: int = RAM_SCAN_F64):
        self._stream()
        check(self._lib.ram_shift_adjoint(
            self._h, ctypes.byref(rows.layout), _dtype_code(qbar_out), int(scan),
            _dev_ptr(q_fwd, qbar_out.dtype, "q_fwd"),
            _dev_ptr(qbar_out, qbar_out.dtype, "qbar_out"),
            _dev_ptr(qbar_in, qbar_out.dtype, "qbar_in"),
            _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(v0, torch.float64, "v0"), float(dt), int(order),
            _dev_ptr(v0bar, torch.float64, "v0bar")))
        return qbar_in

    def ram_residual_adjoint(self, rows: Rows, q_fwd, dv, qbar_out, qbar_in,
                             dt: float, dvbar=None):
        self._stream()
        check(self._lib.ram_residual_adjoint(
            self._h, ctypes.byref(rows.layout), _dtype_code(q_fwd),
            _dev_ptr(q_fwd, q_fwd.dtype, "q_fwd"), _dev_ptr(dv, q_fwd.dtype, "dv"),
            _dev_ptr(qbar_out, q_fwd.dtype, "qbar_out"),
            _dev_ptr(qbar_in, q_fwd.dtype, "qbar_in"),
            _dev_ptr(rows.edges, torch.float64, "edges"), float(dt),
            _dev_ptr(dvbar, q_fwd.dtype, "dvbar")))
        return qbar_in

    def ram_step_record(self, rows: Rows, q_traj, q_half, v0, dv, dt: float,
                        order: int, n_steps: int, scan: int = RAM_SCAN_F64):
        """q_traj: (n_steps+1, n_cells), slot 0 the input; q_half: (n_steps,
        n_cells) or None when dv is None."""
        self._stream()
        n = int(n_steps)
        if q_traj.numel() < (n + 1) * rows.n_cells:
            raise ValueError("q_traj holds fewer than n_steps+1 states")
        if dv is not None and (q_half is None or q_half.numel() < n * rows.n_cells):
            raise ValueError("q_half holds fewer than n_steps states")
        check(self._lib.ram_step_record(
            self._h, ctypes.byref(rows.layout), _dtype_code(q_traj), int(scan),
            _dev_ptr(q_traj, q_traj.dtype, "q_traj"),
            _dev_ptr(q_half, q_traj.dtype, "q_half"),
            _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(v0, torch.float64, "v0"), _dev_ptr(dv, q_traj.dtype, "dv"),
            float(dt), int(order), n))
        return q_traj

    def ram_step_adjoint(self, rows: Rows, q_fwd, q_half, dv, qbar_out, qbar_in,
                         v0, dt: float, order: int, dvbar=None, v0bar=None):
        self._stream()
        t = qbar_out.dtype
        check(self._lib.ram_step_adjoint(
            self._h, ctypes.byref(rows.layout), _dtype_code(qbar_out),
            _dev_ptr(q_fwd, t, "q_fwd"), _dev_ptr(q_half, t, "q_half"),
            _dev_ptr(dv, t, "dv"), _dev_ptr(qbar_out, t, "qbar_out"),
            _dev_ptr(qbar_in, t, "qbar_in"),
            _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(v0, torch.float64, "v0"), float(dt), int(order),
            _dev_ptr(dvbar, t, "dvbar"), _dev_ptr(v0bar, torch.float64, "v0bar")))
        return qbar_in

    def ram_step_adjoint_steps(self, rows: Rows, q_traj, q_half, dv, qbar, qbar_work, v0,
                               dt: float, order: int, n_steps: int, dvbar=None, v0bar=None):
        """qbar (in: gradient of Q^n_steps; out: gradient of Q^0) through
        n_steps recorded steps; q_traj / q_half hold at least n_steps states."""
        self._stream()
        t = qbar.dtype
        n = int(n_steps)
        need = n * rows.n_cells
        if q_traj.numel() < need or (dv is not None and (q_half is None or q_half.numel() < need)):
            raise ValueError("q_traj / q_half hold fewer than n_steps states")
        check(self._lib.ram_step_adjoint_steps(
            self._h, ctypes.byref(rows.layout), _dtype_code(qbar),
            _dev_ptr(q_traj, t, "q_traj"), _dev_ptr(q_half, t, "q_half"),
            _dev_ptr(dv, t, "dv"), _dev_ptr(qbar, t, "qbar"),
            _dev_ptr(qbar_work, t, "qbar_work"),
            _dev_ptr(rows.edges, torch.float64, "edges"),
            _dev_ptr(v0, torch.float64, "v0"), float(dt), int(order), n,
            _dev_ptr(dvbar, t, "dvbar"), _dev_ptr(v0bar, torch.float64, "v0bar")))
        return qbar

    def ram_validate(self, rows: Rows, dtype, dv=None, dt: float = 0.0):
        self._stream()
        code = RAM_F64 if dtype == torch.float64 else RAM_F32
        check(self._lib.ram_validate(
            self._h, ctypes.byref(rows.layout), code,
            _dev_ptr(rows.edges, torch.float64, "edges"),
            None if dv is None else _dev_ptr(dv, dv.dtype, "dv"), float(dt)))


_contexts = {}


def context(device: Optional[int] = None) -> Context:
    """The per-device default context."""
    if device is None:
        device = torch.cuda.current_device()
    ctx = _contexts.get(device)
    if ctx is None:
        ctx = Context(device)
        _contexts[device] = ctx
    return ctx


def ram_shift(rows, q_in, q_out, v0, dt, order, scan=RAM_SCAN_F64):
    return context(q_in.device.index).ram_shift(rows, q_in, q_out, v0, dt, order, scan)


def ram_shift_limited(rows, q_in, q_out, v0, dt, recon):
    return context(q_in.device.index).ram_shift_limited(rows, q_in, q_out, v0, dt, recon)


def ram_step_limited(rows, q, v0, dv, dt, recon, n_steps):
    return context(q.device.index).ram_step_limited(rows, q, v0, dv, dt, recon, n_steps)


def ram_shift_limited_adjoint(rows, q_fwd, qbar_out, qbar_in, v0, dt, recon, v0bar=None):
    return context(qbar_out.device.index).ram_shift_limited_adjoint(
        rows, q_fwd, qbar_out, qbar_in, v0, dt, recon, v0bar)


def ram_step_limited_adjoint(rows, q_fwd, q_half, dv, qbar_out, qbar_in, v0, dt, recon,
                             dvbar=None, v0bar=None):
    return context(qbar_out.device.index).ram_step_limited_adjoint(
        rows, q_fwd, q_half, dv, qbar_out, qbar_in, v0, dt, recon, dvbar, v0bar)


def ram_step_tile_paths(rows, v0, dt, order, with_residual):
    return context(v0.device.index).ram_step_tile_paths(rows, v0, dt, order, with_residual)


def ram_row_norms(rows, q, q_ref=None, out=None):
    return context(q.device.index).ram_row_norms(rows, q, q_ref, out)


def ram_radial_step(rows, q_in, q_out, r_edges, u, dt):
    return context(q_in.device.index).ram_radial_step(rows, q_in, q_out, r_edges, u, dt)


def ram_step_split2d(rows, q, v0, dv, r_edges, u, dt, order, n_steps, scan=RAM_SCAN_F64,
                     recon=0):
    return context(q.device.index).ram_step_split2d(rows, q, v0, dv, r_edges, u, dt, order,
                                                    n_steps, scan, recon)


def ram_cell_average(rows, q_in, q_out, to_centre=False):
    return context(q_in.device.index).ram_cell_average(rows, q_in, q_out, to_centre)


def ram_step_point4(rows, q, v0, dv, dt, order, n_steps, scan=RAM_SCAN_F64, recon=0):
    return context(q.device.index).ram_step_point4(rows, q, v0, dv, dt, order, n_steps, scan,
                                                   recon)


def ram_residual(rows, q_in, q_out, dv, dt):
    return context(q_in.device.index).ram_residual(rows, q_in, q_out, dv, dt)


def ram_step(rows, q, v0, dv, dt, order, n_steps, scan=RAM_SCAN_F64):
    return context(q.device.index).ram_step(rows, q, v0, dv, dt, order, n_steps, scan)


def ram_shift_adjoint(rows, q_fwd, qbar_out, qbar_in, v0, dt, order,
                      v0bar=None, scan=RAM_SCAN_F64):
    return context(qbar_out.device.index).ram_shift_adjoint(
        rows, q_fwd, qbar_out, qbar_in, v0, dt, order, v0bar, scan)


def ram_residual_adjoint(rows, q_fwd, dv, qbar_out, qbar_in, dt, dvbar=None):
    return context(q_fwd.device.index).ram_residual_adjoint(
        rows, q_fwd, dv, qbar_out, qbar_in, dt, dvbar)


def ram_step_record(rows, q_traj, q_half, v0, dv, dt, order, n_steps, scan=RAM_SCAN_F64):
    return context(q_traj.device.index).ram_step_record(
        rows, q_traj, q_half, v0, dv, dt, order, n_steps, scan)


def ram_step_adjoint(rows, q_fwd, q_half, dv, qbar_out, qbar_in, v0, dt, order,
                     dvbar=None, v0bar=None):
    return context(qbar_out.device.index).ram_step_adjoint(
        rows, q_fwd, q_half, dv, qbar_out, qbar_in, v0, dt, order, dvbar, v0bar)


def ram_step_adjoint_steps(rows, q_traj, q_half, dv, qbar, qbar_work, v0, dt, order, n_steps,
                           dvbar=None, v0bar=None):
    return context(qbar.device.index).ram_step_adjoint_steps(
        rows, q_traj, q_half, dv, qbar, qbar_work, v0, dt, order, n_steps, dvbar, v0bar)


def ram_validate(rows, dtype, dv=None, dt=0.0):
    return context(rows.edges.device.index).ram_validate(rows, dtype, dv, dt)
