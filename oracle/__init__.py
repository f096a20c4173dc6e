"""FP64 CPU oracle for the RAM advection step -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never calls it, and it
shares no code with the device library.

The arithmetic lives in ``ram_oracle.c`` (plain loops, FP64, fixed summation
order, one row at a time).  This module only marshals numpy arrays into it.
Every function follows one passage of the paper:

  shift            Section 3, Steps 1-3 (Eqs. Qmass_i, mass_advected,
                   condition_p, mass_shift_algo, step3), reconstruction read as
                   the derivative of the order-p Lagrange interpolant of the
                   node cumulative;
  residual         Eq. splitting_second with the PLM / van Leer slope of
                   Section 3.1 and the swept-interval upwind face state;
  step             the operator split of Section 1: shift, then residual;
  shift_recon      Section 3's remap with the limited reconstructions of
                   Section 3.1 (PLM / van Leer, PPM with App. A), and
  step_recon       the split step built on it;
  shift_recon_adjoint  transpose of the limited shift's Jacobian at the
                   forward state (the branch each limiter takes), plus dL/dv0;
  radial           the radial transport of a polar grid (the residual's upwind
                   scheme along r in polar geometry, closed edges);
  average4, point4 centre values -> cell averages with the fourth-order <Q>
                   correction of Section 3.1, and back; step_point4 composes
                   them with step for a state of centre values;
  shift_adjoint    transpose of the (linear) shift, plus dL/dv0;
  residual_adjoint transpose of the residual Jacobian, plus dL/d(dv).

Pins (tests/test_oracle_*.py) tie each function to what the paper and the
mathematics fix; see the test module docstrings.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ram_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libram_oracle.so")
# a separately built copy (the sanitizer test's ASan/UBSan build) can stand in
_LIB_OVERRIDE = os.environ.get("RAM_ORACLE_LIB")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over rows, no FP contraction)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _LIB_OVERRIDE:
        lib = ctypes.CDLL(_LIB_OVERRIDE)
    else:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    D = ctypes.c_double
    I = ctypes.c_int
    lib.oracle_shift.argtypes = [I64, P, P, I, P, P, P, D, I, I, I]
    lib.oracle_residual.argtypes = [I64, P, P, I, P, P, P, D, I]
    lib.oracle_step.argtypes = [I64, P, P, I, P, P, P, D, I, I64, I]
    lib.oracle_shift_adjoint.argtypes = [I64, P, P, I, P, P, P, P, D, I, P, I]
    lib.oracle_residual_adjoint.argtypes = [I64, P, P, I, P, P, P, P, P, D, I]
    lib.oracle_edges.argtypes = [P, P, I64, D, I, P, P, P, P, P]
    lib.oracle_max_threads.argtypes = []
    lib.oracle_shift_recon.argtypes = [I64, P, P, I, P, P, P, D, I, I]
    lib.oracle_step_recon.argtypes = [I64, P, P, I, P, P, P, D, I, I64, I]
    lib.oracle_recon_cells.argtypes = [P, P, I64, I, I, P, P, P]
    lib.oracle_edges_recon.argtypes = [P, P, I64, D, I, P, P]
    lib.oracle_shift_recon_adjoint.argtypes = [I64, P, P, I, P, P, P, P, D, I, P, I]
    lib.oracle_radial.argtypes = [I64, I64, P, P, P, D, P, I]
    lib.oracle_average4.argtypes = [I64, P, P, I, P, P, I, I]
    for f in ("oracle_shift", "oracle_residual", "oracle_step",
              "oracle_shift_adjoint", "oracle_residual_adjoint", "oracle_edges",
              "oracle_max_threads", "oracle_shift_recon", "oracle_step_recon",
              "oracle_recon_cells", "oracle_edges_recon", "oracle_shift_recon_adjoint",
              "oracle_radial", "oracle_average4"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class Rows:
    """Row geometry: ``row_ptr`` cell offsets and edges (shared or per row)."""

    def __init__(self, row_ptr, edges, shared: bool):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.edges = _f64(edges)
        self.shared = bool(shared)
        self.n_rows = len(self.row_ptr) - 1
        self.n_cells = int(self.row_ptr[-1])

    @classmethod
    def from_workload(cls, wl) -> "Rows":
        return cls(wl.row_ptr, wl.edges, wl.edges_shared)

    @classmethod
    def single(cls, edges) -> "Rows":
        edges = _f64(edges)
        return cls(np.array([0, len(edges) - 1]), edges, True)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def shift(rows: Rows, q, v0, dt: float, order: int, variant: int = 0,
          nthreads: int = 0) -> np.ndarray:
    """One bulk shift of every row (variant 0 local form, 1 global cumulative)."""
    q = _f64(q).reshape(-1)
    v0 = _f64(np.broadcast_to(v0, (rows.n_rows,)))
    out = np.empty_like(q)
    rc = _load().oracle_shift(rows.n_rows, _ptr(rows.row_ptr), _ptr(rows.edges),
                              int(rows.shared), _ptr(q), _ptr(out), _ptr(v0),
                              float(dt), int(order), int(variant), int(nthreads))
    _check(rc, "shift")
    return out


def residual(rows: Rows, q, dv, dt: float, nthreads: int = 0) -> np.ndarray:
    q = _f64(q).reshape(-1)
    dv = _f64(dv).reshape(-1)
    out = np.empty_like(q)
    rc = _load().oracle_residual(rows.n_rows, _ptr(rows.row_ptr),
                                 _ptr(rows.edges), int(rows.shared), _ptr(q),
                                 _ptr(out), _ptr(dv), float(dt), int(nthreads))
    _check(rc, "residual")
    return out


def step(rows: Rows, q, v0, dv, dt: float, order: int, n_steps: int,
         nthreads: int = 0) -> np.ndarray:
    """n_steps of shift then residual (dv None: shift only)."""
    q = _f64(q).reshape(-1).copy()
    v0 = _f64(np.broadcast_to(v0, (rows.n_rows,)))
    dvp = None if dv is None else _f64(dv).reshape(-1)
    rc = _load().oracle_step(rows.n_rows, _ptr(rows.row_ptr), _ptr(rows.edges),
                             int(rows.shared), _ptr(q), _ptr(v0), _ptr(dvp),
                             float(dt), int(order), int(n_steps), int(nthreads))
    _check(rc, "step")
    return q


def shift_adjoint(rows: Rows, q, qbar_out, v0, dt: float, order: int,
                  want_v0bar: bool = True, nthreads: int = 0):
    """Returns (qbar_in, v0bar) with v0bar = dt * d<qbar_out, S q>/ds per row."""
    q = _f64(q).reshape(-1)
    qb = _f64(qbar_out).reshape(-1)
    v0 = _f64(np.broadcast_to(v0, (rows.n_rows,)))
    out = np.empty_like(qb)
    v0bar = np.zeros(rows.n_rows) if want_v0bar else None
    rc = _load().oracle_shift_adjoint(rows.n_rows, _ptr(rows.row_ptr),
                                      _ptr(rows.edges), int(rows.shared),
                                      _ptr(q), _ptr(qb), _ptr(out), _ptr(v0),
                                      float(dt), int(order), _ptr(v0bar),
                                      int(nthreads))
    _check(rc, "shift_adjoint")
    return out, v0bar


def residual_adjoint(rows: Rows, q, dv, qbar_out, dt: float,
                     want_dvbar: bool = True, nthreads: int = 0):
    """Returns (qbar_in, dvbar) at the forward state q."""
    q = _f64(q).reshape(-1)
    dv = _f64(dv).reshape(-1)
    qb = _f64(qbar_out).reshape(-1)
    out = np.empty_like(qb)
    dvbar = np.zeros_like(qb) if want_dvbar else None
    rc = _load().oracle_residual_adjoint(rows.n_rows, _ptr(rows.row_ptr),
                                         _ptr(rows.edges), int(rows.shared),
                                         _ptr(q), _ptr(dv), _ptr(qb), _ptr(out),
                                         _ptr(dvbar), float(dt), int(nthreads))
    _check(rc, "residual_adjoint")
    return out, dvbar


def edges_info(x, q, s: float, order: int):
    """Per shifted node of one row: (xh, k, c, ell, dell) for e = 0..N-1."""
    x = _f64(x)
    q = _f64(q)
    n = len(q)
    xh = np.empty(n); ell = np.empty(n); dell = np.empty(n)
    k = np.empty(n, dtype=np.int64); c = np.empty(n, dtype=np.int64)
    _load().oracle_edges(_ptr(x), _ptr(q), n, float(s), int(order), _ptr(xh),
                         _ptr(k), _ptr(c), _ptr(ell), _ptr(dell))
    return xh, k, c, ell, dell


# limited reconstructions of the bulk shift (Section 3.1, App. A)
PLM = 1
PPM = 2
FREE_DELTA = 1      # recon_cells only: leave delta<Q> unlimited
FREE_PARABOLA = 2   # recon_cells only: skip the (QL, QR) constraints


def shift_recon(rows: Rows, q, v0, dt: float, recon: int,
                nthreads: int = 0) -> np.ndarray:
    """One bulk shift of every row with the PLM (1) or PPM (2) reconstruction."""
    q = _f64(q).reshape(-1)
    v0 = _f64(np.broadcast_to(v0, (rows.n_rows,)))
    out = np.empty_like(q)
    rc = _load().oracle_shift_recon(rows.n_rows, _ptr(rows.row_ptr), _ptr(rows.edges),
                                    int(rows.shared), _ptr(q), _ptr(out), _ptr(v0),
                                    float(dt), int(recon), int(nthreads))
    _check(rc, "shift_recon")
    return out


def step_recon(rows: Rows, q, v0, dv, dt: float, recon: int, n_steps: int,
               nthreads: int = 0) -> np.ndarray:
    """n_steps of limited shift then residual (dv None: shift only)."""
    q = _f64(q).reshape(-1).copy()
    v0 = _f64(np.broadcast_to(v0, (rows.n_rows,)))
    dvp = None if dv is None else _f64(dv).reshape(-1)
    rc = _load().oracle_step_recon(rows.n_rows, _ptr(rows.row_ptr), _ptr(rows.edges),
                                   int(rows.shared), _ptr(q), _ptr(v0), _ptr(dvp),
                                   float(dt), int(recon), int(n_steps), int(nthreads))
    _check(rc, "step_recon")
    return q


def recon_cells(x, q, recon: int, flags: int = 0):
    """Per cell of one row: PLM (Q, sigma, 0) or PPM (QL, QR, Q6)."""
    x = _f64(x)
    q = _f64(q)
    n = len(q)
    c0, c1, c2 = np.empty(n), np.empty(n), np.empty(n)
    rc = _load().oracle_recon_cells(_ptr(x), _ptr(q), n, int(recon), int(flags),
                                    _ptr(c0), _ptr(c1), _ptr(c2))
    _check(rc, "recon_cells")
    return c0, c1, c2


def edges_recon(x, q, s: float, recon: int):
    """Per shifted node of one row: extended source index g and partial integral."""
    x = _f64(x)
    q = _f64(q)
    n = len(q)
    g = np.empty(n, dtype=np.int64)
    ell = np.empty(n)
    rc = _load().oracle_edges_recon(_ptr(x), _ptr(q), n, float(s), int(recon),
                                    _ptr(g), _ptr(ell))
    _check(rc, "edges_recon")
    return g, ell


def shift_recon_adjoint(rows: Rows, q, qbar_out, v0, dt: float, recon: int,
                        want_v0bar: bool = True, nthreads: int = 0):
    """Transpose of the limited shift's Jacobian at q: (qbar_in, v0bar)."""
    q = _f64(q).reshape(-1)
    qb = _f64(qbar_out).reshape(-1)
    v0 = _f64(np.broadcast_to(v0, (rows.n_rows,)))
    out = np.empty_like(qb)
    v0bar = np.zeros(rows.n_rows) if want_v0bar else None
    rc = _load().oracle_shift_recon_adjoint(rows.n_rows, _ptr(rows.row_ptr),
                                            _ptr(rows.edges), int(rows.shared), _ptr(q),
                                            _ptr(qb), _ptr(out), _ptr(v0), float(dt),
                                            int(recon), _ptr(v0bar), int(nthreads))
    _check(rc, "shift_recon_adjoint")
    return out, v0bar


def radial(r_edges, q, u, dt: float, nthreads: int = 0) -> np.ndarray:
    """Radial transport step: q [n_rows, n_cols] (rows = radii), u
    [n_rows + 1, n_cols] on the radial faces, r_edges [n_rows + 1]."""
    re = _f64(r_edges)
    q = _f64(q)
    u = _f64(u)
    n_rows, n_cols = q.shape
    assert u.shape == (n_rows + 1, n_cols) and re.shape == (n_rows + 1,)
    out = np.empty_like(q)
    rc = _load().oracle_radial(n_rows, n_cols, _ptr(re), _ptr(q), _ptr(u), float(dt),
                               _ptr(out), int(nthreads))
    _check(rc, "radial")
    return out


def average4(rows: Rows, q, inverse: bool = False, nthreads: int = 0) -> np.ndarray:
    """Centre values -> cell averages, <Q>_i = Q_i + dx_i^2 Q''_i / 24 with the
    three-point Q'' through the neighbouring centres (inverse: averages ->
    centre values, subtracting the same correction)."""
    q = _f64(q).reshape(-1)
    out = np.empty_like(q)
    rc = _load().oracle_average4(rows.n_rows, _ptr(rows.row_ptr), _ptr(rows.edges),
                                 int(rows.shared), _ptr(q), _ptr(out), int(bool(inverse)),
                                 int(nthreads))
    _check(rc, "average4")
    return out


def point4(rows: Rows, qavg, nthreads: int = 0) -> np.ndarray:
    """Cell averages -> centre values (the inverse of average4)."""
    return average4(rows, qavg, True, nthreads)


def step_point4(rows: Rows, q, v0, dv, dt: float, order: int, n_steps: int,
                nthreads: int = 0) -> np.ndarray:
    """n steps on a state of centre values: each step converts to cell
    averages, takes the split step (shift, then residual), and converts
    back."""
    q = _f64(q).reshape(-1).copy()
    for _ in range(n_steps):
        a = average4(rows, q, False, nthreads)
        a = step(rows, a, v0, dv, dt, order, 1, nthreads)
        q = average4(rows, a, True, nthreads)
    return q
