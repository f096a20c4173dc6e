"""Seeded synthetic inputs for the RAM advection step.

This module only *generates* inputs (meshes, initial states, residual
velocities, bulk velocities, time steps).  It holds none of the transport
arithmetic: both the device path and the CPU oracle consume its arrays
unchanged, and neither is imported here.

Meshes
  * uniform and log-spaced node sets;
  * the periodic-bump mesh density of the paper's Appendix B.1 (two uniform
    resolution levels joined by a cos^2 ramp; normalisation Eq. Inorm), whose
    nodes satisfy F(x_j) = j with F = N * int psi / I_psi (Section 3.2.1,
    Eq. mesh, read with one index step per cell: N cells, N + 1 nodes);
  * randomly stretched rows (cell-size ratio bounded by a given factor).

Workloads (the five synthetic configurations)
  1. one periodic row, uniform dyadic mesh, N=256, smooth sine, 10.3 cells of
     shift per step, order 5, no residual velocity (the 1D test of Section 4.1
     re-shaped);
  2. polar disk 512 x 2048, log radii on [0.4, 2.5], periodic-bump azimuthal
     mesh 10x finer inside |phi| < 0.2, Keplerian per-row bulk speed, noisy
     residual velocity, Gaussian bump at the planet location (Section 4.2
     re-shaped);
  3. 4096 ragged rows of 64..8192 cells, random stretching with ratio <= 20;
  4. polar 1024 x 4096 (adjoint workload);
  5. polar 2048 x 16384 (production-shaped; throughput workload).

Seeds: ``20230509 + 10*cfg + stream`` with stream 0 = state noise, 1 =
residual velocity, 2 = row lengths and stretching, 3 = bulk speeds,
4 = target perturbation, 5 = finite-difference coordinates, 6 = radial
velocity.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED_BASE = 20230509


def seed_for(cfg: int, stream: int) -> int:
    return SEED_BASE + 10 * cfg + stream


def rng_for(cfg: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(seed_for(cfg, stream))


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------

def uniform_edges(n: int, x0: float = 0.0, x1: float = 1.0) -> np.ndarray:
    """N+1 uniformly spaced nodes on [x0, x1]."""
    j = np.arange(n + 1, dtype=np.float64)
    e = x0 + (x1 - x0) * j / n
    e[0], e[-1] = x0, x1
    return e


def log_edges(n: int, r0: float, r1: float) -> np.ndarray:
    """N+1 log-spaced radial nodes (radial bump of Appendix B.2 with c=0)."""
    e = np.geomspace(r0, r1, n + 1)
    e[0], e[-1] = r0, r1
    return e


def bump_density(s: np.ndarray, a: float, b: float, c: float) -> np.ndarray:
    """Unnormalised periodic-bump mesh density psi(s) (Appendix B.1)."""
    s = np.abs(np.asarray(s, dtype=np.float64))
    out = np.ones_like(s)
    out[s <= a] = 1.0 + c
    mid = (s > a) & (s < b)
    out[mid] = 1.0 + c * np.cos(0.5 * math.pi * (s[mid] - a) / (b - a)) ** 2
    return out


def bump_norm(xmin: float, xmax: float, a: float, b: float, c: float) -> float:
    """I_psi = (xmax - xmin) + c (a + b)  (Appendix B.1, Eq. Inorm)."""
    return (xmax - xmin) + c * (a + b)


def bump_cumulative(x, xmin: float, xmax: float, a: float, b: float,
                    c: float) -> np.ndarray:
    """Closed-form u(x) = int_{xmin}^{x} psi(s) ds / I_psi for the periodic bump.

    Written from the antiderivative of psi on each of its five pieces: the flat
    outer level (slope 1), the two cos^2 ramps (slope 1 + c/2 plus a sine term of
    half-period b - a) and the flat inner level (slope 1 + c).  Requires
    xmin <= -b < -a < 0 < a < b <= xmax.
    """
    x = np.asarray(x, dtype=np.float64)
    inorm = bump_norm(xmin, xmax, a, b, c)
    w = b - a

    def prim(t):
        # antiderivative of psi (unnormalised), continuous, with prim(0) = 0
        t = np.asarray(t, dtype=np.float64)
        at = np.abs(t)
        sgn = np.sign(t)
        inner = (1.0 + c) * at
        ramp = ((1.0 + c) * a + (1.0 + 0.5 * c) * (at - a)
                + 0.5 * c * w / math.pi * np.sin(math.pi * (at - a) / w))
        ramp_end = (1.0 + c) * a + (1.0 + 0.5 * c) * w
        outer = ramp_end + (at - b)
        val = np.where(at <= a, inner, np.where(at < b, ramp, outer))
        return sgn * val

    return (prim(x) - prim(xmin)) / inorm


def bump_edges(n: int, xmin: float, xmax: float, a: float, b: float, c: float,
               tol: float = 1e-15) -> np.ndarray:
    """Nodes of the periodic-bump mesh: F(x_j) = j with F = n * u, by bisection.

    Section 3.2.1 (Eq. mesh) defines the nodes implicitly; Appendix B says the
    paper solves it by bisection on the closed-form F.  Vectorised bisection on
    all interior nodes at once.
    """
    target = np.arange(1, n, dtype=np.float64) / n
    lo = np.full(n - 1, xmin)
    hi = np.full(n - 1, xmax)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        f = bump_cumulative(mid, xmin, xmax, a, b, c)
        below = f < target
        lo = np.where(below, mid, lo)
        hi = np.where(below, hi, mid)
        if np.max(hi - lo) <= tol * max(abs(xmin), abs(xmax), 1.0):
            break
    e = np.empty(n + 1)
    e[0], e[-1] = xmin, xmax
    e[1:-1] = 0.5 * (lo + hi)
    return e


def stretched_edges(n: int, ratio: float, rng: np.random.Generator,
                    x0: float = 0.0, x1: float = 1.0) -> np.ndarray:
    """Random stretching: widths ratio**u, u ~ U[0,1), normalised to [x0, x1]."""
    w = ratio ** rng.random(n)
    e = np.empty(n + 1)
    e[0] = 0.0
    np.cumsum(w, out=e[1:])
    e = x0 + (x1 - x0) * e / e[-1]
    e[0], e[-1] = x0, x1
    return e


# --------------------------------------------------------------------------
# exact cell averages used as initial states
# --------------------------------------------------------------------------

def sine_cell_averages(edges: np.ndarray, mean=1.0, amp=0.5, m=1.0,
                       phase=0.0, period=1.0) -> np.ndarray:
    """Exact cell averages of mean + amp*sin(2 pi m x / period + phase)."""
    k = 2.0 * math.pi * m / period
    a, b = edges[:-1], edges[1:]
    integ = -(np.cos(k * b + phase) - np.cos(k * a + phase)) / k
    return mean + amp * integ / (b - a)


def poly_cell_averages(edges: np.ndarray, coeffs) -> np.ndarray:
    """Exact cell averages of sum_k coeffs[k] x^k."""
    a, b = edges[:-1], edges[1:]
    tot = np.zeros_like(a)
    for k, ck in enumerate(coeffs):
        tot += ck * (b ** (k + 1) - a ** (k + 1)) / (k + 1)
    return tot / (b - a)


# --------------------------------------------------------------------------
# workload container
# --------------------------------------------------------------------------

@dataclass
class Workload:
    """Host arrays describing one batch of periodic rows.

    Layout: ``row_ptr`` (n_rows+1 cell offsets).  Uniform batches have
    ``n_cols > 0``; ragged ones ``n_cols == 0``.  ``edges`` is either one shared
    node array (``edges_shared``) or all rows' nodes concatenated, row r at
    offset ``row_ptr[r] + r`` with ``N_r + 1`` entries.  ``dv`` holds the
    residual velocity on faces: entry i of a row is face i-1/2 (left face of
    cell i).  ``v0`` is per row; the bulk shift of row r is ``v0[r]*dt``.
    """
    name: str
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray
    edges: np.ndarray
    edges_shared: bool
    q0: np.ndarray
    dv: Optional[np.ndarray]
    v0: np.ndarray
    dt: float
    order: int
    steps: int
    meta: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return int(self.row_ptr[-1])

    def row_edges(self, r: int) -> np.ndarray:
        if self.edges_shared:
            return self.edges
        off = int(self.row_ptr[r]) + r
        n = int(self.row_ptr[r + 1] - self.row_ptr[r])
        return self.edges[off:off + n + 1]


def _uniform_row_ptr(n_rows: int, n_cols: int) -> np.ndarray:
    return np.arange(n_rows + 1, dtype=np.int64) * n_cols


def residual_cfl_dt(edges: np.ndarray, dv: np.ndarray, beta: float = 0.5,
                    ) -> float:
    """dt = beta * min over faces of min(dx_left, dx_right)/|dv_f| (1D CFL rule
    of Section 4.1 applied to the residual velocity)."""
    dx = np.diff(edges)
    dx_left = np.roll(dx, 1)            # cell i-1 for face i-1/2 (periodic)
    lim = np.minimum(dx_left, dx)
    adv = np.abs(dv)
    with np.errstate(divide="ignore"):
        r = np.where(adv > 0, lim[None, :] / adv, np.inf)
    return float(beta * np.min(r))


def cfg1() -> Workload:
    """One periodic row, N=256 on [0,1), dyadic nodes x_j = j/256, exact cell
    averages of 1 + 0.5 sin(2 pi x), v0 = 1, dt = 10.3/256, order 5, 100 steps,
    no residual velocity."""
    n = 256
    edges = uniform_edges(n, 0.0, 1.0)
    q0 = sine_cell_averages(edges, 1.0, 0.5)
    return Workload("cfg1_row256_fp64", 1, n, _uniform_row_ptr(1, n), edges,
                    True, q0[None, :].copy(), None, np.array([1.0]),
                    10.3 / 256.0, 5, 100)


def polar(n_r: int, n_phi: int, cfg: int, order: int, steps: int,
          sigma: float = 0.05, noise: float = 1e-3, r0: float = 0.4,
          r1: float = 2.5, a: float = 0.2, b: float = 0.3, c: float = 9.0,
          name: str = "polar", phi: Optional[np.ndarray] = None) -> Workload:
    """Polar disk rows: one row per radius, azimuthal periodic-bump mesh
    (or the azimuthal edges ``phi`` given, n_phi + 1 of them on [-pi, pi]).

    v0_j = r_j^-1.5 (angular Keplerian speed, r_j the arithmetic centre);
    dv_{j,i-1/2} = 0.01 v0_j sin(phi_{i-1/2}) xi (xi ~ N(0,1), stream 1);
    Q0 = 1 + exp(-d^2/(2 sigma^2)) + noise*eta (stream 0) with
    d^2 = r^2 + 1 - 2 r cos(phi) (bump at the planet location (1, 0));
    dt from the residual CFL rule with beta = 0.5.
    """
    redges = log_edges(n_r, r0, r1)
    rc = 0.5 * (redges[:-1] + redges[1:])
    if phi is None:
        phi = bump_edges(n_phi, -math.pi, math.pi, a, b, c)
    pc = 0.5 * (phi[:-1] + phi[1:])
    v0 = rc ** -1.5
    xi = rng_for(cfg, 1).standard_normal((n_r, n_phi))
    dv = 0.01 * v0[:, None] * np.sin(phi[:-1])[None, :] * xi
    d2 = rc[:, None] ** 2 + 1.0 - 2.0 * rc[:, None] * np.cos(pc)[None, :]
    q0 = 1.0 + np.exp(-d2 / (2.0 * sigma ** 2))
    if noise:
        q0 += noise * rng_for(cfg, 0).standard_normal((n_r, n_phi))
    dt = residual_cfl_dt(phi, dv, 0.5)
    area = 0.5 * (redges[1:] ** 2 - redges[:-1] ** 2)[:, None] * np.diff(phi)[None, :]
    return Workload(name, n_r, n_phi, _uniform_row_ptr(n_r, n_phi), phi, True,
                    q0, dv, v0, dt, order, steps,
                    meta={"r_edges": redges, "area": area,
                          "bump": (a, b, c)})


def radial_velocity(wl: Workload, cfg: int, amp: float = 0.01) -> np.ndarray:
    """Radial velocity of a polar workload on its radial faces, [n_r + 1,
    n_phi] (face j between rows j-1 and j):
    u_{j-1/2,i} = amp r_{j-1/2}^-1/2 sin(phi_i) zeta (zeta ~ N(0,1), stream 6,
    phi_i the cell centre), a fraction `amp` of the Keplerian speed with the
    residual's angular pattern; zero on the inner and outer edges."""
    re = wl.meta["r_edges"]
    pc = 0.5 * (wl.edges[:-1] + wl.edges[1:])
    zeta = rng_for(cfg, 6).standard_normal((wl.n_rows + 1, wl.n_cols))
    u = amp * re[:, None] ** -0.5 * np.sin(pc)[None, :] * zeta
    u[0] = 0.0
    u[-1] = 0.0
    return u


def radial_cfl_dt(r_edges: np.ndarray, u: np.ndarray, beta: float = 0.5) -> float:
    """dt = beta * min over interior radial faces of min(dr_below, dr_above)/|u_f|
    (the residual's Courant rule across the rows)."""
    dr = np.diff(r_edges)
    lim = np.minimum(dr[:-1], dr[1:])[:, None]
    adv = np.abs(u[1:-1])
    with np.errstate(divide="ignore"):
        r = np.where(adv > 0, lim / adv, np.inf)
    return float(beta * np.min(r)) if r.size else math.inf


def cfl_2d_dt(phi_edges: np.ndarray, r_edges: np.ndarray, v_phi: np.ndarray,
              u: np.ndarray, beta: float = 0.5) -> float:
    """The 2D Courant rule of a split step (the advective terms of Section
    4.2's time-step estimate): dt = beta min over cells of
    [ |v_phi| / dphi + |u| / dr ]^-1, with v_phi the azimuthal (angular)
    velocity the row step advects with at the cell's left face and |u| the
    larger of the cell's two radial face speeds."""
    dphi = np.diff(phi_edges)[None, :]
    dr = np.diff(r_edges)[:, None]
    um = np.maximum(np.abs(u[:-1]), np.abs(u[1:]))
    rate = np.abs(v_phi) / dphi + um / dr
    return float(beta / np.max(rate))


def cfg2(order: int = 5) -> Workload:
    return polar(512, 2048, 2, order, 500, name=f"cfg2_polar512x2048_p{order}")


def cfg4() -> Workload:
    return polar(1024, 4096, 4, 5, 200, name="cfg4_polar1024x4096_adjoint")


def cfg5() -> Workload:
    """2048 x 16384 polar disk with a sigma = 0.01 planet-like density bump in
    the refined azimuthal zone; residual velocity from the same recipe."""
    return polar(2048, 16384, 5, 5, 1000, sigma=0.01, noise=0.0,
                 name="cfg5_polar2048x16384")


def stretched_disk(ratio: float = 8.0) -> Workload:
    """cfg5's disk (2048 x 16384, the same density bump, Keplerian shifts and
    residual recipe) on an azimuthal mesh of random cell sizes, widths
    ratio**u (u ~ U[0,1), stream 2 of seed 7): no run of equal cells, so
    every tile of the streaming step locates its shifted nodes."""
    phi = stretched_edges(16384, ratio, rng_for(7, 2), -math.pi, math.pi)
    return polar(2048, 16384, 5, 5, 1000, sigma=0.01, noise=0.0,
                 name=f"disk_stretched{ratio:g}_2048x16384", phi=phi)


def cfg3(n_rows: int = 4096, nmin: int = 64, nmax: int = 8192,
         ratio: float = 20.0, order: int = 5, steps: int = 200) -> Workload:
    """Ragged rows: N_r ~ U{nmin..nmax}, each row on [0,1) with stretched
    cells (ratio <= 20), v0_r ~ U[0.5, 20] mean cells per step (s_r = v0_r/N_r
    with dt = 1), Q0 = 1 + sum of 3 random sines as exact cell averages,
    no residual velocity."""
    rng = rng_for(3, 2)
    lens = rng.integers(nmin, nmax + 1, size=n_rows).astype(np.int64)
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    edges = np.empty(int(row_ptr[-1]) + n_rows)
    q0 = np.empty(int(row_ptr[-1]))
    rq = rng_for(3, 0)
    for r in range(n_rows):
        n = int(lens[r])
        e = stretched_edges(n, ratio, rng)
        edges[row_ptr[r] + r: row_ptr[r] + r + n + 1] = e
        q = np.ones(n)
        for _ in range(3):
            amp = rq.uniform(0.0, 0.25)
            m = int(rq.integers(1, 17))
            ph = rq.uniform(0.0, 2.0 * math.pi)
            q += sine_cell_averages(e, 0.0, amp, m, ph, 1.0)
        q0[row_ptr[r]: row_ptr[r + 1]] = q
    v0_cells = rng_for(3, 3).uniform(0.5, 20.0, size=n_rows)
    v0 = v0_cells / lens
    return Workload("cfg3_ragged4096", n_rows, 0, row_ptr, edges, False, q0,
                    None, v0, 1.0, order, steps)


def small_polar(n_r: int = 8, n_phi: int = 300, cfg: int = 2,
                order: int = 5) -> Workload:
    """A reduced polar workload with the same recipe (for parity tests)."""
    return polar(n_r, n_phi, cfg, order, 4, name=f"polar{n_r}x{n_phi}")


def small_ragged(n_rows: int = 24, nmin: int = 8, nmax: int = 700,
                 ratio: float = 20.0, seed: int = 7, order: int = 5,
                 with_dv: bool = True) -> Workload:
    """Reduced ragged batch (per-row stretched meshes) for parity tests."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(nmin, nmax + 1, size=n_rows).astype(np.int64)
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    edges = np.empty(int(row_ptr[-1]) + n_rows)
    q0 = np.empty(int(row_ptr[-1]))
    dv = np.empty(int(row_ptr[-1])) if with_dv else None
    dts = []
    for r in range(n_rows):
        n = int(lens[r])
        e = stretched_edges(n, ratio, rng)
        edges[row_ptr[r] + r: row_ptr[r] + r + n + 1] = e
        q0[row_ptr[r]: row_ptr[r + 1]] = (
            1.0 + sine_cell_averages(e, 0.0, 0.3, int(rng.integers(1, 5)),
                                     rng.uniform(0, 6.28), 1.0)
            + 0.05 * rng.standard_normal(n))
        if with_dv:
            d = 0.3 * rng.standard_normal(n)
            dv[row_ptr[r]: row_ptr[r + 1]] = d
            dts.append(residual_cfl_dt(e, d[None, :], 0.5))
    v0 = rng.uniform(-30.0, 30.0, size=n_rows) / lens
    dt = min(dts) if dts else 1.0
    v0 = v0 / dt   # shift of -30..30 mean cells per step
    return Workload(f"ragged{n_rows}", n_rows, 0, row_ptr, edges, False, q0,
                    dv, v0, dt, order, 3)


CONFIGS = {1: cfg1, 2: cfg2, 3: cfg3, 4: cfg4, 5: cfg5}
