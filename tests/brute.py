"""Exact rational brute force for tiny rows (test pins for the oracle).

Independent of the oracle's formulation: instead of searching the cell of each
shifted node, summing whole-cell masses and differencing partial integrals, it
builds every source cell's reconstruction polynomial explicitly (exact
Vandermonde solve through the p+1 cumulative nodes, then its derivative) and
integrates each destination interval by enumerating its overlaps with every
periodic image of every source cell (Eq. mass_advected taken literally).

Also: the residual step with the PLM reconstruction of Section 3.1 and the
face flux taken as the exact integral of the upwind linear profile over the
swept interval.
"""
from __future__ import annotations

from fractions import Fraction as Fr
from typing import List, Sequence


def _solve(a: List[List[Fr]], b: List[Fr]) -> List[Fr]:
    n = len(b)
    m = [row[:] + [bb] for row, bb in zip(a, b)]
    for col in range(n):
        piv = next(r for r in range(col, n) if m[r][col] != 0)
        m[col], m[piv] = m[piv], m[col]
        for r in range(n):
            if r != col and m[r][col] != 0:
                f = m[r][col] / m[col][col]
                m[r] = [x - f * y for x, y in zip(m[r], m[col])]
    return [m[i][n] / m[i][i] for i in range(n)]


def _poly_eval(coef: Sequence[Fr], x: Fr) -> Fr:
    acc = Fr(0)
    for c in reversed(coef):
        acc = acc * x + c
    return acc


def reconstruction(edges: Sequence[Fr], q: Sequence[Fr], p: int):
    """Per source cell c: coefficients (in x) of the cumulative interpolant
    through nodes c-lo..c-lo+p of the periodically extended mesh."""
    n = len(q)
    L = edges[n] - edges[0]
    mass = [q[i] * (edges[i + 1] - edges[i]) for i in range(n)]
    tot = sum(mass, Fr(0))
    cum = [Fr(0)]
    for m in mass:
        cum.append(cum[-1] + m)

    def X(j):
        k, j0 = divmod(j, n)
        return edges[j0] + k * L

    def C(j):
        k, j0 = divmod(j, n)
        return cum[j0] + k * tot

    lo = (p - 1) // 2
    polys = []
    for c in range(n):
        nodes = [c - lo + a for a in range(p + 1)]
        A = [[X(j) ** k for k in range(p + 1)] for j in nodes]
        coef = _solve(A, [C(j) for j in nodes])
        polys.append(coef)
    return polys, mass


def shift_exact(edges: Sequence[Fr], q: Sequence[Fr], s: Fr, p: int) -> List[Fr]:
    """Exact cell averages after shifting by s (any sign, any size)."""
    n = len(q)
    L = edges[n] - edges[0]
    polys, mass = reconstruction(edges, q, p)
    # sanity: conservative per cell (Eq. Qmass_interp_1)
    for c in range(n):
        got = _poly_eval(polys[c], edges[c + 1]) - _poly_eval(polys[c], edges[c])
        assert got == mass[c]
    out = []
    for i in range(n):
        a, b = edges[i] - s, edges[i + 1] - s
        kmin = int((a - edges[0]) // L) - 1
        kmax = int((b - edges[0]) // L) + 1
        tot = Fr(0)
        for k in range(kmin, kmax + 1):
            for c in range(n):
                lo_c, hi_c = edges[c] + k * L, edges[c + 1] + k * L
                lo_, hi_ = max(a, lo_c), min(b, hi_c)
                if hi_ > lo_:
                    # image k of cell c: q~_c(x - kL)
                    tot += (_poly_eval(polys[c], hi_ - k * L)
                            - _poly_eval(polys[c], lo_ - k * L))
        out.append(tot / (edges[i + 1] - edges[i]))
    return out


def vl_slope_exact(edges, q, i):
    n = len(q)
    L = edges[n] - edges[0]

    def xc(j):
        k, j0 = divmod(j, n)
        return (edges[j0] + edges[j0 + 1]) / 2 + k * L

    def Q(j):
        return q[j % n]

    dp = (Q(i + 1) - Q(i)) / (xc(i + 1) - xc(i))
    dm = (Q(i) - Q(i - 1)) / (xc(i) - xc(i - 1))
    if dp * dm <= 0:
        return Fr(0)
    return 2 * dp * dm / (dp + dm)


def residual_exact(edges, q, dv, dt) -> List[Fr]:
    """Upwind PLM step with fluxes from exact swept-interval integrals."""
    n = len(q)
    sig = [vl_slope_exact(edges, q, i) for i in range(n)]
    xcen = [(edges[i] + edges[i + 1]) / 2 for i in range(n)]

    def lin_integral(u, a, b):
        # int_a^b (Q_u + sig_u (x - x_u)) dx
        return q[u] * (b - a) + sig[u] * ((b - xcen[u]) ** 2 - (a - xcen[u]) ** 2) / 2

    flux = []
    for f in range(n):
        v = dv[f]
        xf = edges[f]
        if v >= 0:
            u = (f - 1) % n
            xr = edges[u + 1]          # face f seen from cell f-1 (periodic)
            swept = lin_integral(u, xr - v * dt, xr) if v != 0 else Fr(0)
        else:
            u = f
            swept = -lin_integral(u, xf, xf - v * dt)
        flux.append(swept / dt)        # mass crossing the face per unit time
    out = []
    for i in range(n):
        dx = edges[i + 1] - edges[i]
        m = q[i] * dx - dt * (flux[(i + 1) % n] - flux[i])
        out.append(m / dx)
    return out


def to_fr(a) -> List[Fr]:
    return [Fr(x) for x in a]


def shift_piecewise_exact(edges: Sequence[Fr], qfun, s: Fr) -> List[Fr]:
    """Exact cell averages after shifting by s a piecewise function given
    pointwise: qfun(c, xi) is the value of source cell c's reconstruction at
    the normalised coordinate xi = (x - x_c)/dx_c in [0, 1].  Every overlap of
    a destination interval with a periodic image of a source cell is
    integrated by Simpson's rule, exact for the polynomials of degree <= 3 the
    limited reconstructions are (Eq. mass_advected taken literally)."""
    n = len(edges) - 1
    L = edges[n] - edges[0]
    out = []
    for i in range(n):
        a, b = edges[i] - s, edges[i + 1] - s
        kmin = int((a - edges[0]) // L) - 1
        kmax = int((b - edges[0]) // L) + 1
        tot = Fr(0)
        for k in range(kmin, kmax + 1):
            for c in range(n):
                lo_c, hi_c = edges[c] + k * L, edges[c + 1] + k * L
                lo_, hi_ = max(a, lo_c), min(b, hi_c)
                if hi_ > lo_:
                    h = edges[c + 1] - edges[c]
                    xa = (lo_ - lo_c) / h
                    xb = (hi_ - lo_c) / h
                    simpson = (qfun(c, xa) + 4 * qfun(c, (xa + xb) / 2) + qfun(c, xb)) / 6
                    tot += simpson * (hi_ - lo_)
        out.append(tot / (edges[i + 1] - edges[i]))
    return out


def lagrange_derivative(X: Sequence[Fr], Y: Sequence[Fr], t: Fr) -> Fr:
    """Derivative at t of the polynomial through the points (X[a], Y[a])."""
    m = len(X)
    tot = Fr(0)
    for a in range(m):
        for b in range(m):
            if b == a:
                continue
            term = Fr(1) / (X[a] - X[b])
            for c in range(m):
                if c != a and c != b:
                    term *= (t - X[c]) / (X[a] - X[c])
            tot += Y[a] * term
    return tot


def radial_exact(re, q, u, dt) -> List[Fr]:
    """Radial transport of one column in polar geometry, exactly: van Leer
    slopes from centre gaps (zero in the first and last rows), the flux
    through face f as the exact integral of the upwind row's linear profile
    over the swept interval divided by dt, the update divided by the row's
    area per unit angle; no flux through the inner and outer edges."""
    R = len(q)
    c = [(re[j] + re[j + 1]) / 2 for j in range(R)]

    def slope(j):
        if j == 0 or j == R - 1:
            return Fr(0)
        dp = (q[j + 1] - q[j]) / (c[j + 1] - c[j])
        dm = (q[j] - q[j - 1]) / (c[j] - c[j - 1])
        if dp * dm <= 0:
            return Fr(0)
        return 2 * dp * dm / (dp + dm)

    sig = [slope(j) for j in range(R)]

    def integral(w, a, b):
        # int_a^b (q_w + sig_w (r - c_w)) dr
        return q[w] * (b - a) + sig[w] * ((b - c[w]) ** 2 - (a - c[w]) ** 2) / 2

    flux = [Fr(0)] * (R + 1)
    for f in range(1, R):
        v = u[f]
        if v >= 0:
            flux[f] = integral(f - 1, re[f] - v * dt, re[f]) / dt if v != 0 else Fr(0)
        else:
            flux[f] = -integral(f, re[f], re[f] - v * dt) / dt
    out = []
    for j in range(R):
        area = (re[j + 1] ** 2 - re[j] ** 2) / 2
        out.append(q[j] - dt * (re[j + 1] * flux[j + 1] - re[j] * flux[j]) / area)
    return out
