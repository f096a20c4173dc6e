/*
 * ram_oracle.c -- plain, slow FP64 CPU oracle for the RAM advection step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the device path.
 *
 * What it computes, per periodic row of N cells bounded by N+1 nodes x[0..N]
 * (Section 2 of the paper):
 *
 *   shift      the bulk step of the operator split (Section 1, Eq.
 *              splitting_first): the conservative remap of Section 3, Steps 1-3
 *              (Eqs. Qmass_i, mass_advected, condition_p, mass_shift_algo,
 *              step3).  The reconstruction q~ inside source cell c is the
 *              derivative of the degree-p Lagrange interpolant of the node
 *              cumulative C through the p+1 nodes c-lo .. c-lo+p (lo=(p-1)/2).
 *              The mass of a destination cell is then the whole-cell masses it
 *              covers plus two partial integrals of q~, exactly the shape of
 *              Eq. mass_shift_algo.  Node N is node 0 of the next period
 *              ("p(N) = p(0)", Section 3.2).
 *   residual   the second half of the split (Eq. splitting_second): a finite-
 *              volume upwind step with the PLM reconstruction and the van Leer
 *              harmonic slope of Section 3.1; the face state is the average of
 *              the upwind linear profile over the swept interval, i.e. Eq.
 *              mass_shift_algo in its sub-cell (Lufkin) limit of Section 3.2.
 *   step       shift, then residual (Section 1).
 *   radial     the radial transport of a polar grid (standard upwind along r in
 *              polar geometry, closed edges), the other half of a 2D split step.
 *   average4   centre values -> cell averages with the fourth-order correction
 *              of Section 3.1 (and the inverse), for a state of point values.
 *   shift_recon the same remap with the limited (monotone) reconstructions of
 *              Section 3.1 instead: PLM with the van Leer slope, or PPM with
 *              the interface values and constraints of App. A.
 *   adjoints   transposes of the two linearised maps, written as scatter loops
 *              (the device path gathers); plus the derivative w.r.t. the bulk
 *              speed v0 (through x~ = x - v0 dt, Section 3.2).
 *
 * Everything is FP64, in a fixed summation order; build with
 * -O2 -ffp-contract=off.  OpenMP parallelises over independent rows only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_ORDER 9

static int64_t wrap(int64_t m, int64_t n)
{
    int64_t r = m % n;
    return r < 0 ? r + n : r;
}

/* Node coordinate of the periodically extended mesh, j in [-N, 2N]. */
static double node_x(const double *x, int64_t n, double len, int64_t j)
{
    if (j < 0) return x[j + n] - len;
    if (j > n) return x[j - n] + len;
    return x[j];
}

/* Mass of (wrapped) cell m. */
static double cell_mass(const double *x, const double *q, int64_t n, int64_t m)
{
    int64_t w = wrap(m, n);
    return q[w] * (x[w + 1] - x[w]);
}

/* C(j) - C(c) for extended node indices, summed over the cells in between in
 * ascending order (no global prefix, so it is exact for a single cell). */
static double cum_diff(const double *x, const double *q, int64_t n, int64_t c,
                       int64_t j)
{
    double s = 0.0;
    if (j > c) {
        for (int64_t m = c; m < j; ++m) s += cell_mass(x, q, n, m);
        return s;
    }
    for (int64_t m = j; m < c; ++m) s += cell_mass(x, q, n, m);
    return -s;
}

/* Largest j in [0, n-1] with x[j] <= xh (Eq. condition_p; right-continuous). */
static int64_t find_cell(const double *x, int64_t n, double xh)
{
    int64_t lo = 0, hi = n - 1;
    if (!(xh >= x[0])) return 0;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo + 1) / 2;
        if (x[mid] <= xh) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* Shifted node: x~ = x_e - s, written as xh + k L with xh in [x0, xN). */
static void shifted_node(const double *x, int64_t n, double s, int64_t e,
                         double *xh_out, int64_t *k_out)
{
    double len = x[n] - x[0];
    double xt = x[e] - s;
    double kf = floor((xt - x[0]) / len);
    double xh = xt - kf * len;
    int64_t k = (int64_t)kf;
    if (xh >= x[n]) { xh -= len; k += 1; }
    else if (xh < x[0]) { xh += len; k -= 1; }
    *xh_out = xh;
    *k_out = k;
}

/* Lagrange basis weight a on nodes X[0..p] evaluated at t. */
static double lagrange_w(const double *X, int p, int a, double t)
{
    double w = 1.0;
    for (int b = 0; b <= p; ++b)
        if (b != a) w *= (t - X[b]) / (X[a] - X[b]);
    return w;
}

/* Derivative of the Lagrange basis weight a at t. */
static double lagrange_dw(const double *X, int p, int a, double t)
{
    double tot = 0.0;
    for (int b = 0; b <= p; ++b) {
        if (b == a) continue;
        double term = 1.0 / (X[a] - X[b]);
        for (int c = 0; c <= p; ++c)
            if (c != a && c != b) term *= (t - X[c]) / (X[a] - X[c]);
        tot += term;
    }
    return tot;
}

typedef struct {
    double xh;      /* wrapped shifted node */
    int64_t k;      /* wrap count */
    int64_t c;      /* source cell containing xh */
    int64_t g;      /* extended source index c + k N */
    double ell;     /* C~(xh) - C(c): the partial integral of q~_c */
    double dell;    /* q~_c(xh) = d C~ / dx at xh */
} edge_t;

/* Step 1 + the partial integrals of Step 2 for one shifted node. */
static void edge_eval(const double *x, const double *q, int64_t n, double s,
                      int p, int64_t e, int want_deriv, edge_t *out)
{
    double len = x[n] - x[0];
    int lo = (p - 1) / 2;
    double X[ORACLE_MAX_ORDER + 1], D[ORACLE_MAX_ORDER + 1];
    shifted_node(x, n, s, e, &out->xh, &out->k);
    out->c = find_cell(x, n, out->xh);
    out->g = out->c + out->k * n;
    for (int a = 0; a <= p; ++a) {
        int64_t j = out->c - lo + a;
        X[a] = node_x(x, n, len, j);
        D[a] = cum_diff(x, q, n, out->c, j);
    }
    double ell = 0.0, dell = 0.0;
    for (int a = 0; a <= p; ++a) {
        ell += lagrange_w(X, p, a, out->xh) * D[a];
        if (want_deriv) dell += lagrange_dw(X, p, a, out->xh) * D[a];
    }
    out->ell = ell;
    out->dell = dell;
}

/* ---------------------------------------------------------------------- */
/* bulk shift of one row                                                    */
/* ---------------------------------------------------------------------- */

/* variant 0: local form  M'_i = sum_{m=g_i}^{g_{i+1}-1} M_m + ell_{i+1} - ell_i
 * variant 1: global form M'_i = (C(g_{i+1}) + ell_{i+1}) - (C(g_i) + ell_i)
 *            with the extended cumulative C(j + kN) = C(j) + k M_tot. */
static int shift_row(const double *x, const double *q, double *qout, int64_t n,
                     double s, int p, int variant)
{
    edge_t *ed = (edge_t *)malloc(sizeof(edge_t) * (size_t)(n + 1));
    double *cum = NULL;
    if (!ed) return -6;
    for (int64_t e = 0; e < n; ++e) edge_eval(x, q, n, s, p, e, 0, &ed[e]);
    ed[n] = ed[0];
    ed[n].k += 1;
    ed[n].g += n;
    if (variant == 1) {
        cum = (double *)malloc(sizeof(double) * (size_t)(n + 1));
        if (!cum) { free(ed); return -6; }
        cum[0] = 0.0;
        for (int64_t m = 0; m < n; ++m) cum[m + 1] = cum[m] + cell_mass(x, q, n, m);
    }
    for (int64_t i = 0; i < n; ++i) {
        double dx = x[i + 1] - x[i];
        double mp;
        if (variant == 0) {
            double whole = 0.0;
            for (int64_t m = ed[i].g; m < ed[i + 1].g; ++m) whole += cell_mass(x, q, n, m);
            mp = whole + ed[i + 1].ell - ed[i].ell;
        } else {
            int64_t ga = ed[i].g, gb = ed[i + 1].g;
            int64_t ka = (ga - wrap(ga, n)) / n, kb = (gb - wrap(gb, n)) / n;
            double va = cum[wrap(ga, n)] + (double)ka * cum[n] + ed[i].ell;
            double vb = cum[wrap(gb, n)] + (double)kb * cum[n] + ed[i + 1].ell;
            mp = vb - va;
        }
        qout[i] = mp / dx;
    }
    free(ed);
    free(cum);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* residual upwind step of one row                                          */
/* ---------------------------------------------------------------------- */

static double centre(const double *x, int64_t i) { return 0.5 * (x[i] + x[i + 1]); }

/* distance between the centres of cells i and i+1 (periodic) */
static double centre_gap(const double *x, int64_t n, int64_t i)
{
    double len = x[n] - x[0];
    int64_t w = wrap(i, n);
    if (w == n - 1) return centre(x, 0) + len - centre(x, n - 1);
    return centre(x, w + 1) - centre(x, w);
}

/* van Leer harmonic slope of cell i (Section 3.1) */
static double vl_slope(const double *x, const double *q, int64_t n, int64_t i)
{
    double qm = q[wrap(i - 1, n)], q0 = q[wrap(i, n)], qp = q[wrap(i + 1, n)];
    double dp = (qp - q0) / centre_gap(x, n, i);
    double dm = (q0 - qm) / centre_gap(x, n, i - 1);
    if (dp * dm <= 0.0) return 0.0;
    return 2.0 * dp * dm / (dp + dm);
}

/* upwind face state on face f (between cells f-1 and f) */
static double face_state(const double *x, const double *q, int64_t n, int64_t f,
                         double v, double dt)
{
    if (v >= 0.0) {
        int64_t u = wrap(f - 1, n);
        double dx = x[u + 1] - x[u];
        return q[u] + 0.5 * vl_slope(x, q, n, u) * (dx - v * dt);
    } else {
        int64_t u = wrap(f, n);
        double dx = x[u + 1] - x[u];
        return q[u] - 0.5 * vl_slope(x, q, n, u) * (dx + v * dt);
    }
}

static int residual_row(const double *x, const double *q, const double *dv,
                        double *qout, int64_t n, double dt)
{
    for (int64_t i = 0; i < n; ++i) {
        double dx = x[i + 1] - x[i];
        double fl = dv[i] * face_state(x, q, n, i, dv[i], dt);
        int64_t r = wrap(i + 1, n);
        double fr = dv[r] * face_state(x, q, n, r, dv[r], dt);
        /* M'' = M - dt (F_{i+1/2} - F_{i-1/2}), divided by dx (Eq. step3);
         * written on Q so that dv = 0 is an exact identity */
        qout[i] = q[i] - dt * (fr - fl) / dx;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* limited (monotone) reconstructions for the bulk shift                    */
/* ---------------------------------------------------------------------- */
/*
 * The two reconstructions Section 3.1 uses for Step 1 of the shift:
 *
 *   PLM   q_c(x) = Q_c + sigma_c (x - x_c), x_c the cell centre (Section 2),
 *         sigma_c the van Leer harmonic slope (the same slope as the residual).
 *   PPM   the parabola of Colella & Woodward (1984) in the form Section 3.1
 *         writes it, q_c = QL + xi (QR - QL) + Q6 xi (1 - xi),
 *         Q6 = 6 Q_c - 3 (QL + QR), with xi = (x - x_{c-1/2}) / dx_c measured
 *         from the cell's left node (the reading under which the parabola keeps
 *         the cell's mass, Eq. Qmass_interp_1).  QL and QR are the interface
 *         values of App. A (interpolation of the averages, limited slope
 *         delta<Q>) after the App. A monotonicity constraints.
 *
 * App. A reading: the weights w1, w2, w3 take SUMS of neighbouring cell sizes
 * where the printed text shows products (Colella & Woodward's Eq. 1.6; the
 * printed products are not even dimensionally consistent), the limited slope
 * keeps the sign of the unlimited one (their Eq. 1.8), and the third
 * constraint reads -(QR - QL)^2 / 6 > (QR - QL) Qa.
 *
 * flags (used by the pins only): RECON_FREE_DELTA leaves delta<Q> unlimited,
 * RECON_FREE_PARABOLA skips the constraints on (QL, QR).
 */
#define RECON_PLM 1
#define RECON_PPM 2
#define RECON_FREE_DELTA 1
#define RECON_FREE_PARABOLA 2

/* size and average of (wrapped) cell m */
static double dx_w(const double *x, int64_t n, int64_t m)
{
    int64_t w = wrap(m, n);
    return x[w + 1] - x[w];
}

static double q_w(const double *q, int64_t n, int64_t m) { return q[wrap(m, n)]; }

/* delta<Q>_j of App. A: the slope of cell j times its size, limited so that
 * the interface values stay between neighbouring averages */
static double ppm_delta(const double *x, const double *q, int64_t n, int64_t j,
                        int flags)
{
    double hm = dx_w(x, n, j - 1), h0 = dx_w(x, n, j), hp = dx_w(x, n, j + 1);
    double up = q_w(q, n, j + 1) - q_w(q, n, j);
    double dn = q_w(q, n, j) - q_w(q, n, j - 1);
    double d = h0 / (hm + h0 + hp) *
               ((2.0 * hm + h0) / (hp + h0) * up + (h0 + 2.0 * hp) / (hm + h0) * dn);
    if (flags & RECON_FREE_DELTA) return d;
    if (up * dn <= 0.0) return 0.0;
    double mag = fmin(fabs(d), fmin(2.0 * fabs(up), 2.0 * fabs(dn)));
    return copysign(mag, d);
}

/* <Q>_{j+1/2}: the value on the node between cells j and j+1 (App. A) */
static double ppm_interface(const double *x, const double *q, int64_t n,
                            int64_t j, int flags)
{
    double hm = dx_w(x, n, j - 1), h0 = dx_w(x, n, j);
    double hp = dx_w(x, n, j + 1), hpp = dx_w(x, n, j + 2);
    double a0 = q_w(q, n, j), a1 = q_w(q, n, j + 1);
    double w1 = 2.0 * hp * h0 / (h0 + hp) *
                ((hm + h0) / (2.0 * h0 + hp) - (hpp + hp) / (2.0 * hp + h0));
    double w2 = -h0 * (hm + h0) / (2.0 * h0 + hp);
    double w3 = hp * (hp + hpp) / (h0 + 2.0 * hp);
    double corr = w1 * (a1 - a0) + w2 * ppm_delta(x, q, n, j + 1, flags) +
                  w3 * ppm_delta(x, q, n, j, flags);
    return a0 + h0 / (h0 + hp) * (a1 - a0) + corr / (hm + h0 + hp + hpp);
}

/* (QL, QR, Q6) of cell c after the App. A constraints */
static void ppm_parabola(const double *x, const double *q, int64_t n, int64_t c,
                         int flags, double *ql, double *qr, double *q6)
{
    double a = q_w(q, n, c);
    double L = ppm_interface(x, q, n, c - 1, flags);
    double R = ppm_interface(x, q, n, c, flags);
    if (!(flags & RECON_FREE_PARABOLA)) {
        if ((R - a) * (a - L) <= 0.0) {
            /* a local extremum: the cell is flat */
            L = a;
            R = a;
        } else {
            double dq = R - L, qa = a - 0.5 * (L + R);
            if (dq * qa > dq * dq / 6.0) L = 3.0 * a - 2.0 * R;
            else if (-dq * dq / 6.0 > dq * qa) R = 3.0 * a - 2.0 * L;
        }
    }
    *ql = L;
    *qr = R;
    *q6 = 6.0 * a - 3.0 * (L + R);
}

/* Integral of the limited q_c from the cell's left node to xh (Step 2's partial
 * integral; x_c <= xh <= x_{c+1}, c in [0, n-1]). */
static double limited_partial(const double *x, const double *q, int64_t n,
                              int64_t c, double xh, int recon)
{
    double xl = x[c], h = x[c + 1] - x[c];
    if (recon == RECON_PLM) {
        double xc = centre(x, c), sig = vl_slope(x, q, n, c);
        /* antiderivative of Q_c + sigma (y - x_c) between xl and xh */
        return q[c] * (xh - xl) +
               0.5 * sig * ((xh - xc) * (xh - xc) - (xl - xc) * (xl - xc));
    }
    double ql, qr, q6;
    ppm_parabola(x, q, n, c, 0, &ql, &qr, &q6);
    double th = (xh - xl) / h;
    return h * (ql * th + 0.5 * (qr - ql) * th * th +
                q6 * (0.5 * th * th - th * th * th / 3.0));
}

/* Bulk shift with a limited reconstruction, in the local form
 * M'_i = sum_{m=g_i}^{g_{i+1}-1} M_m + ell_{i+1} - ell_i (Eq. mass_shift_algo). */
static int shift_row_recon(const double *x, const double *q, double *qout,
                           int64_t n, double s, int recon)
{
    int64_t *g = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    double *ell = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    if (!g || !ell) { free(g); free(ell); return -6; }
    for (int64_t e = 0; e < n; ++e) {
        double xh;
        int64_t k;
        shifted_node(x, n, s, e, &xh, &k);
        int64_t c = find_cell(x, n, xh);
        g[e] = c + k * n;
        ell[e] = limited_partial(x, q, n, c, xh, recon);
    }
    /* node N is node 0 one period on */
    g[n] = g[0] + n;
    ell[n] = ell[0];
    for (int64_t i = 0; i < n; ++i) {
        double whole = 0.0;
        for (int64_t m = g[i]; m < g[i + 1]; ++m) whole += cell_mass(x, q, n, m);
        qout[i] = (whole + ell[i + 1] - ell[i]) / (x[i + 1] - x[i]);
    }
    free(g);
    free(ell);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* radial transport of a polar grid (the other half of a 2D split step)     */
/* ---------------------------------------------------------------------- */
/*
 * Rows are radii, bounded by the radial edges re[0..R]; each azimuthal column
 * is advected along r by the radial velocity u on the radial faces (face j at
 * radius re[j], between rows j-1 and j) with the standard upwind scheme of the
 * residual step (PLM, van Leer slope, swept-interval face value) in polar
 * geometry: per unit angle a face has length re[j] and row j the area
 * A_j = (re[j+1]^2 - re[j]^2) / 2, so
 *     q'_j = q_j - dt (re[j+1] F_{j+1} - re[j] F_j) / A_j,   F = u q*.
 * The inner and outer edges are closed (no flux through them) and the first
 * and last rows take a zero slope.  This is how Section 3's dimensional
 * splitting combines RAM along the bulk flow with standard transport across
 * it; the column scheme is this build's reading of that standard transport.
 */
static double rc_centre(const double *re, int64_t j) { return 0.5 * (re[j] + re[j + 1]); }

static double radial_slope(const double *re, const double *q, int64_t R, int64_t j)
{
    if (j <= 0 || j >= R - 1) return 0.0;
    double dp = (q[j + 1] - q[j]) / (rc_centre(re, j + 1) - rc_centre(re, j));
    double dm = (q[j] - q[j - 1]) / (rc_centre(re, j) - rc_centre(re, j - 1));
    if (dp * dm <= 0.0) return 0.0;
    return 2.0 * dp * dm / (dp + dm);
}

/* one column: q[R] -> out[R], u[R+1] on the faces */
static void radial_column(const double *re, int64_t R, const double *q, const double *u,
                          double dt, double *out)
{
    for (int64_t j = 0; j < R; ++j) {
        double fl = 0.0, fr = 0.0;
        for (int side = 0; side < 2; ++side) {
            int64_t f = j + side;                 /* face f between rows f-1 and f */
            if (f == 0 || f == R) continue;       /* closed edges */
            double v = u[f], qs;
            if (v >= 0.0) {
                int64_t w = f - 1;
                qs = q[w] + 0.5 * radial_slope(re, q, R, w) * ((re[w + 1] - re[w]) - v * dt);
            } else {
                int64_t w = f;
                qs = q[w] - 0.5 * radial_slope(re, q, R, w) * ((re[w + 1] - re[w]) + v * dt);
            }
            if (side == 0) fl = re[f] * v * qs; else fr = re[f] * v * qs;
        }
        double area = 0.5 * (re[j + 1] * re[j + 1] - re[j] * re[j]);
        out[j] = q[j] - dt * (fr - fl) / area;
    }
}

/* ---------------------------------------------------------------------- */
/* point values <-> cell averages (the fourth-order <Q> correction)         */
/* ---------------------------------------------------------------------- */
/*
 * Section 3.1 notes that taking the state Q_i as the cell average <Q>_i is a
 * second-order assumption and names the fourth-order correction
 * <Q>_i = Q_i + (Q_{i+1} - 2 Q_i + Q_{i-1}) / 24 on a uniform periodic mesh.
 * With Q_i the value at the cell's centre, the average is
 * Q_i + dx_i^2 Q''(x_i) / 24 + O(dx^4) (the midpoint expansion has no odd
 * terms).  On any mesh Q'' is taken as the three-point second derivative
 * through the centres of cells i-1, i, i+1 (periodic), which reduces to the
 * paper's formula on a uniform mesh.  The inverse map takes averages back to
 * centre values by subtracting the same correction formed from the averages;
 * both are fourth-order accurate on smooth meshes.
 */
static void average4_row(const double *x, const double *q, double *out, int64_t n,
                         int inverse)
{
    for (int64_t i = 0; i < n; ++i) {
        const double gm = centre_gap(x, n, i - 1), gp = centre_gap(x, n, i);
        const double qm = q[wrap(i - 1, n)], q0 = q[i], qp = q[wrap(i + 1, n)];
        const double d2 = 2.0 * ((qp - q0) / gp - (q0 - qm) / gm) / (gm + gp);
        const double dx = x[i + 1] - x[i];
        const double corr = dx * dx / 24.0 * d2;
        out[i] = inverse ? q0 - corr : q0 + corr;
    }
}

/* ---- linearisation of the limited shift (its adjoint) ------------------ */
/*
 * The limited shift is nonlinear in Q; its adjoint is the transpose of its
 * Jacobian at the forward state.  Away from the limiters' switching points the
 * Jacobian is that of the branch each limiter takes there; at a switching
 * point the branch the forward evaluation takes is used (a zero slope where
 * the one-sided differences do not share a sign, as for the residual).
 *
 * lim_partial_grad: the partial integral ell of source cell c at xh, its
 * derivatives g[a] = d ell / d Q_{c-lo+a} (a = 0 .. 2 lo, lo = 1 PLM, 2 PPM),
 * and the reconstruction's value q_c(xh) = d ell / d xh.
 */
static double lim_partial_grad(const double *x, const double *q, int64_t n,
                               int64_t c, double xh, int recon, double *g,
                               double *qval)
{
    double xl = x[c], h = x[c + 1] - x[c];
    double th = (xh - xl) / h;
    if (recon == RECON_PLM) {
        double qm = q_w(q, n, c - 1), q0 = q[c], qp = q_w(q, n, c + 1);
        double hp = centre_gap(x, n, c), hm = centre_gap(x, n, c - 1);
        double a = (qp - q0) / hp, b = (q0 - qm) / hm;
        double sig = 0.0, dsa = 0.0, dsb = 0.0;
        if (a * b > 0.0) {
            sig = 2.0 * a * b / (a + b);
            dsa = 2.0 * b * b / ((a + b) * (a + b));
            dsb = 2.0 * a * a / ((a + b) * (a + b));
        }
        /* ell = Q_c h th + sigma h^2 (th^2 - th) / 2 */
        double ks = 0.5 * h * h * (th * th - th);
        g[0] = ks * dsb * (-1.0 / hm);
        g[1] = h * th + ks * (dsa * (-1.0 / hp) + dsb * (1.0 / hm));
        g[2] = ks * dsa * (1.0 / hp);
        *qval = q0 + sig * (xh - centre(x, c));
        return q0 * h * th + ks * sig;
    }
    /* PPM: cells c-2 .. c+2 */
    double av[5], hv[6];
    for (int k = 0; k < 5; ++k) av[k] = q_w(q, n, c - 2 + k);
    for (int k = 0; k < 6; ++k) hv[k] = dx_w(x, n, c - 2 + k);
    /* limited slopes of cells c-1, c, c+1 (index k = 0, 1, 2) and their
     * derivatives w.r.t. the averages of cells j-1, j, j+1 */
    double dl[3], dd[3][3];
    for (int k = 0; k < 3; ++k) {
        double hm = hv[k], h0 = hv[k + 1], hp = hv[k + 2];
        double up = av[k + 2] - av[k + 1], dn = av[k + 1] - av[k];
        double f = h0 / (hm + h0 + hp);
        double w1 = f * (2.0 * hm + h0) / (hp + h0), w2 = f * (h0 + 2.0 * hp) / (hm + h0);
        double d = w1 * up + w2 * dn;
        dd[k][0] = dd[k][1] = dd[k][2] = 0.0;
        dl[k] = 0.0;
        if (up * dn > 0.0) {
            double mag = fmin(fabs(d), fmin(2.0 * fabs(up), 2.0 * fabs(dn)));
            dl[k] = copysign(mag, d);
            if (fabs(d) <= 2.0 * fabs(up) && fabs(d) <= 2.0 * fabs(dn)) {
                dd[k][0] = -w2; dd[k][1] = w2 - w1; dd[k][2] = w1;
            } else if (fabs(up) <= fabs(dn)) {
                dd[k][1] = -2.0; dd[k][2] = 2.0;          /* 2 up */
            } else {
                dd[k][0] = -2.0; dd[k][1] = 2.0;          /* 2 dn */
            }
        }
    }
    /* interfaces c-1/2 (between cells c-1, c) and c+1/2 (c, c+1) */
    double ew[2][3];
    for (int side = 0; side < 2; ++side) {
        double hm = hv[side], h0 = hv[side + 1], hp = hv[side + 2], hpp = hv[side + 3];
        double w1 = 2.0 * hp * h0 / (h0 + hp) *
                    ((hm + h0) / (2.0 * h0 + hp) - (hpp + hp) / (2.0 * hp + h0));
        double inv = 1.0 / (hm + h0 + hp + hpp);
        ew[side][0] = h0 / (h0 + hp) + w1 * inv;
        ew[side][1] = -h0 * (hm + h0) / (2.0 * h0 + hp) * inv;
        ew[side][2] = hp * (hp + hpp) / (h0 + 2.0 * hp) * inv;
    }
    /* Lr = a_{c-1} + e1 (a_c - a_{c-1}) + e2 delta_c + e3 delta_{c-1}, likewise Rr */
    double Lr = av[1] + ew[0][0] * (av[2] - av[1]) + ew[0][1] * dl[1] + ew[0][2] * dl[0];
    double Rr = av[2] + ew[1][0] * (av[3] - av[2]) + ew[1][1] * dl[2] + ew[1][2] * dl[1];
    double a = av[2], L = Lr, R = Rr;
    int branch = 0;      /* 0 none, 1 flat, 2 L pulled in, 3 R pulled in */
    if ((R - a) * (a - L) <= 0.0) {
        L = a; R = a; branch = 1;
    } else {
        double dq = R - L, qa = a - 0.5 * (L + R);
        if (dq * qa > dq * dq / 6.0) { L = 3.0 * a - 2.0 * R; branch = 2; }
        else if (-dq * dq / 6.0 > dq * qa) { R = 3.0 * a - 2.0 * L; branch = 3; }
    }
    double q6 = 6.0 * a - 3.0 * (L + R);
    double th2 = th * th, th3 = th2 * th;
    double ell = h * (L * th + 0.5 * (R - L) * th2 + q6 * (0.5 * th2 - th3 / 3.0));
    *qval = L + th * (R - L) + q6 * th * (1.0 - th);
    /* d ell / d (a, L, R) with Q6 expanded */
    double ga = h * (3.0 * th2 - 2.0 * th3);
    double gl = h * (th - 2.0 * th2 + th3);
    double gr = h * (th3 - th2);
    double ba = 0.0, bl = 0.0, br = 0.0;    /* adjoints of a, Lr, Rr */
    switch (branch) {
    case 1: ba = ga + gl + gr; break;
    case 2: ba = ga + 3.0 * gl; br = -2.0 * gl + gr; break;
    case 3: ba = ga + 3.0 * gr; bl = gl - 2.0 * gr; break;
    default: ba = ga; bl = gl; br = gr; break;
    }
    double gb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    double bd[3] = {0.0, 0.0, 0.0};         /* adjoints of the three slopes */
    gb[2] += ba;
    gb[1] += bl * (1.0 - ew[0][0]);
    gb[2] += bl * ew[0][0];
    bd[1] += bl * ew[0][1];
    bd[0] += bl * ew[0][2];
    gb[2] += br * (1.0 - ew[1][0]);
    gb[3] += br * ew[1][0];
    bd[2] += br * ew[1][1];
    bd[1] += br * ew[1][2];
    for (int k = 0; k < 3; ++k)
        for (int t = 0; t < 3; ++t) gb[k + t] += bd[k] * dd[k][t];
    for (int k = 0; k < 5; ++k) g[k] = gb[k];
    return ell;
}

/* Transpose of the limited shift's Jacobian at q: qbar_in (overwritten) and
 * sbar = d <qbar_out, S(q; s)> / ds. */
static int shift_recon_adjoint_row(const double *x, const double *q,
                                   const double *qbar_out, double *qbar_in,
                                   int64_t n, double s, int recon, double *sbar)
{
    int lo = recon == RECON_PLM ? 1 : 2;
    int64_t *g = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    double *gw = (double *)malloc(sizeof(double) * 5 * (size_t)(n + 1));
    double *qv = (double *)malloc(sizeof(double) * (size_t)(n + 1));
    int64_t *cc = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!g || !gw || !qv || !cc) { free(g); free(gw); free(qv); free(cc); return -6; }
    for (int64_t e = 0; e < n; ++e) {
        double xh;
        int64_t k;
        shifted_node(x, n, s, e, &xh, &k);
        cc[e] = find_cell(x, n, xh);
        g[e] = cc[e] + k * n;
        lim_partial_grad(x, q, n, cc[e], xh, recon, gw + 5 * e, &qv[e]);
    }
    g[n] = g[0] + n;
    cc[n] = cc[0];
    qv[n] = qv[0];
    memcpy(gw + 5 * n, gw, 5 * sizeof(double));
    for (int64_t m = 0; m < n; ++m) qbar_in[m] = 0.0;
    double sb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        /* M'_i = sum_{m=g_i}^{g_{i+1}-1} Q_m dx_m + ell_{i+1} - ell_i, Q'_i = M'_i / dx_i */
        double mb = qbar_out[i] / (x[i + 1] - x[i]);
        for (int64_t m = g[i]; m < g[i + 1]; ++m) qbar_in[wrap(m, n)] += mb * dx_w(x, n, m);
        for (int a = 0; a <= 2 * lo; ++a) {
            qbar_in[wrap(cc[i + 1] - lo + a, n)] += mb * gw[5 * (i + 1) + a];
            qbar_in[wrap(cc[i] - lo + a, n)] -= mb * gw[5 * i + a];
        }
        /* d ell / d s = -q_c(xh) */
        sb -= mb * (qv[i + 1] - qv[i]);
    }
    if (sbar) *sbar = sb;
    free(g); free(gw); free(qv); free(cc);
    return 0;
}

/* fewest cells a row needs: the reconstruction stencil (3 or 5 cells) plus one */
static int64_t recon_min_cells(int recon) { return recon == RECON_PLM ? 4 : 6; }

/* ---------------------------------------------------------------------- */
/* adjoints (scatter form)                                                  */
/* ---------------------------------------------------------------------- */

/* Transpose of the bulk shift at fixed s, plus s-bar.  qbar_in is overwritten.
 * q is the forward input (only used for the v0 derivative). */
static int shift_adjoint_row(const double *x, const double *q,
                             const double *qbar_out, double *qbar_in, int64_t n,
                             double s, int p, double *sbar)
{
    int lo = (p - 1) / 2;
    double len = x[n] - x[0];
    edge_t *ed = (edge_t *)malloc(sizeof(edge_t) * (size_t)(n + 1));
    double *mbar = (double *)calloc((size_t)n, sizeof(double));
    double *vbar = (double *)calloc((size_t)(n + 1), sizeof(double));
    if (!ed || !mbar || !vbar) { free(ed); free(mbar); free(vbar); return -6; }
    for (int64_t e = 0; e < n; ++e) edge_eval(x, q, n, s, p, e, sbar != NULL, &ed[e]);
    ed[n] = ed[0];
    ed[n].k += 1;
    ed[n].g += n;
    /* M'_i = whole_i + ell_{i+1} - ell_i */
    for (int64_t i = 0; i < n; ++i) {
        double mb = qbar_out[i] / (x[i + 1] - x[i]);
        for (int64_t m = ed[i].g; m < ed[i + 1].g; ++m) mbar[wrap(m, n)] += mb;
        vbar[i + 1] += mb;
        vbar[i] -= mb;
    }
    /* node N shares node 0's partial integral */
    vbar[0] += vbar[n];
    double sb = 0.0;
    for (int64_t e = 0; e < n; ++e) {
        const edge_t *E = &ed[e];
        double X[ORACLE_MAX_ORDER + 1];
        for (int a = 0; a <= p; ++a) X[a] = node_x(x, n, len, E->c - lo + a);
        for (int a = 0; a <= p; ++a) {
            int64_t j = E->c - lo + a;
            double w = lagrange_w(X, p, a, E->xh) * vbar[e];
            /* D_a = C(j) - C(c) */
            if (j > E->c)
                for (int64_t m = E->c; m < j; ++m) mbar[wrap(m, n)] += w;
            else
                for (int64_t m = j; m < E->c; ++m) mbar[wrap(m, n)] -= w;
        }
        /* d ell / d s = -q~(xh) */
        sb -= vbar[e] * E->dell;
    }
    for (int64_t m = 0; m < n; ++m) qbar_in[m] = mbar[m] * (x[m + 1] - x[m]);
    if (sbar) *sbar = sb;
    free(ed); free(mbar); free(vbar);
    return 0;
}

/* Transpose of the Jacobian of the residual step at the forward state q.
 * qbar_in is overwritten; dvbar is accumulated into when non-NULL. */
static int residual_adjoint_row(const double *x, const double *q,
                                const double *dv, const double *qbar_out,
                                double *qbar_in, double *dvbar, int64_t n,
                                double dt)
{
    double *sbar = (double *)calloc((size_t)n, sizeof(double));
    if (!sbar) return -6;
    for (int64_t i = 0; i < n; ++i) qbar_in[i] = qbar_out[i];
    for (int64_t f = 0; f < n; ++f) {
        int64_t fm = wrap(f - 1, n);
        double v = dv[f];
        /* F_f enters Q''_f with +dt/dx_f and Q''_{f-1} with -dt/dx_{f-1} */
        double fbar = dt * (qbar_out[f] / (x[f + 1] - x[f])
                            - qbar_out[fm] / (x[fm + 1] - x[fm]));
        int64_t u = v >= 0.0 ? fm : f;
        double dxu = x[u + 1] - x[u];
        double sig = vl_slope(x, q, n, u);
        double qs = face_state(x, q, n, f, v, dt);
        if (dvbar) dvbar[f] += fbar * (qs - 0.5 * sig * v * dt);
        double qsbar = fbar * v;
        qbar_in[u] += qsbar;
        sbar[u] += qsbar * 0.5 * (v >= 0.0 ? (dxu - v * dt) : -(dxu + v * dt));
    }
    for (int64_t i = 0; i < n; ++i) {
        if (sbar[i] == 0.0) continue;
        double qm = q[wrap(i - 1, n)], q0 = q[i], qp = q[wrap(i + 1, n)];
        double hp = centre_gap(x, n, i), hm = centre_gap(x, n, i - 1);
        double a = (qp - q0) / hp, b = (q0 - qm) / hm;
        if (a * b <= 0.0) continue;
        double den = (a + b) * (a + b);
        double abar = sbar[i] * 2.0 * b * b / den;
        double bbar = sbar[i] * 2.0 * a * a / den;
        qbar_in[wrap(i + 1, n)] += abar / hp;
        qbar_in[i] -= abar / hp;
        qbar_in[i] += bbar / hm;
        qbar_in[wrap(i - 1, n)] -= bbar / hm;
    }
    free(sbar);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* batched entry points (rows are independent)                              */
/* ---------------------------------------------------------------------- */

static const double *row_mesh(const double *edges, int shared,
                              const int64_t *row_ptr, int64_t r)
{
    return shared ? edges : edges + row_ptr[r] + r;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int oracle_shift(int64_t n_rows, const int64_t *row_ptr, const double *edges,
                 int shared, const double *q, double *qout, const double *v0,
                 double dt, int order, int variant, int nthreads)
{
    if (order < 1 || order > ORACLE_MAX_ORDER || (order % 2) == 0) return -2;
    set_threads(nthreads);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t n = row_ptr[r + 1] - row_ptr[r];
        if (n < order + 1) { err |= 1; continue; }
        err |= shift_row(row_mesh(edges, shared, row_ptr, r), q + row_ptr[r],
                         qout + row_ptr[r], n, v0[r] * dt, order, variant) != 0;
    }
    return err ? -1 : 0;
}

int oracle_residual(int64_t n_rows, const int64_t *row_ptr, const double *edges,
                    int shared, const double *q, double *qout, const double *dv,
                    double dt, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t n = row_ptr[r + 1] - row_ptr[r];
        residual_row(row_mesh(edges, shared, row_ptr, r), q + row_ptr[r],
                     dv + row_ptr[r], qout + row_ptr[r], n, dt);
    }
    return 0;
}

/* n_steps of (shift, then residual when dv != NULL); q is updated in place. */
int oracle_step(int64_t n_rows, const int64_t *row_ptr, const double *edges,
                int shared, double *q, const double *v0, const double *dv,
                double dt, int order, int64_t n_steps, int nthreads)
{
    if (order < 1 || order > ORACLE_MAX_ORDER || (order % 2) == 0) return -2;
    set_threads(nthreads);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t n = row_ptr[r + 1] - row_ptr[r];
        const double *x = row_mesh(edges, shared, row_ptr, r);
        double *qr = q + row_ptr[r];
        double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
        if (!tmp || n < order + 1) { err |= 1; free(tmp); continue; }
        for (int64_t st = 0; st < n_steps; ++st) {
            shift_row(x, qr, tmp, n, v0[r] * dt, order, 0);
            if (dv) residual_row(x, tmp, dv + row_ptr[r], qr, n, dt);
            else memcpy(qr, tmp, sizeof(double) * (size_t)n);
        }
        free(tmp);
    }
    return err ? -1 : 0;
}

/* v0bar (per row) is accumulated with dt * s-bar when non-NULL. */
int oracle_shift_adjoint(int64_t n_rows, const int64_t *row_ptr,
                         const double *edges, int shared, const double *q,
                         const double *qbar_out, double *qbar_in,
                         const double *v0, double dt, int order, double *v0bar,
                         int nthreads)
{
    if (order < 1 || order > ORACLE_MAX_ORDER || (order % 2) == 0) return -2;
    set_threads(nthreads);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t n = row_ptr[r + 1] - row_ptr[r];
        double sb = 0.0;
        err |= shift_adjoint_row(row_mesh(edges, shared, row_ptr, r),
                                 q + row_ptr[r], qbar_out + row_ptr[r],
                                 qbar_in + row_ptr[r], n, v0[r] * dt, order,
                                 v0bar ? &sb : NULL) != 0;
        if (v0bar) v0bar[r] += dt * sb;
    }
    return err ? -1 : 0;
}

int oracle_residual_adjoint(int64_t n_rows, const int64_t *row_ptr,
                            const double *edges, int shared, const double *q,
                            const double *dv, const double *qbar_out,
                            double *qbar_in, double *dvbar, double dt,
                            int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t n = row_ptr[r + 1] - row_ptr[r];
        residual_adjoint_row(row_mesh(edges, shared, row_ptr, r), q + row_ptr[r],
                             dv + row_ptr[r], qbar_out + row_ptr[r],
                             qbar_in + row_ptr[r],
                             dvbar ? dvbar + row_ptr[r] : NULL, n, dt);
    }
    return 0;
}

/* Per-edge diagnostics of one row (tests): xh, k, c, ell for e = 0..N-1. */
int oracle_edges(const double *x, const double *q, int64_t n, double s,
                 int order, double *xh, int64_t *k, int64_t *c, double *ell,
                 double *dell)
{
    for (int64_t e = 0; e < n; ++e) {
        edge_t E;
        edge_eval(x, q, n, s, order, e, 1, &E);
        xh[e] = E.xh; k[e] = E.k; c[e] = E.c; ell[e] = E.ell; dell[e] = E.dell;
    }
    return 0;
}

/* Bulk shift with a limited reconstruction (recon 1 PLM, 2 PPM). */
int oracle_shift_recon(int64_t n_rows, const int64_t *row_ptr, const double *edges,
                       int shared, const double *q, double *qout, const double *v0,
                       double dt, int recon, int nthreads)
{
    if (recon != RECON_PLM && recon != RECON_PPM) return -2;
    set_threads(nthreads);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t n = row_ptr[r + 1] - row_ptr[r];
        if (n < recon_min_cells(recon)) { err |= 1; continue; }
        err |= shift_row_recon(row_mesh(edges, shared, row_ptr, r), q + row_ptr[r],
                               qout + row_ptr[r], n, v0[r] * dt, recon) != 0;
    }
    return err ? -1 : 0;
}

/* n_steps of (limited shift, then residual when dv != NULL), q in place. */
int oracle_step_recon(int64_t n_rows, const int64_t *row_ptr, const double *edges,
                      int shared, double *q, const double *v0, const double *dv,
                      double dt, int recon, int64_t n_steps, int nthreads)
{
    if (recon != RECON_PLM && recon != RECON_PPM) return -2;
    set_threads(nthreads);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t n = row_ptr[r + 1] - row_ptr[r];
        const double *x = row_mesh(edges, shared, row_ptr, r);
        double *qr = q + row_ptr[r];
        double *tmp = (double *)malloc(sizeof(double) * (size_t)n);
        if (!tmp || n < recon_min_cells(recon)) { err |= 1; free(tmp); continue; }
        for (int64_t st = 0; st < n_steps; ++st) {
            shift_row_recon(x, qr, tmp, n, v0[r] * dt, recon);
            if (dv) residual_row(x, tmp, dv + row_ptr[r], qr, n, dt);
            else memcpy(qr, tmp, sizeof(double) * (size_t)n);
        }
        free(tmp);
    }
    return err ? -1 : 0;
}

/* Per-cell reconstruction of one row (tests): PLM (Q, sigma, 0), PPM
 * (QL, QR, Q6); flags as for ppm_parabola. */
int oracle_recon_cells(const double *x, const double *q, int64_t n, int recon,
                       int flags, double *c0, double *c1, double *c2)
{
    if (recon != RECON_PLM && recon != RECON_PPM) return -2;
    for (int64_t c = 0; c < n; ++c) {
        if (recon == RECON_PLM) {
            c0[c] = q[c];
            c1[c] = vl_slope(x, q, n, c);
            c2[c] = 0.0;
        } else {
            ppm_parabola(x, q, n, c, flags, &c0[c], &c1[c], &c2[c]);
        }
    }
    return 0;
}

/* Limited-reconstruction partial integrals of one row's shifted nodes (tests). */
int oracle_edges_recon(const double *x, const double *q, int64_t n, double s,
                       int recon, int64_t *g, double *ell)
{
    if (recon != RECON_PLM && recon != RECON_PPM) return -2;
    for (int64_t e = 0; e < n; ++e) {
        double xh;
        int64_t k;
        shifted_node(x, n, s, e, &xh, &k);
        int64_t c = find_cell(x, n, xh);
        g[e] = c + k * n;
        ell[e] = limited_partial(x, q, n, c, xh, recon);
    }
    return 0;
}

/* Adjoint of the limited shift at the forward state q: qbar_in overwritten;
 * v0bar (per row, when non-NULL) accumulated with dt * d<qbar_out, S q>/ds. */
int oracle_shift_recon_adjoint(int64_t n_rows, const int64_t *row_ptr,
                               const double *edges, int shared, const double *q,
                               const double *qbar_out, double *qbar_in,
                               const double *v0, double dt, int recon, double *v0bar,
                               int nthreads)
{
    if (recon != RECON_PLM && recon != RECON_PPM) return -2;
    set_threads(nthreads);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t n = row_ptr[r + 1] - row_ptr[r];
        if (n < recon_min_cells(recon)) { err |= 1; continue; }
        double sb = 0.0;
        err |= shift_recon_adjoint_row(row_mesh(edges, shared, row_ptr, r), q + row_ptr[r],
                                       qbar_out + row_ptr[r], qbar_in + row_ptr[r], n,
                                       v0[r] * dt, recon, v0bar ? &sb : NULL) != 0;
        if (v0bar) v0bar[r] += dt * sb;
    }
    return err ? -1 : 0;
}

/* Radial transport step of a polar grid: q and out [n_rows][n_cols], u
 * [n_rows+1][n_cols] (face j of a column between rows j-1 and j), radial edges
 * re[n_rows+1]. */
int oracle_radial(int64_t n_rows, int64_t n_cols, const double *re, const double *q,
                  const double *u, double dt, double *out, int nthreads)
{
    if (n_rows < 1 || n_cols < 1) return -1;
    set_threads(nthreads);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : err)
    for (int64_t i = 0; i < n_cols; ++i) {
        double *col = (double *)malloc(sizeof(double) * (size_t)(3 * n_rows + 1));
        if (!col) { err |= 1; continue; }
        double *uc = col + n_rows, *oc = uc + n_rows + 1;
        for (int64_t j = 0; j < n_rows; ++j) col[j] = q[j * n_cols + i];
        for (int64_t j = 0; j <= n_rows; ++j) uc[j] = u[j * n_cols + i];
        radial_column(re, n_rows, col, uc, dt, oc);
        for (int64_t j = 0; j < n_rows; ++j) out[j * n_cols + i] = oc[j];
        free(col);
    }
    return err ? -6 : 0;
}

/* Centre values -> cell averages (inverse = 0) or back (inverse = 1), every
 * row; q and out must not alias. */
int oracle_average4(int64_t n_rows, const int64_t *row_ptr, const double *edges, int shared,
                    const double *q, double *out, int inverse, int nthreads)
{
    set_threads(nthreads);
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t r = 0; r < n_rows; ++r) {
        int64_t n = row_ptr[r + 1] - row_ptr[r];
        if (n < 1) { err |= 1; continue; }
        average4_row(row_mesh(edges, shared, row_ptr, r), q + row_ptr[r], out + row_ptr[r], n,
                     inverse);
    }
    return err ? -1 : 0;
}
