// ram_adjoint.hip -- adjoint kernels of the RAM step for gfx950.
//
// The bulk shift is linear in Q: with V_e the interpolated cumulative at the
// shifted node e and M'_i = V_{i+1} - V_i, its transpose is, per source cell m,
//     Mbar_m = sum_e Vbar_e H_e(m),   Vbar_e = Mbar'_{e-1} - Mbar'_e,
// where H_e(m) is the weight of M_m in V_e: 1 below the interpolation stencil,
// a suffix sum of the Lagrange weights inside it, 0 above it.  Per destination
// tile the sum telescopes to one Mbar' value plus the few stencils that
// straddle m, so each source cell of the tile's window is a short gather.
// Window cells shared with the neighbouring tiles (the P cells of the stencil
// of each tile-boundary node) go to a per-tile side buffer, and a second
// kernel sums each of them over the tiles whose windows hold it, in a fixed
// order (usually two; more where a row's last tile is shorter than P cells
// and its window overlaps itself); every other cell is written once, so the
// result is the same in every run.  v0bar takes one term per tile, summed per
// row in a fixed order by another kernel.
//
// The derivative with respect to v0 enters through x~ = x - v0 dt:
//     dM'_i/ds = -(q~(x~_{i+1}) - q~(x~_i)),
// with q~ the reconstruction (derivative of the interpolated cumulative).
//
// The residual adjoint is a gather over the two-cell halo: face fluxes,
// upwind face states and van Leer slopes are transposed cell by cell; the
// limiter's derivative is taken as zero where the one-sided slopes do not
// have the same sign, and dv = 0 uses the dv >= 0 branch.
#include "ram_device.h"

namespace ram {
namespace {

using namespace dev;

// Derivatives of the Lagrange basis at xh.
template <int P>
__device__ inline void lagrange_dweights(double xh, const double *X, double *dw)
{
    double t[P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) t[a] = xh - X[a];
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        double den = 1.0;
#pragma unroll
        for (int b = 0; b <= P; ++b)
            if (b != a) den *= X[a] - X[b];
        double sum = 0.0;
#pragma unroll
        for (int b = 0; b <= P; ++b) {
            if (b == a) continue;
            double prod = 1.0;
#pragma unroll
            for (int c = 0; c <= P; ++c)
                if (c != a && c != b) prod *= t[c];
            sum += prod;
        }
        dw[a] = sum / den;
    }
}

template <typename TQ>
__device__ inline double mass_at(const double *x, const TQ *q, int n, int64_t m)
{
    const int w = wrapi(m, n);
    return (double)q[w] * (x[w + 1] - x[w]);
}

// Shifted node e of a row (node N = node 0 of the next period): g = c + k N.
__device__ inline int64_t locate(const double *x, int n, double s, int e,
                                 double &xh, const Rows &R)
{
    int64_t k;
    if (e == n) {
        shifted_node(x, n, s, 0, xh, k);
        k += 1;
    } else {
        shifted_node(x, n, s, e, xh, k);
    }
    // a shared mesh's bucket index (one lookup and a short walk) or a binary
    // search of the row; the same exact cell either way
    const int c = R.has_tab ? find_cell_tab(x, n, R.tab, R.tab.scal[0], xh)
                            : find_cell(x, n, xh);
    return (int64_t)c + k * (int64_t)n;
}

// Window cell j (of W; row cell mm) of a tile: a cell only this tile's window
// holds goes to the state, the window's first P and last P cells to the
// tile's side buffer (head, tail; overlap-free when W < 2P).
template <typename TQ, int P>
__device__ inline void put_window_cell(TQ *qbi, TQ *edge, int mm, int j, int W, TQ v)
{
    if (j >= P && j < W - P) qbi[mm] = v;
    else if (j < P) edge[j] = v;
    else edge[P + j - max(P, W - P)] = v;
}

template <typename TQ, int P>
__global__ __launch_bounds__(kBlock) void k_shift_adj(ShiftAdjArgs a)
{
    constexpr int LO = (P - 1) / 2;
    __shared__ int64_t sg[kTile + 1];
    __shared__ double svb[kTile + 1];     // tile-local Vbar of each node
    __shared__ double shs[kTile + 1][P];  // suffix sums of the weights
    __shared__ double sred[kBlock / 64];

    Tile ti;
    if (!get_tile(a.rows, blockIdx.x, ti)) return;
    const int n = ti.n;
    if (n < P + 1) return;
    const double *x = ti.x;
    const TQ *qbo = (const TQ *)a.qbar_out + ti.qoff;
    TQ *qbi = (TQ *)a.qbar_in + ti.qoff;
    const TQ *qf = a.q_fwd ? (const TQ *)a.q_fwd + ti.qoff : nullptr;
    const double s = a.v0[ti.row] * a.dt;
    const double len = x[n] - x[0];
    const int i0 = ti.i0;
    const int nd = min(a.rows.tile, n - i0);
    const int ne = nd + 1;
    const bool want_v0 = a.v0bar != nullptr && qf != nullptr;

    double vpart = 0.0;
    for (int t = threadIdx.x; t < ne; t += kBlock) {
        double xh;
        const int64_t g = locate(x, n, s, i0 + t, xh, a.rows);
        const int c = wrapi(g, n);
        double X[P + 1], w[P + 1];
#pragma unroll
        for (int b = 0; b <= P; ++b) X[b] = node_x(x, n, len, c - LO + b);
        lagrange_weights<P>(xh, X, w);
        double acc = 0.0;
#pragma unroll
        for (int b = P; b >= 1; --b) {
            acc += w[b];
            shs[t][b - 1] = acc;
        }
        double vb = 0.0;
        if (t >= 1) {
            const int i = i0 + t - 1;
            vb += (double)qbo[i] / (x[i + 1] - x[i]);
        }
        if (t <= nd - 1) {
            const int i = i0 + t;
            vb -= (double)qbo[i] / (x[i + 1] - x[i]);
        }
        svb[t] = vb;
        sg[t] = g;
        if (want_v0) {
            double dw[P + 1];
            lagrange_dweights<P>(xh, X, dw);
            double dq = 0.0;
#pragma unroll
            for (int b = 0; b <= P; ++b) {
                const int j = c - LO + b;
                double d = 0.0;
                if (j > c) {
                    for (int m = c; m < j; ++m) d += mass_at(x, qf, n, m);
                } else if (j < c) {
                    for (int m = j; m < c; ++m) d += mass_at(x, qf, n, m);
                    d = -d;
                }
                dq += dw[b] * d;
            }
            vpart -= vb * dq;
        }
    }
    if (want_v0) {
        for (int d = 32; d >= 1; d >>= 1) vpart += __shfl_xor(vpart, d);
        if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = vpart;
    }
    __syncthreads();
    if (want_v0 && threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) tot += sred[w];
        a.v0part[blockIdx.x] = a.dt * tot;
    }

    const int64_t wlo = sg[0] - LO;
    const int W = (int)(sg[nd] - sg[0] + P);
    const int base = wrapi(wlo, n);
    TQ *edge = (TQ *)a.edge + (int64_t)blockIdx.x * (2 * P);
    if (threadIdx.x == 0) a.wstart[blockIdx.x] = wlo;
    for (int j = threadIdx.x; j < W; j += kBlock) {
        const int64_t target = wlo + j + LO;
        // first tile node whose stencil lies wholly above cell j
        int lo = 0, hi = ne;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sg[mid] > target) hi = mid; else lo = mid + 1;
        }
        double S = (lo >= 1 && lo <= nd)
                       ? (double)qbo[i0 + lo - 1] / (x[i0 + lo] - x[i0 + lo - 1])
                       : 0.0;
        for (int t = lo - 1; t >= 0 && sg[t] > target - P; --t) {
            const int b = (int)min((int64_t)(P - 1), max((int64_t)0, target - sg[t]));
            S += svb[t] * shs[t][b];
        }
        const int mm = (base + j) % n;
        const double val = S * (x[mm + 1] - x[mm]);
        put_window_cell<TQ, P>(qbi, edge, mm, j, W, (TQ)val);
    }
}

// ---------------------------------------------------------------------------
// adjoint of the limited (PLM / PPM) shift
// ---------------------------------------------------------------------------
//
// The limited shift is nonlinear in Q; its adjoint is the transpose of the
// Jacobian at the forward state, each limiter differentiated on the branch it
// takes there (a zero slope where the one-sided differences do not share a
// sign).  Node e's partial integral ell_e depends on the averages of its
// source cell's stencil c-lo .. c+lo, so the transpose gathers, for every
// source cell m of a tile's window,
//     Qbar_m = dx_m Mbar'_i  (m a whole cell of destination cell i)
//            + sum_{e : |c_e - m| <= lo} Vbar_e d ell_e / d Q_m,
// with Vbar_e = Mbar'_{e-1} - Mbar'_e.  Shared window cells are accumulated
// with atomics after the zeroing pass, as for the Lagrange shift.

// d ell / d Q_{c-lo+a} (a = 0 .. 2 lo) of the partial integral of cell c at
// xh, and the reconstruction's value q_c(xh) (= d ell / d xh); FP64.  A shared
// mesh passes its tables (reciprocal centre gaps, PPM weights); per-row meshes
// pass null and the mesh terms are formed from the nodes.
template <typename TQ, int R>
__device__ inline void lim_grad(const double *x, const TQ *q, int n, double len, int c,
                                double xh, const double *hinv, const double *pw, double *gw,
                                double &qval)
{
    const double h = x[c + 1] - x[c];
    const double th = (xh - x[c]) / h;
    if constexpr (R == kReconPLM) {
        const double qm = (double)q[wrapi(c - 1, n)], q0 = (double)q[c];
        const double qp = (double)q[wrapi(c + 1, n)];
        // reciprocal centre gaps (c, c+1) and (c-1, c)
        const double gp = hinv ? hinv[c] : 1.0 / centre_gap(x, n, len, c);
        const double gm = hinv ? hinv[wrapi(c - 1, n)] : 1.0 / centre_gap(x, n, len, c - 1);
        const double a = (qp - q0) * gp, b = (q0 - qm) * gm;
        double sig = 0.0, dsa = 0.0, dsb = 0.0;
        if (a * b > 0.0) {
            const double s2 = (a + b) * (a + b);
            sig = 2.0 * a * b / (a + b);
            dsa = 2.0 * b * b / s2;
            dsb = 2.0 * a * a / s2;
        }
        // ell = Q_c h theta + sigma h^2 (theta^2 - theta) / 2
        const double ks = 0.5 * h * h * (th * th - th);
        gw[0] = -ks * dsb * gm;
        gw[1] = h * th + ks * (dsb * gm - dsa * gp);
        gw[2] = ks * dsa * gp;
        qval = q0 + sig * (xh - 0.5 * (x[c] + x[c + 1]));
    } else {
        double av[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) av[k] = (double)q[wrapi(c - 2 + k, n)];
        // mesh weights of cells c-1, c, c+1: their slopes' (d1, d2), and the
        // interface weights (e1, e2, e3) of cells c-1 and c
        PpmW w[3];
        if (pw) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int m = wrapi(c - 1 + k, n);
                w[k] = {pw[m], pw[n + m], pw[2 * n + m], pw[3 * n + m], pw[4 * n + m]};
            }
        } else {
            double hv[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const int m = wrapi(c - 2 + k, n);
                hv[k] = x[m + 1] - x[m];
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) w[k] = ppm_weights(hv[k], hv[k + 1], hv[k + 2], hv[k + 3]);
        }
        // limited slopes of cells c-1, c, c+1 and their derivatives w.r.t.
        // the averages of each slope's cells j-1, j, j+1
        double dl[3], dd[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double up = av[k + 2] - av[k + 1], dn = av[k + 1] - av[k];
            const double d = w[k].d1 * up + w[k].d2 * dn;
            dd[k][0] = dd[k][1] = dd[k][2] = 0.0;
            dl[k] = 0.0;
            if (up * dn > 0.0) {
                dl[k] = copysign(fmin(fabs(d), 2.0 * fmin(fabs(up), fabs(dn))), d);
                if (fabs(d) <= 2.0 * fabs(up) && fabs(d) <= 2.0 * fabs(dn)) {
                    dd[k][0] = -w[k].d2;
                    dd[k][1] = w[k].d2 - w[k].d1;
                    dd[k][2] = w[k].d1;
                } else if (fabs(up) <= fabs(dn)) {
                    dd[k][1] = -2.0;          // twice the upper difference
                    dd[k][2] = 2.0;
                } else {
                    dd[k][0] = -2.0;          // twice the lower difference
                    dd[k][1] = 2.0;
                }
            }
        }
        // interface values c-1/2 and c+1/2 before the constraints
        const PpmW &wl = w[0], &wr = w[1];
        const double Lr = av[1] + wl.e1 * (av[2] - av[1]) + wl.e2 * dl[1] + wl.e3 * dl[0];
        const double Rr = av[2] + wr.e1 * (av[3] - av[2]) + wr.e2 * dl[2] + wr.e3 * dl[1];
        const double a = av[2];
        double L = Lr, Rv = Rr;
        int branch = 0;                       // 1 flat, 2 L pulled in, 3 R pulled in
        if ((Rv - a) * (a - L) <= 0.0) {
            L = a;
            Rv = a;
            branch = 1;
        } else {
            const double dq = Rv - L, qa = a - 0.5 * (L + Rv);
            if (dq * qa > dq * dq / 6.0) { L = 3.0 * a - 2.0 * Rv; branch = 2; }
            else if (-dq * dq / 6.0 > dq * qa) { Rv = 3.0 * a - 2.0 * L; branch = 3; }
        }
        const double q6 = 6.0 * a - 3.0 * (L + Rv);
        qval = L + th * (Rv - L) + q6 * th * (1.0 - th);
        // d ell / d (a, L, R) with Q6 expanded, then back through the branch
        const double th2 = th * th, th3 = th2 * th;
        const double ga = h * (3.0 * th2 - 2.0 * th3);
        const double gl = h * (th - 2.0 * th2 + th3);
        const double gr = h * (th3 - th2);
        double ba = ga, bl = gl, br = gr;
        if (branch == 1) { ba = ga + gl + gr; bl = 0.0; br = 0.0; }
        else if (branch == 2) { ba = ga + 3.0 * gl; bl = 0.0; br = gr - 2.0 * gl; }
        else if (branch == 3) { ba = ga + 3.0 * gr; bl = gl - 2.0 * gr; br = 0.0; }
        double gb[5] = {0.0, 0.0, ba, 0.0, 0.0};
        double bd[3] = {bl * wl.e3, bl * wl.e2 + br * wr.e3, br * wr.e2};
        gb[1] += bl * (1.0 - wl.e1);
        gb[2] += bl * wl.e1 + br * (1.0 - wr.e1);
        gb[3] += br * wr.e1;
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int t = 0; t < 3; ++t) gb[k + t] += bd[k] * dd[k][t];
#pragma unroll
        for (int k = 0; k < 5; ++k) gw[k] = gb[k];
    }
}

template <typename TQ, int R>
__global__ __launch_bounds__(kBlock) void k_shift_lim_adj(ShiftAdjArgs a)
{
    constexpr int LO = LimHalo<R>::lo;
    constexpr int P = 2 * LO + 1;         // stencil cells
    __shared__ int64_t sg[kTile + 1];     // extended source cell of each node
    __shared__ double svb[kTile + 1];     // tile-local Vbar of each node
    __shared__ double sgw[kTile + 1][P];  // d ell / d Q of its stencil cells
    __shared__ double sred[kBlock / 64];

    Tile ti;
    if (!get_tile(a.rows, blockIdx.x, ti)) return;
    const int n = ti.n;
    if (n < P + 1) return;
    const double *x = ti.x;
    const TQ *qbo = (const TQ *)a.qbar_out + ti.qoff;
    TQ *qbi = (TQ *)a.qbar_in + ti.qoff;
    const TQ *qf = (const TQ *)a.q_fwd + ti.qoff;
    const double s = a.v0[ti.row] * a.dt;
    const double len = x[n] - x[0];
    const int i0 = ti.i0;
    const int nd = min(a.rows.tile, n - i0);
    const int ne = nd + 1;
    const bool want_v0 = a.v0bar != nullptr;
    const double *hinv = a.rows.has_tab ? a.rows.tab.hinv : nullptr;
    const double *pw = a.rows.has_tab ? a.rows.tab.ppmd : nullptr;

    double vpart = 0.0;
    for (int t = threadIdx.x; t < ne; t += kBlock) {
        double xh;
        const int64_t g = locate(x, n, s, i0 + t, xh, a.rows);
        const int c = wrapi(g, n);
        double gw[P], qv;
        lim_grad<TQ, R>(x, qf, n, len, c, xh, hinv, pw, gw, qv);
        double vb = 0.0;
        if (t >= 1) {
            const int i = i0 + t - 1;
            vb += (double)qbo[i] / (x[i + 1] - x[i]);
        }
        if (t <= nd - 1) {
            const int i = i0 + t;
            vb -= (double)qbo[i] / (x[i + 1] - x[i]);
        }
        svb[t] = vb;
        sg[t] = g;
#pragma unroll
        for (int b = 0; b < P; ++b) sgw[t][b] = gw[b];
        vpart -= vb * qv;                 // d ell / d s = -q_c(xh)
    }
    if (want_v0) {
        for (int d = 32; d >= 1; d >>= 1) vpart += __shfl_xor(vpart, d);
        if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = vpart;
    }
    __syncthreads();
    if (want_v0 && threadIdx.x == 0) {
        double tot = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) tot += sred[w];
        a.v0part[blockIdx.x] = a.dt * tot;
    }

    const int64_t wlo = sg[0] - LO;
    const int W = (int)(sg[nd] - sg[0] + P);
    const int base = wrapi(wlo, n);
    TQ *edge = (TQ *)a.edge + (int64_t)blockIdx.x * (2 * P);
    if (threadIdx.x == 0) a.wstart[blockIdx.x] = wlo;
    for (int j = threadIdx.x; j < W; j += kBlock) {
        const int64_t m = wlo + j;
        const int mm = (base + j) % n;
        const double dxm = x[mm + 1] - x[mm];
        // the destination cell whose whole-cell run holds m: the last node at
        // or below m starts it
        int lo = 0, hi = ne;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sg[mid] > m) hi = mid; else lo = mid + 1;
        }
        double val = (lo >= 1 && lo <= nd)
                         ? (double)qbo[i0 + lo - 1] / (x[i0 + lo] - x[i0 + lo - 1]) * dxm
                         : 0.0;
        // nodes whose stencil holds m: source cell within lo of m
        lo = 0;
        hi = ne;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sg[mid] < m - LO) lo = mid + 1; else hi = mid;
        }
        for (int t = lo; t < ne && sg[t] <= m + LO; ++t)
            val += svb[t] * sgw[t][(int)(m - (sg[t] - LO))];
        put_window_cell<TQ, P>(qbi, edge, mm, j, W, (TQ)val);
    }
}

template <typename TQ>
__global__ __launch_bounds__(kBlock) void k_residual_adj(ResidualAdjArgs a)
{
    __shared__ double sq[kTile + 4];    // forward state, cells i0-2 .. i0+nd+1
    __shared__ double sb[kTile + 4];    // qbar_out, same cells
    __shared__ double sda[kTile + 2];   // dsigma/da / h+, cells i0-1 .. i0+nd
    __shared__ double sdb[kTile + 2];   // dsigma/db / h-
    __shared__ double sqsb[kTile + 3];  // face-state adjoint, faces i0-1 .. i0+nd+1
    __shared__ double ssc[kTile + 3];   // slope adjoint each face sends upwind
    __shared__ float sup[kTile + 3];    // 1 if the face's upwind cell is its left

    Tile ti;
    if (!get_tile(a.rows, blockIdx.x, ti)) return;
    const int n = ti.n;
    const double *x = ti.x;
    const TQ *q = (const TQ *)a.q_fwd + ti.qoff;
    const TQ *dv = (const TQ *)a.dv + ti.qoff;
    const TQ *qbo = (const TQ *)a.qbar_out + ti.qoff;
    TQ *qbi = (TQ *)a.qbar_in + ti.qoff;
    TQ *dvb = a.dvbar ? (TQ *)a.dvbar + ti.qoff : nullptr;
    const double dt = a.dt;
    const double len = x[n] - x[0];
    const int i0 = ti.i0;
    const int nd = min(a.rows.tile, n - i0);

    for (int t = threadIdx.x; t < nd + 4; t += kBlock) {
        const int c = wrapi((int64_t)i0 - 2 + t, n);
        sq[t] = (double)q[c];
        sb[t] = (double)qbo[c];
    }
    __syncthreads();
    // slopes' partial derivatives, cells i0-1+t
    for (int t = threadIdx.x; t < nd + 2; t += kBlock) {
        const int64_t i = (int64_t)i0 - 1 + t;
        const double hp = centre_gap(x, n, len, i);
        const double hm = centre_gap(x, n, len, i - 1);
        const double ap = (sq[t + 2] - sq[t + 1]) / hp;
        const double bm = (sq[t + 1] - sq[t]) / hm;
        double da = 0.0, db = 0.0;
        if (ap * bm > 0.0) {
            const double den = (ap + bm) * (ap + bm);
            da = 2.0 * bm * bm / den / hp;
            db = 2.0 * ap * ap / den / hm;
        }
        sda[t] = da;
        sdb[t] = db;
    }
    // faces i0-1+t: flux adjoint, face-state adjoint, slope adjoint sent upwind
    for (int t = threadIdx.x; t < nd + 3; t += kBlock) {
        const int64_t f = (int64_t)i0 - 1 + t;
        const int fw = wrapi(f, n), fm = wrapi(f - 1, n);
        const double v = (double)dv[fw];
        // cells f and f-1 are sq/sb index t+1 and t
        const double fbar = dt * (sb[t + 1] / (x[fw + 1] - x[fw]) -
                                  sb[t] / (x[fm + 1] - x[fm]));
        const double qsb = fbar * v;
        const int u = v >= 0.0 ? fm : fw;
        const double dxu = x[u + 1] - x[u];
        sqsb[t] = qsb;
        ssc[t] = qsb * 0.5 * (v >= 0.0 ? (dxu - v * dt) : -(dxu + v * dt));
        sup[t] = v >= 0.0 ? 1.0f : 0.0f;
        if (dvb && t >= 1 && t <= nd) {
            // owned face i0+t-1; its upwind cell's slope from the forward state
            const int su = v >= 0.0 ? t : t + 1;   // sq index of the upwind cell
            const int64_t ui = (int64_t)i0 - 2 + su;
            const double hp = centre_gap(x, n, len, ui);
            const double hm = centre_gap(x, n, len, ui - 1);
            const double dp = (sq[su + 1] - sq[su]) / hp;
            const double dm = (sq[su] - sq[su - 1]) / hm;
            const double sig = (dp * dm <= 0.0) ? 0.0 : 2.0 * dp * dm / (dp + dm);
            const double qs = v >= 0.0 ? sq[su] + 0.5 * sig * (dxu - v * dt)
                                       : sq[su] - 0.5 * sig * (dxu + v * dt);
            dvb[fw] = (TQ)((double)dvb[fw] + fbar * (qs - 0.5 * sig * v * dt));
        }
    }
    __syncthreads();
    // cells: identity + face states + slopes of cells i-1, i, i+1
    for (int t = threadIdx.x; t < nd; t += kBlock) {
        // slope adjoint of cell i0-1+k gathered from its two faces (k, k+1)
        auto sigbar = [&](int k) {
            return (sup[k] == 0.0f ? ssc[k] : 0.0) + (sup[k + 1] != 0.0f ? ssc[k + 1] : 0.0);
        };
        const double sbm = sigbar(t), sb0 = sigbar(t + 1), sbp = sigbar(t + 2);
        double g = sb[t + 2];
        if (sup[t + 1] == 0.0f) g += sqsb[t + 1];   // face i, upwind = i
        if (sup[t + 2] != 0.0f) g += sqsb[t + 2];   // face i+1, upwind = i
        g += sbm * sda[t] + sb0 * (sdb[t + 1] - sda[t + 1]) - sbp * sdb[t + 2];
        qbi[i0 + t] = (TQ)g;
    }
}

template <typename TQ, int P>
hipError_t shift_adj_order(const ShiftAdjArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((k_shift_adj<TQ, P>), dim3((unsigned)a.rows.n_tiles),
                       dim3(kBlock), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_edge_sum(a.rows, a.wstart, a.edge, a.qbar_in, sizeof(TQ) == 8, P, st);
}

template <typename TQ>
hipError_t shift_adj_dispatch(const ShiftAdjArgs &a, int order, hipStream_t st)
{
    switch (order) {
    case 1: return shift_adj_order<TQ, 1>(a, st);
    case 3: return shift_adj_order<TQ, 3>(a, st);
    default: return shift_adj_order<TQ, 5>(a, st);
    }
}

} // namespace

hipError_t launch_shift_limited_adjoint(const ShiftAdjArgs &a, bool f64, int recon,
                                        hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    const dim3 g((unsigned)a.rows.n_tiles), b(kBlock);
    if (f64) {
        if (recon == kReconPLM)
            hipLaunchKernelGGL((k_shift_lim_adj<double, kReconPLM>), g, b, 0, stream, a);
        else
            hipLaunchKernelGGL((k_shift_lim_adj<double, kReconPPM>), g, b, 0, stream, a);
    } else {
        if (recon == kReconPLM)
            hipLaunchKernelGGL((k_shift_lim_adj<float, kReconPLM>), g, b, 0, stream, a);
        else
            hipLaunchKernelGGL((k_shift_lim_adj<float, kReconPPM>), g, b, 0, stream, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_edge_sum(a.rows, a.wstart, a.edge, a.qbar_in, f64, recon == kReconPLM ? 3 : 5,
                        stream);
    if (e != hipSuccess || !(a.v0bar && a.q_fwd)) return e;
    return launch_v0_reduce(a.rows, a.v0part, a.v0bar, stream);
}

hipError_t launch_shift_adjoint(const ShiftAdjArgs &a, bool f64, int order,
                                hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    hipError_t e = f64 ? shift_adj_dispatch<double>(a, order, stream)
                       : shift_adj_dispatch<float>(a, order, stream);
    if (e != hipSuccess || !(a.v0bar && a.q_fwd)) return e;
    return launch_v0_reduce(a.rows, a.v0part, a.v0bar, stream);
}

namespace {

// Boundary T of a row (one thread): the cells from its window start up to p
// cells on or the next tile's start, each the sum, tile T first and then
// down, of the terms the tiles whose windows hold it stored (tile k's window
// runs from wstart[k] to the next tile's start plus p; across the row's ends
// the row's tiles one period away).
template <typename TQ, int P>
__global__ __launch_bounds__(256) void k_edge_sum(Rows R, const int64_t *wstart, const TQ *edge,
                                                  TQ *qbar)
{
    const int64_t tile = (int64_t)blockIdx.x * 256 + threadIdx.x;
    Tile ti;
    if (tile >= R.n_tiles || !get_tile(R, tile, ti)) return;
    const int n = ti.n;
    if (n < P + 1) return;                  // the adjoint kernels skip such rows
    int64_t t0;
    int tpr;
    if (R.n_cols > 0) {
        tpr = (int)((n + R.tile - 1) / R.tile);
        t0 = ti.row * tpr;
    } else {
        t0 = R.tile_ptr[ti.row];
        tpr = (int)(R.tile_ptr[ti.row + 1] - t0);
    }
    const int k0 = (int)(tile - t0);
    auto start = [&](int k, int64_t &id) {
        const int q = k >= 0 ? k / tpr : -((-k + tpr - 1) / tpr);
        id = t0 + (k - q * tpr);
        return wstart[id] + (int64_t)q * n;
    };
    int64_t idp, id0, idn;
    const int64_t ap = start(k0 - 1, idp), a0 = start(k0, id0), a1 = start(k0 + 1, idn);
    TQ *q = qbar + ti.qoff;
    if (a1 - a0 >= P && a0 - ap >= P) {
        // two terms a cell: this tile's head and the previous tile's tail
        const TQ *e0 = edge + id0 * (2 * P), *ep = edge + idp * (2 * P);
        for (int k = 0; k < P; ++k) q[wrapi(a0 + k, n)] = ((TQ)0 + e0[k]) + ep[P + k];
        return;
    }
    const int64_t mend = min(a0 + P, a1);
    for (int64_t m = a0; m < mend; ++m) {
        TQ sum = (TQ)0;
        int64_t at = a0, an = a1, id = id0;
        for (int k = k0; k > k0 - tpr - 1; --k) {
            if (k != k0) {
                an = at;
                at = start(k, id);
            }
            const int64_t W = an - at + P;
            if (at + W <= m) break;
            const int pos = (int)(m - at);
            const TQ *e = edge + id * (2 * P);
            sum += pos < P ? e[pos] : e[P + pos - (int)max((int64_t)P, W - P)];
        }
        q[wrapi(m, n)] = sum;
    }
}

template <typename TQ>
hipError_t edge_sum_t(const Rows &R, const int64_t *wstart, const void *edge, void *qbar, int p,
                      hipStream_t st)
{
    const dim3 g((unsigned)((R.n_tiles + 255) / 256)), b(256);
    const TQ *e = (const TQ *)edge;
    TQ *q = (TQ *)qbar;
    switch (p) {
    case 1: hipLaunchKernelGGL((k_edge_sum<TQ, 1>), g, b, 0, st, R, wstart, e, q); break;
    case 3: hipLaunchKernelGGL((k_edge_sum<TQ, 3>), g, b, 0, st, R, wstart, e, q); break;
    default: hipLaunchKernelGGL((k_edge_sum<TQ, 5>), g, b, 0, st, R, wstart, e, q); break;
    }
    return hipGetLastError();
}

} // namespace

hipError_t launch_edge_sum(const Rows &R, const int64_t *wstart, const void *edge, void *qbar,
                           bool f64, int p, hipStream_t stream)
{
    if (R.n_tiles <= 0) return hipSuccess;
    if (!wstart || !edge) return hipErrorInvalidValue;
    return f64 ? edge_sum_t<double>(R, wstart, edge, qbar, p, stream)
               : edge_sum_t<float>(R, wstart, edge, qbar, p, stream);
}

namespace {

// One wave per row: lane l sums the row's tile terms l, l + 64, ... in order,
// then the lanes combine in a fixed butterfly (the same sum in every run).
__global__ __launch_bounds__(256) void k_v0_reduce(Rows R, const double *part, double *v0bar)
{
    const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    const int lane = (int)threadIdx.x % 64;
    if (row >= R.n_rows) return;
    int64_t t0, t1;
    if (R.n_cols > 0) {
        const int64_t tpr = (R.n_cols + R.tile - 1) / R.tile;
        t0 = row * tpr;
        t1 = t0 + tpr;
    } else {
        t0 = R.tile_ptr[row];
        t1 = R.tile_ptr[row + 1];
    }
    double s = 0.0;
    for (int64_t t = t0 + lane; t < t1; t += 64) s += part[t];
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
    if (lane == 0) v0bar[row] += s;
}

} // namespace

hipError_t launch_v0_reduce(const Rows &R, const double *part, double *v0bar,
                            hipStream_t stream)
{
    if (R.n_rows <= 0 || !v0bar) return hipSuccess;
    const dim3 g((unsigned)((R.n_rows + 3) / 4));
    hipLaunchKernelGGL(k_v0_reduce, g, dim3(256), 0, stream, R, part, v0bar);
    return hipGetLastError();
}

hipError_t launch_residual_adjoint(const ResidualAdjArgs &a, bool f64,
                                   hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.rows.n_tiles), block(kBlock);
    if (f64)
        hipLaunchKernelGGL(k_residual_adj<double>, grid, block, 0, stream, a);
    else
        hipLaunchKernelGGL(k_residual_adj<float>, grid, block, 0, stream, a);
    return hipGetLastError();
}

} // namespace ram
