// ram_step_fast64.hip -- the FP64 RAM step on rows that share one mesh, on the
// tile plan of the FP32 streaming kernels (gfx950).
//
// The computation of k_step_sh<double> (bulk shift of Section 3, Steps 1-3,
// Eqs. Qmass_i, condition_p, mass_shift_algo, step3, then the residual upwind
// step with the van Leer slope of Section 3.1) in the FP32 path's streaming
// layout: one tile of kFastTile destination cells per wave, no workgroup
// barrier, each tile's window and node data planned once per call
// (k_plan_fast, k_node_plan).  What FP64 changes:
//   * no stencil shortcut on uniform runs.  A run counts as uniform when its
//     cell sizes agree to kUniformTol of their size, far above FP64 rounding
//     (the bisection-solved meshes here vary by about 1e-11), so every node's
//     Lagrange weights are formed in FP64 from its source cell's stencil
//     data.  A uniform tile saves the node plan (node m of the tile lies in
//     window cell LO + m, or one cell beside it where the mesh's rounding
//     puts it there) and reads its cells' stencil data as FP32 deviations
//     from those of equally spaced nodes, which restore the FP64 values to
//     far below their rounding (the deviations are below about 1e-9 there);
//   * each node's position in its cell is formed here in FP64 from its
//     shifted coordinate (the plan keeps an FP32 one);
//   * the window's masses are staged in LDS (16-byte pairs where the row
//     allows), and in the prefix mode also their FP64 cumulative (four masses
//     a lane, scanned across the wave in DPP steps); each destination cell's mass
//     is its whole window cells plus the difference of its nodes' partial
//     integrals; the residual then runs on four consecutive cells a lane
//     from the shifted values in LDS.
// Tiles whose window exceeds the LDS buffer take the nodes' cells from the
// bucket index and sum from global memory.
#include "ram_device.h"
#include "ram_wave.h"

namespace ram {
namespace {

using namespace dev;

constexpr int kFT = kFastTile;
// LDS window of a wave, in cells: the plan's window capacity with direct
// sums; the prefix mode keeps the masses beside their cumulative (a single
// whole cell's mass is taken directly, as the general kernel does, so a shift
// by whole cells stays exact), in two arrays of kWinPre cells (wider windows
// take the global-memory path); each with room for the prefix's end and the
// 16-byte pairs' slack
constexpr int kWinPre = 384;
template <int S> constexpr int win64_cells() { return S == kScanF64 ? kWinPre : kFastWin; }

// Residual step in FP64 on four consecutive cells of a lane from the shifted
// state s[0..7] of cells i0+4l-2 .. i0+4l+5 (Section 3.1's upwind step, the
// face state the upwind linear profile averaged over the swept interval): fluxes
// on the five faces i0+4l .. i0+4l+4 with the upwind cell's van Leer slope
// and the swept-interval average, then the conservative update.  rr(c) gives
// (dx, 1/centre gap to the right) of s-index c, dxi(k) 1/dx of own cell k.
template <typename RR, typename DXI>
__device__ __forceinline__ void residual4d(const double *s, const double *dvv, double dt, RR rr,
                                           DXI dxi, double *out)
{
    double F[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const double v = dvv[k];
        const bool up = v >= 0.0;
        const double qm = up ? s[k] : s[k + 1];
        const double q0 = up ? s[k + 1] : s[k + 2];
        const double qp = up ? s[k + 2] : s[k + 3];
        const double2 rc = up ? rr(k + 1) : rr(k + 2);
        const double gm = up ? rr(k).y : rr(k + 1).y;
        const double dp = (qp - q0) * rc.y;
        const double dm = (q0 - qm) * gm;
        const double sig = (dp * dm <= 0.0) ? 0.0 : harmonic2(dp, dm);
        const double half = up ? 0.5 * (rc.x - v * dt) : -0.5 * (rc.x + v * dt);
        F[k] = v * (q0 + sig * half);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = s[k + 2] - dt * (F[k + 1] - F[k]) * dxi(k);
}

// Lagrange weights of the cumulative at theta through source cell c's nodes,
// from the mesh's FP64 stencil planes (pairs 1 .. P of stpd: node offsets th_b
// in units of dx_c other than the cell's own edges, 0 and 1, then reciprocal
// denominators rd_b other than the own node's, whose weight no partial
// integral uses), as prefix and suffix products of (theta - th_b).
// Neighbouring lanes read neighbouring cells' pairs: 16 bytes a lane a load.
template <int P>
__device__ __forceinline__ void node_weights(const double2 *stpd, int n, int c, double th,
                                             double (&wk)[P + 1])
{
    constexpr int LO = (P - 1) / 2;
    double v[2 * P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const double2 pr = stpd[(k + 1) * n + c];
        v[2 * k] = pr.x;
        v[2 * k + 1] = pr.y;
    }
    double rth[P + 1], rrd[P + 1];
    int k = 0;
#pragma unroll
    for (int b = 0; b <= P; ++b) rth[b] = b == LO ? 0.0 : (b == LO + 1 ? 1.0 : v[k++]);
#pragma unroll
    for (int b = 0; b <= P; ++b) rrd[b] = b == LO ? 0.0 : v[k++];
    double tt[P + 1], pre[P + 1], suf[P + 1];
#pragma unroll
    for (int b = 0; b <= P; ++b) tt[b] = th - rth[b];
    pre[0] = 1.0;
#pragma unroll
    for (int b = 1; b <= P; ++b) pre[b] = pre[b - 1] * tt[b - 1];
    suf[P] = 1.0;
#pragma unroll
    for (int b = P - 1; b >= 0; --b) suf[b] = suf[b + 1] * tt[b + 1];
#pragma unroll
    for (int b = 0; b <= P; ++b) wk[b] = rrd[b] * (pre[b] * suf[b]);
}

// Reciprocal Lagrange denominator of node a among P+1 equally spaced nodes.
template <int P>
__host__ __device__ constexpr double eq_denominator_inv(int a)
{
    double d = 1.0;
    for (int b = 0; b <= P; ++b)
        if (b != a) d *= (double)(a - b);
    return 1.0 / d;
}

// The same weights for a cell of a uniform run, from the FP32 deviations of
// its offsets and denominators from those of equally spaced nodes (stdv:
// float4, float4, float planes): 36 bytes a node instead of 80.
template <int P>
__device__ __forceinline__ void node_weights_uni(const float *stdv, int n, int c, double th,
                                                 double (&wk)[P + 1])
{
    constexpr int LO = (P - 1) / 2;
    float v[12];
    const float4 A = ((const float4 *)stdv)[c];
    v[0] = A.x; v[1] = A.y; v[2] = A.z; v[3] = A.w;
    if constexpr (2 * P - 1 > 4) {
        const float4 B = ((const float4 *)stdv)[n + c];
        v[4] = B.x; v[5] = B.y; v[6] = B.z; v[7] = B.w;
    }
    if constexpr (2 * P - 1 > 8) v[8] = stdv[8 * n + c];
    double rth[P + 1], rrd[P + 1];
    int k = 0;
#pragma unroll
    for (int b = 0; b <= P; ++b)
        rth[b] = b == LO ? 0.0 : (b == LO + 1 ? 1.0 : (double)(b - LO) + (double)v[k++]);
#pragma unroll
    for (int b = 0; b <= P; ++b)
        rrd[b] = b == LO ? 0.0 : eq_denominator_inv<P>(b) * (1.0 + (double)v[k++]);
    double tt[P + 1], pre[P + 1], suf[P + 1];
#pragma unroll
    for (int b = 0; b <= P; ++b) tt[b] = th - rth[b];
    pre[0] = 1.0;
#pragma unroll
    for (int b = 1; b <= P; ++b) pre[b] = pre[b - 1] * tt[b - 1];
    suf[P] = 1.0;
#pragma unroll
    for (int b = P - 1; b >= 0; --b) suf[b] = suf[b + 1] * tt[b + 1];
#pragma unroll
    for (int b = 0; b <= P; ++b) wk[b] = rrd[b] * (pre[b] * suf[b]);
}

// A node's shifted coordinate wrapped into [x0, xN), as node_pos forms it
// (the bucket, which a planned node does not need, left out).
__device__ __forceinline__ double shifted_xt(double xe, const RowShift &rs, double x0, double xN)
{
    const double xs = xe - rs.s;
    const double v0 = xs - rs.p0, vp = xs - rs.pp, vm = xs - rs.pm;
    return v0 >= xN ? vp : (v0 < x0 ? vm : v0);
}

// Position in cell c (pair 0 of stpd: its left edge and 1/dx) of a node at
// xt, taken across the period seam when c is the neighbour over it.
__device__ __forceinline__ double cell_theta(const double2 *stpd, int c, double xt, double len)
{
    const double2 g = stpd[c];
    double d = xt - g.x;
    d = d > 0.5 * len ? d - len : (d < -0.5 * len ? d + len : d);
    return d * g.y;
}

// One tile.  S: kSumDirect (partials and whole cells summed from the window
// masses) or kScanF64 (differences of the window's FP64 cumulative).
template <int P, int H, int S, bool VEC>
__device__ __forceinline__ void tile64(const StepArgs &a, const FastTile &ft, double *sw,
                                       double *sp, double *sell, short *sjc, int t)
{
    constexpr int LO = (P - 1) / 2;
    constexpr bool kPre = S == kScanF64;
    constexpr int NS = (kFT + 2 * H + 1 + kLanes - 1) / kLanes;   // node slots
    constexpr int NCS = (kFT + 2 * H + kLanes - 1) / kLanes;      // shifted-cell slots
    const Rows &R = a.rows;
    const MeshTab &tb = R.tab;
    const int n = (int)R.n_cols;
    const int c4 = 4 * t;
    const TilePos tp = tile_pos(ft.pad[0], n, H);
    const int row = tp.row, i0 = tp.i0, nd = tp.nd;
    const int NC = nd + 2 * H;
    const int NE = NC + 1;
    const int64_t qoff = (int64_t)row * n;
    const double *q = (const double *)a.q_in + qoff;
    double *qo = (double *)a.q_out + qoff;
    const int W = ft.w, base = ft.base;
    const bool direct = ft.kind == kFastDirect || ft.w > win64_cells<S>();
    const bool uniform = ft.kind == kFastUniform;
    const double *x = R.edges;
    const double x0 = x[0], xN = x[n];
    const double len = xN - x0;
    const RowShift rs = row_shift(a.v0[row] * a.dt, len, tb.scal[1]);
    int64_t *sg = (int64_t *)sw;                     // direct tiles: the nodes' extended cells

    // faces of the residual (issued first: they are not needed until the end)
    double dvv[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if constexpr (H != 0) {
        const double *dvp = (const double *)a.dv + qoff;
        const int cc = min(c4, nd - 1);
        if constexpr (VEC) {
            // rows of a multiple of four cells: the lane's four faces in whole
            // 16-byte pairs
            const int fb = i0 + (cc & ~3);
            const double2 f0 = *(const double2 *)(dvp + fb);
            const double2 f1 = *(const double2 *)(dvp + fb + 2);
            dvv[0] = f0.x;
            dvv[1] = f0.y;
            dvv[2] = f1.x;
            dvv[3] = f1.y;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int f = i0 + min(cc + k, nd);
                dvv[k] = dvp[f >= n ? f - n : f];
            }
        }
        const int f4 = i0 + min(cc + 4, nd);
        dvv[4] = dvp[f4 >= n ? f4 - n : f4];
    }

    // the destination cells' 1/dx (issued here, used after the partials)
    double dxc[NCS];
#pragma unroll
    for (int u = 0; u < NCS; ++u) dxc[u] = tb.dxinv[wrap1f(i0 - H + min(t + u * kLanes, NC - 1), n)];

    // window cell j at sw[j + off]
    int off = 0;
    if (!direct) {
        // ---- window masses M = Q dx, every load issued ---------------------------
        if (VEC && base + W + 1 < 2 * n) {
            // 16-byte pairs from the even cell at or below the window start
            off = base & 1;
            const int a0 = base - off;
            const int gl = (W + off - 1) >> 1;           // last pair
            const int nps = gl / kLanes + 1;
            for (int r0 = 0; r0 < nps; r0 += 3) {
                double2 wq[3], wd[3];
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    int c = a0 + 2 * min(t + (r0 + u) * kLanes, gl);
                    c = c >= n ? c - n : c;
                    wq[u] = *(const double2 *)(q + c);
                    wd[u] = *(const double2 *)(tb.dx + c);
                }
#pragma unroll
                for (int u = 0; u < 3; ++u) {
                    const int g = min(t + (r0 + u) * kLanes, gl);
                    if (r0 + u < nps)
                        *(double2 *)(sw + 2 * g) = make_double2(wq[u].x * wd[u].x, wq[u].y * wd[u].y);
                }
            }
        } else {
            const int nws = (W + kLanes - 1) / kLanes;
            const bool wraps = W + base > 2 * n;     // rows shorter than the window
            for (int r0 = 0; r0 < nws; r0 += 4) {
                double wq[4], wd[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    int mm = base + min(t + (r0 + u) * kLanes, W - 1);
                    mm = wraps ? wrap_small(mm, n) : (mm >= n ? mm - n : mm);
                    wq[u] = q[mm];
                    wd[u] = tb.dx[mm];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (r0 + u < nws) sw[t + (r0 + u) * kLanes] = wq[u] * wd[u];
            }
        }
        // ---- each node's window index and position in its cell ---------------------
        const int16_t *jcp =
            ft.kind == kFastWindow ? a.fast.jc + (int64_t)ft.pad[1] * kFastNodes : nullptr;
        // (a window wraps the row at most once unless the row is shorter than it)
        const bool wrapw = W + base > 2 * n;
        auto wcell = [&](int j) {
            const int c = base + j;
            return wrapw ? wrap_small(c, n) : (c >= n ? c - n : c);
        };
        int jv[NS], cv[NS];
        double thv[NS];
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const int m = min(t + u * kLanes, NE - 1);
            int e = i0 - H + m;
            e = e < 0 ? e + n : (e >= n ? e - n : e);
            const double xt = shifted_xt(x[e], rs, x0, xN);
            int j = jcp ? (int)jcp[m] : LO + m;
            int c = wcell(j);
            double th = cell_theta(tb.stpd, c, xt, len);
            // a uniform tile's inner node that the mesh's rounding puts in a
            // neighbouring cell (the end nodes' cells came from the search)
            if (!jcp && m > 0 && m < NE - 1 && (th < 0.0 || th >= 1.0)) {
                j += th < 0.0 ? -1 : 1;
                c = wcell(j);
                th = cell_theta(tb.stpd, c, xt, len);
            }
            jv[u] = j;
            cv[u] = c;
            thv[u] = th;
        }
        wave_sync();                                 // the window masses
        if constexpr (kPre) {
            // exclusive FP64 cumulative of the masses into sp: LDS cells 4g ..
            // 4g+3 a lane (group g = lane + 64 s), cells past the window as zero
            using AC = Acc<kScanF64>;
            const int WL = W + off;
            const int gl = (WL - 1) >> 2;
            double carry = 0.0;
            for (int s = 0; s * kLanes <= gl; ++s) {
                const int g = t + s * kLanes;
                double m[4] = {0.0, 0.0, 0.0, 0.0};
                if (g <= gl) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) m[k] = 4 * g + k < WL ? sw[4 * g + k] : 0.0;
                }
                const double tot = g <= gl ? (m[0] + m[1]) + (m[2] + m[3]) : 0.0;
                const double inc = wave_inclusive<AC>(tot);
                double ex = AC::dpp<kDppWaveShr1, 0xf, 0xf>(inc);
                if (t == 0) ex = 0.0;
                double e = carry + ex;
                if (g <= gl) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        sp[4 * g + k] = e;
                        e += m[k];
                    }
                    if (g == gl) sp[4 * g + 4] = e;
                }
                carry += lane63(inc);
            }
            wave_sync();
        }
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const int m = min(t + u * kLanes, NE - 1);
            double wk[P + 1];
            if (uniform)
                node_weights_uni<P>(tb.stdv, n, cv[u], thv[u], wk);
            else
                node_weights<P>(tb.stpd, n, cv[u], thv[u], wk);
            const int j = jv[u] + off;
            double ell = 0.0;
            if constexpr (kPre) {
                const double pc = sp[j];
#pragma unroll
                for (int b = 0; b <= P; ++b)
                    if (b != LO) ell += wk[b] * (sp[j - LO + b] - pc);
            } else {
                double up = 0.0, dn = 0.0;
#pragma unroll
                for (int b = LO + 1; b <= P; ++b) {
                    up += sw[j + b - LO - 1];
                    ell += wk[b] * up;
                }
#pragma unroll
                for (int b = LO - 1; b >= 0; --b) {
                    dn += sw[j - LO + b];
                    ell -= wk[b] * dn;
                }
            }
            sell[m] = ell;
            sjc[m] = (short)j;
        }
        wave_sync();
    } else {
        // window wider than the LDS buffer: nodes located here, partial
        // integrals and whole-cell sums from global memory
        const double sh = a.v0[row] * a.dt;
        for (int m = t; m < NE; m += kLanes) {
            int e = i0 - H + m;
            const int kx = e < 0 ? -n : (e >= n ? n : 0);
            e -= kx;
            const NodePos np = node_pos(x[e], rs, x0, xN, tb.scal[0], tb.scal[2], tb.nb);
            const double2 nx = tb.bnext[np.b];
            int c = cell_from_bucket(tb.bucket[np.b], nx, np.xt);
            if (np.xt >= nx.y) c = cell_walk(x, n, c, np.xt);
            const int64_t g = (int64_t)c + (rs.kf0 + np.dk) * (int64_t)n + kx;
            sg[m] = g;
            sell[m] = direct_partial<double, P>(x, q, n, len, sh, tb.scal[1], i0 - H + m, g);
        }
        wave_sync();
    }

    // the residual's geometry (on its way during the destination cells' sums):
    // each tile cell's (dx, 1/centre gap) one cell a lane, passed through LDS
    // to the four-cells-a-lane layout (read there directly, the lanes' 16-byte
    // pairs four cells apart would each span 32 cache lines), and 1/dx of the
    // lane's own four cells
    double2 gq[H != 0 ? NCS : 1];
    double dxi[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (H != 0) {
#pragma unroll
        for (int u = 0; u < NCS; ++u) gq[u] = tb.rrd[wrap1f(i0 - H + min(t + u * kLanes, NC - 1), n)];
        if constexpr (VEC) {
            const int d0 = i0 + (min(c4, nd - 1) & ~3);
            const double2 x01 = *(const double2 *)(tb.dxinv + d0);
            const double2 x23 = *(const double2 *)(tb.dxinv + d0 + 2);
            dxi[0] = x01.x;
            dxi[1] = x01.y;
            dxi[2] = x23.x;
            dxi[3] = x23.y;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) dxi[k] = tb.dxinv[min(i0 + c4 + k, n - 1)];
        }
    }

    // ---- destination cells, one a lane: whole cells + two partials, / dx -------
    // (lanes past the last cell repeat it: same values, same places)
    double qs[NCS];
#pragma unroll
    for (int u = 0; u < NCS; ++u) {
        const int ci = min(t + u * kLanes, NC - 1);
        const int cell = wrap1f(i0 - H + ci, n);
        double mp;
        if (!direct) {
            const int ja = sjc[ci], jb = sjc[ci + 1];
            double whole;
            if constexpr (kPre) {
                whole = jb - ja == 1 ? sw[ja] : sp[jb] - sp[ja];
            } else {
                whole = jb > ja ? sw[ja] : 0.0;
                for (int mm = ja + 1; mm < jb; ++mm) whole += sw[mm];
            }
            mp = whole + (sell[ci + 1] - sell[ci]);
        } else {
            mp = direct_whole<double>(x, q, n, sg[ci], sg[ci + 1]) + (sell[ci + 1] - sell[ci]);
        }
        qs[u] = mp * dxc[u];
        if constexpr (H == 0) {
            qo[cell] = qs[u];
        } else if (a.q_mid && ci >= H && ci < H + nd) {
            ((double *)a.q_mid + qoff)[cell] = qs[u];
        }
    }
    if constexpr (H != 0) {
        wave_sync();                                 // window and partials are dead
        // tile cell ci (cell i0 - H + ci): shifted value, dx, 1/centre gap
        double *sq = sell;
        double *sdx = sw;
        double *shi = kPre ? sp : sw + kFastNodes;
#pragma unroll
        for (int u = 0; u < NCS; ++u) {
            const int ci = min(t + u * kLanes, NC - 1);
            sq[ci] = qs[u];
            sdx[ci] = gq[u].x;
            shi[ci] = gq[u].y;
        }
        wave_sync();
        if (c4 < nd) {
            double sv[8];
            double2 rr[7];
#pragma unroll
            for (int c = 0; c < 8; ++c) sv[c] = sq[min(c4 + c, NC - 1)];
#pragma unroll
            for (int c = 0; c < 7; ++c) {
                const int ci = min(c4 + c, NC - 1);
                rr[c] = make_double2(sdx[ci], shi[ci]);
            }
            double o[4];
            residual4d(sv, dvv, a.dt, [&](int c) { return rr[c]; },
                       [&](int k) { return dxi[k]; }, o);
            if (VEC) {
                *(double2 *)(qo + i0 + c4) = make_double2(o[0], o[1]);
                *(double2 *)(qo + i0 + c4 + 2) = make_double2(o[2], o[3]);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (c4 + k < nd) qo[i0 + c4 + k] = o[k];
            }
        }
    }
}

// Every tile in tile order, one a wave; LDS of one wave: the window (masses,
// cumulative, or the direct tiles' node cells, then the shifted values), the
// nodes' partial integrals and window indices.
template <int P, int H, int S, bool VEC>
__global__ __launch_bounds__(kBlock) void k_step64(StepArgs a)
{
    constexpr int WC = win64_cells<S>() + 8;
    __shared__ __attribute__((aligned(16))) double sw_[kWaves][WC];
    __shared__ __attribute__((aligned(16))) double sp_[kWaves][S == kScanF64 ? WC : 1];
    __shared__ __attribute__((aligned(16))) double sell_[kWaves][kFastNodes];
    __shared__ __attribute__((aligned(16))) short sjc_[kWaves][kFastNodes];
    const int wid = wave_id();
    const int i = (int)blockIdx.x * kWaves + wid;
    if (i >= (int)a.rows.n_tiles) return;
    const FastTile r = load_rec(a.fast.rec, i);
    tile64<P, H, S, VEC>(a, r, sw_[wid], sp_[wid], sell_[wid], sjc_[wid],
                         (int)threadIdx.x % kLanes);
}

template <int P, int S>
hipError_t step64_ps(const StepArgs &a, bool vec, hipStream_t st)
{
    const dim3 g((unsigned)((a.rows.n_tiles + kWaves - 1) / kWaves)), b(kBlock);
    if (a.dv) {
        if (vec) hipLaunchKernelGGL((k_step64<P, 2, S, true>), g, b, 0, st, a);
        else hipLaunchKernelGGL((k_step64<P, 2, S, false>), g, b, 0, st, a);
    } else {
        if (vec) hipLaunchKernelGGL((k_step64<P, 0, S, true>), g, b, 0, st, a);
        else hipLaunchKernelGGL((k_step64<P, 0, S, false>), g, b, 0, st, a);
    }
    return hipGetLastError();
}

template <int P>
hipError_t step64_p(const StepArgs &a, int scan, hipStream_t st)
{
    // 16-byte pairs: rows of a multiple of four cells, 16-byte aligned states
    const bool vec = (a.rows.n_cols % 4) == 0 && ((uintptr_t)a.q_out % 16) == 0 &&
                     ((uintptr_t)a.q_in % 16) == 0 && (!a.dv || ((uintptr_t)a.dv % 16) == 0);
    return scan == kSumDirect ? step64_ps<P, kSumDirect>(a, vec, st)
                              : step64_ps<P, kScanF64>(a, vec, st);
}

} // namespace

hipError_t launch_step_fast64(const StepArgs &a, int order, int scan, hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    if (a.rows.tile != kFastTile) return hipErrorInvalidValue;
    switch (order) {
    case 1: return step64_p<1>(a, scan, stream);
    case 3: return step64_p<3>(a, scan, stream);
    default: return step64_p<5>(a, scan, stream);
    }
}

} // namespace ram
