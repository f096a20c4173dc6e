// ram_device.h -- device-side helpers of the RAM HIP kernels (tile mapping,
// periodic mesh access, shifted-node location, Lagrange weights, block scans
// in three precisions).  Private to the library's .hip files.
#pragma once

#include "ram_internal.h"

#include <math.h>

namespace ram {
namespace dev {


struct Tile {
    int64_t row;
    int32_t i0;      // first destination cell of the tile within the row
    int32_t n;       // cells in the row
    int64_t qoff;    // offset of the row's first cell
    const double *x; // the row's N+1 nodes
};

__device__ inline bool get_tile(const Rows &R, int64_t t, Tile &ti)
{
    if (R.n_cols > 0) {
        const int64_t tpr = (R.n_cols + R.tile - 1) / R.tile;
        ti.row = t / tpr;
        if (ti.row >= R.n_rows) return false;
        ti.i0 = (int32_t)((t - ti.row * tpr) * R.tile);
        ti.n = (int32_t)R.n_cols;
        ti.qoff = ti.row * R.n_cols;
        ti.x = R.shared ? R.edges : R.edges + ti.row * (R.n_cols + 1);
    } else {
        if (t >= R.tile_ptr[R.n_rows]) return false;
        ti.row = R.tile_row[t];
        ti.i0 = (int32_t)((t - R.tile_ptr[ti.row]) * R.tile);
        ti.qoff = R.row_ptr[ti.row];
        ti.n = (int32_t)(R.row_ptr[ti.row + 1] - ti.qoff);
        ti.x = R.edges + ti.qoff + ti.row;
    }
    return true;
}

__device__ inline int wrapi(int64_t m, int n)
{
    int64_t r = m % n;
    return (int)(r < 0 ? r + n : r);
}

// Node of the periodically extended mesh, j in [-n, 2n].
__device__ inline double node_x(const double *x, int n, double len, int j)
{
    if (j < 0) return x[j + n] - len;
    if (j > n) return x[j - n] + len;
    return x[j];
}

// Largest j in [0, n-1] with x[j] <= xh (right-continuous).
__device__ inline int find_cell(const double *x, int n, double xh)
{
    if (!(xh >= x[0])) return 0;
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        if (x[mid] <= xh) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Same result as find_cell through the mesh's bucket index: start from the
// bucket's lower-bound cell, step down while the node lies above xh (only after
// rounding in the bucket number) and walk up over the few nodes in the bucket.
__device__ inline int find_cell_tab(const double *x, int n, const MeshTab &tb,
                                    double bscale, double xh)
{
    int b = (int)((xh - x[0]) * bscale);
    b = min(max(b, 0), tb.nb - 1);
    int c = tb.bucket[b];
    while (c > 0 && x[c] > xh) --c;
    while (c + 1 < n && x[c + 1] <= xh) ++c;
    return c;
}

// x~ = x[e] - s written as xh + k L, xh in [x0, xN).
__device__ inline void shifted_node(const double *x, int n, double s, int e,
                                    double &xh, int64_t &k)
{
    const double len = x[n] - x[0];
    const double xt = x[e] - s;
    const double kf = floor((xt - x[0]) / len);
    xh = xt - kf * len;
    k = (int64_t)kf;
    if (xh >= x[n]) { xh -= len; k += 1; }
    else if (xh < x[0]) { xh += len; k -= 1; }
}

// Same as shifted_node with the division by L replaced by a product with
// 1/L: the wrap fix-ups keep xh in [x0, xN) and xh + k L = x~ either way.
__device__ inline void shifted_node_inv(const double *x, int n, double s, int e,
                                        double invlen, double len, double &xh,
                                        int64_t &k)
{
    const double xt = x[e] - s;
    const double kf = floor((xt - x[0]) * invlen);
    xh = xt - kf * len;
    k = (int64_t)kf;
    if (xh >= x[n]) { xh -= len; k += 1; }
    else if (xh < x[0]) { xh += len; k -= 1; }
}

// DPP lane movements of a wave64 (GFX9 encodings): shift right within a row
// of 16 lanes, broadcast of lane 15 / 31 to the following rows, and a shift
// right by one lane across the whole wave.  Lanes without a source read 0.
enum : int {
    kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114,
    kDppRowShr8 = 0x118, kDppWaveShr1 = 0x138, kDppBcast15 = 0x142,
    kDppBcast31 = 0x143
};

template <int CTRL, int RM, int BM>
__device__ inline int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, RM, BM, false);
}
template <int CTRL, int RM, int BM>
__device__ inline float dpp_f(float v)
{
    return __int_as_float(dpp_i<CTRL, RM, BM>(__float_as_int(v)));
}
template <int CTRL, int RM, int BM>
__device__ inline double dpp_d(double v)
{
    const long long u = __double_as_longlong(v);
    const int lo = dpp_i<CTRL, RM, BM>((int)(u & 0xffffffffll));
    const int hi = dpp_i<CTRL, RM, BM>((int)(u >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int P>
__device__ inline void lagrange_weights(double xh, const double *X, double *w)
{
    double t[P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) t[a] = xh - X[a];
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        double num = 1.0, den = 1.0;
#pragma unroll
        for (int b = 0; b <= P; ++b) {
            if (b == a) continue;
            num *= t[b];
            den *= X[a] - X[b];
        }
        w[a] = num / den;
    }
}

// Lagrange weights at t of the nodes X[0..P] given relative to the stencil's
// cell (X[lo] = 0, X[lo+1] = dx_c): normalised by dx_c, products of all
// differences but one, one division per weight, in WT.
template <typename WT, int P>
__device__ inline void lagrange_rel(double t, const double *X, WT *w)
{
    constexpr int LO = (P - 1) / 2;
    const double inv = 1.0 / X[LO + 1];
    WT th[P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) th[a] = (WT)(X[a] * inv);
    const WT tt = (WT)(t * inv);
    WT pre[P + 1], suf[P + 1];
    pre[0] = (WT)1;
#pragma unroll
    for (int a = 1; a <= P; ++a) pre[a] = pre[a - 1] * (tt - th[a - 1]);
    suf[P] = (WT)1;
#pragma unroll
    for (int a = P - 1; a >= 0; --a) suf[a] = suf[a + 1] * (tt - th[a + 1]);
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        WT den = (WT)1;
#pragma unroll
        for (int b = 0; b <= P; ++b)
            if (b != a) den *= th[a] - th[b];
        w[a] = pre[a] * suf[a] / den;
    }
}

// ---------------------------------------------------------------------------
// prefix-sum precisions
// ---------------------------------------------------------------------------

__device__ inline void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

template <int S> struct Acc;

template <> struct Acc<kScanF64> {
    using M = double;
    using A = double;
    using D = double;   // type of prefix differences
    template <typename TQ>
    __device__ static M mass(TQ q, double dx) { return (double)q * dx; }
    __device__ static A zero() { return 0.0; }
    __device__ static A add(A a, M m) { return a + m; }
    __device__ static A comb(A a, A b) { return a + b; }
    __device__ static D diff(A b, A a) { return b - a; }
    __device__ static A shfl_up(A v, int d) { return __shfl_up(v, d); }
    template <int C, int RM, int BM> __device__ static A dpp(A v) { return dpp_d<C, RM, BM>(v); }
};

template <> struct Acc<kScanTwoSum> {
    using M = float;
    using A = float2;   // (hi, lo): value = hi + lo
    using D = float;
    template <typename TQ>
    __device__ static M mass(TQ q, double dx) { return (float)q * (float)dx; }
    __device__ static A zero() { return make_float2(0.f, 0.f); }
    __device__ static A add(A a, M m)
    {
        float s, e;
        two_sum(a.x, m, s, e);
        const float lo = a.y + e;
        const float hi = s + lo;
        return make_float2(hi, lo - (hi - s));
    }
    __device__ static A comb(A a, A b)
    {
        float s, e;
        two_sum(a.x, b.x, s, e);
        const float lo = a.y + b.y + e;
        const float hi = s + lo;
        return make_float2(hi, lo - (hi - s));
    }
    __device__ static D diff(A b, A a)
    {
        return (b.x - a.x) + (b.y - a.y);
    }
    __device__ static A shfl_up(A v, int d)
    {
        return make_float2(__shfl_up(v.x, d), __shfl_up(v.y, d));
    }
    template <int C, int RM, int BM> __device__ static A dpp(A v)
    {
        return make_float2(dpp_f<C, RM, BM>(v.x), dpp_f<C, RM, BM>(v.y));
    }
};

template <> struct Acc<kScanF32> {
    using M = float;
    using A = float;
    using D = float;
    template <typename TQ>
    __device__ static M mass(TQ q, double dx) { return (float)q * (float)dx; }
    __device__ static A zero() { return 0.f; }
    __device__ static A add(A a, M m) { return a + m; }
    __device__ static A comb(A a, A b) { return a + b; }
    __device__ static D diff(A b, A a) { return b - a; }
    __device__ static A shfl_up(A v, int d) { return __shfl_up(v, d); }
    template <int C, int RM, int BM> __device__ static A dpp(A v) { return dpp_f<C, RM, BM>(v); }
};

// Exclusive scan over the workgroup of one value per thread; also returns
// the total.  wave_tot: LDS scratch of kBlock/64 entries.
template <class AC>
__device__ typename AC::A block_exscan(typename AC::A v, typename AC::A *wave_tot,
                                       typename AC::A &total)
{
    using A = typename AC::A;
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    A inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const A o = AC::shfl_up(inc, d);
        if (lane >= d) inc = AC::comb(o, inc);
    }
    A exc = AC::shfl_up(inc, 1);
    if (lane == 0) exc = AC::zero();
    if (lane == 63) wave_tot[wid] = inc;
    __syncthreads();
    A off = AC::zero();
    A tot = AC::zero();
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wid) off = AC::comb(off, wave_tot[w]);
        tot = AC::comb(tot, wave_tot[w]);
    }
    total = tot;
    __syncthreads();
    return AC::comb(off, exc);
}

// Exclusive scan over the workgroup of one value per thread, with DPP lane
// movements inside each wave and the wave totals combined through LDS; also
// returns the total.  wave_tot: LDS scratch of kBlock/64 entries.
template <class AC>
__device__ typename AC::A block_exscan_dpp(typename AC::A v,
                                           typename AC::A *wave_tot,
                                           typename AC::A &total)
{
    using A = typename AC::A;
    const int lane = threadIdx.x & 63;
    const int wid = threadIdx.x >> 6;
    A inc = v;
    inc = AC::comb(AC::template dpp<kDppRowShr1, 0xf, 0xf>(inc), inc);
    inc = AC::comb(AC::template dpp<kDppRowShr2, 0xf, 0xf>(inc), inc);
    inc = AC::comb(AC::template dpp<kDppRowShr4, 0xf, 0xf>(inc), inc);
    inc = AC::comb(AC::template dpp<kDppRowShr8, 0xf, 0xf>(inc), inc);
    inc = AC::comb(AC::template dpp<kDppBcast15, 0xa, 0xf>(inc), inc);
    inc = AC::comb(AC::template dpp<kDppBcast31, 0xc, 0xf>(inc), inc);
    A exc = AC::template dpp<kDppWaveShr1, 0xf, 0xf>(inc);
    if (lane == 0) exc = AC::zero();
    if (lane == 63) wave_tot[wid] = inc;
    __syncthreads();
    A off = AC::zero();
    A tot = AC::zero();
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wid) off = AC::comb(off, wave_tot[w]);
        tot = AC::comb(tot, wave_tot[w]);
    }
    total = tot;
    __syncthreads();
    return AC::comb(off, exc);
}

__device__ inline double centre(const double *x, int i) { return 0.5 * (x[i] + x[i + 1]); }

// Distance between the centres of cells i and i+1 (periodic).
__device__ inline double centre_gap(const double *x, int n, double len, int64_t i)
{
    const int w = wrapi(i, n);
    if (w == n - 1) return centre(x, 0) + len - centre(x, n - 1);
    return centre(x, w + 1) - centre(x, w);
}

// Periodic index for j in [-n, k n).
__device__ inline int wrap_small(int j, int n)
{
    if (j < 0) j += n;
    while (j >= n) j -= n;
    return j;
}

template <typename TQ>
__device__ inline double cell_mass(const double *x, const TQ *q, int n, int64_t m)
{
    const int w = wrapi(m, n);
    return (double)q[w] * (x[w + 1] - x[w]);
}

// Partial integral C~(xh) - C(c) from global memory (direct path).
template <typename TQ, int P>
__device__ double partial_direct(const double *x, const TQ *q, int n, double len,
                                 int64_t g, double xh)
{
    constexpr int LO = (P - 1) / 2;
    const int c = wrapi(g, n);
    double X[P + 1], w[P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) X[a] = node_x(x, n, len, c - LO + a);
    lagrange_weights<P>(xh, X, w);
    double ell = 0.0;
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        const int j = c - LO + a;
        double d = 0.0;
        if (j > c) {
            for (int m = c; m < j; ++m) d += cell_mass(x, q, n, m);
        } else if (j < c) {
            for (int m = j; m < c; ++m) d += cell_mass(x, q, n, m);
            d = -d;
        }
        ell += w[a] * d;
    }
    return ell;
}

// Per-type views of the shared-mesh tables.
template <typename T> struct TabT;
template <> struct TabT<double> {
    using T2 = double2;
    __device__ static const double *dx(const MeshTab &t) { return t.dx; }
    __device__ static const double *dxinv(const MeshTab &t) { return t.dxinv; }
    __device__ static const double *hinv(const MeshTab &t) { return t.hinv; }
    __device__ static const double2 *rr(const MeshTab &t) { return t.rrd; }
};
template <> struct TabT<float> {
    using T2 = float2;
    __device__ static const float *dx(const MeshTab &t) { return t.dxf; }
    __device__ static const float *dxinv(const MeshTab &t) { return t.dxinvf; }
    __device__ static const float *hinv(const MeshTab &t) { return t.hinvf; }
    __device__ static const float2 *rr(const MeshTab &t) { return t.rrf; }
};

// 2ab/(a+b) of the van Leer slope (a b > 0): FP32 with the hardware
// reciprocal, FP64 with a division.
__device__ inline float harmonic2(float a, float b)
{
    return 2.0f * a * b * __builtin_amdgcn_rcpf(a + b);
}
__device__ inline double harmonic2(double a, double b)
{
    return 2.0 * a * b / (a + b);
}

// Direct path of k_step (tiles whose source window does not fit in LDS):
// partial integrals from global memory, FP64.
template <typename TQ, int P>
__device__ __attribute__((noinline)) double direct_partial(
    const double *x, const TQ *q, int n, double len, double s, double invlen,
    int e, int64_t g)
{
    if (e < 0) e += n;
    while (e >= n) e -= n;
    double xh;
    int64_t kk;
    shifted_node_inv(x, n, s, e, invlen, len, xh, kk);
    return partial_direct<TQ, P>(x, q, n, len, g, xh);
}

template <typename TQ>
__device__ __attribute__((noinline)) double direct_whole(const double *x,
                                                         const TQ *q, int n,
                                                         int64_t ga, int64_t gb)
{
    double wh = 0.0;
    for (int64_t m = ga; m < gb; ++m) wh += cell_mass(x, q, n, m);
    return wh;
}

// ---- shifted-node search on a shared mesh (step and adjoint kernels) ----

template <typename T> struct RecT;
template <> struct RecT<float> {
    __device__ static const CellRec<float> *get(const MeshTab &t)
    {
        return (const CellRec<float> *)t.crf;
    }
};
template <> struct RecT<double> {
    __device__ static const CellRec<double> *get(const MeshTab &t)
    {
        return (const CellRec<double> *)t.crd;
    }
};

// Per-row constants of the node search.  kf0 = floor(-s/L) whole periods
// are taken out of every shifted node x - s, which then lies in
// [x0 - kf0 L ... ) so that at most one more period (up or down, the latter
// only through rounding) brings it into [x0, xN).  The products k L are
// formed once, so a node's wrapped position is (x - s) - k L with the same
// two roundings as the plain definition.
struct RowShift {
    double s;       // the shift v0 dt
    double p0;      // kf0 L
    double pp;      // (kf0 + 1) L
    double pm;      // (kf0 - 1) L
    int64_t kf0;
};

__device__ inline RowShift row_shift(double s, double len, double invlen)
{
    const double kf = floor(-s * invlen);
    return {s, kf * len, (kf + 1.0) * len, (kf - 1.0) * len, (int64_t)kf};
}

// Node x (a coordinate of the row's own nodes) shifted by s: its position
// wrapped into [x0, xN), the period it took beyond kf0 (0, 1, or -1 through
// rounding) and its bucket.
struct NodePos {
    double xt;
    int dk;
    int b;
};

__device__ inline NodePos node_pos(double xe, const RowShift &rs, double x0, double xN,
                                   double bsc, double bx0, int nb)
{
    // all three candidates, then selects (no divergent branch)
    const double xs = xe - rs.s;
    const double v0 = xs - rs.p0, vp = xs - rs.pp, vm = xs - rs.pm;
    const bool hi = v0 >= xN, lo = v0 < x0;
    const double v = hi ? vp : (lo ? vm : v0);
    const int d = hi ? 1 : (lo ? -1 : 0);
    int b = (int)(v * bsc - bx0);
    b = min(max(b, 0), nb - 1);
    return {v, d, b};
}

// Source cell from the bucket's lower-bound cell and the next two nodes; the
// walk past them is only taken on meshes finer than the buckets.
__device__ inline int cell_from_bucket(int cb, double2 nx, double xt)
{
    return cb + (xt >= nx.x ? 1 : 0) + (xt >= nx.y ? 1 : 0);
}

__device__ inline int cell_walk(const double *x, int n, int c, double xt)
{
    while (c + 1 < n && x[c + 1] <= xt) ++c;
    return c;
}

// Lagrange weights of the stencil of cell record r at position xt.
template <typename WT, int P>
__device__ inline void rec_weights(const CellRec<WT> &r, double xt, WT *w)
{
    const WT th = (WT)((xt - r.xc) * r.dxinv);
    WT t[P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) t[a] = th - r.th[a];
    WT pre[P + 1], suf[P + 1];
    pre[0] = (WT)1;
#pragma unroll
    for (int a = 1; a <= P; ++a) pre[a] = pre[a - 1] * t[a - 1];
    suf[P] = (WT)1;
#pragma unroll
    for (int a = P - 1; a >= 0; --a) suf[a] = suf[a + 1] * t[a + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) w[a] = r.rd[a] * (pre[a] * suf[a]);
}

// Lagrange weights of a uniform stencil (nodes at -LO .. P-LO cell sizes from
// the cell's left node) at theta: the cell record's weights on a uniform run.
template <typename CT, int P>
__device__ inline void uniform_weights(CT th, CT *w)
{
    constexpr int LO = (P - 1) / 2;
    CT t[P + 1], pre[P + 1], suf[P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) t[a] = th - (CT)(a - LO);
    pre[0] = (CT)1;
#pragma unroll
    for (int a = 1; a <= P; ++a) pre[a] = pre[a - 1] * t[a - 1];
    suf[P] = (CT)1;
#pragma unroll
    for (int a = P - 1; a >= 0; --a) suf[a] = suf[a + 1] * t[a + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        double den = 1.0;                 // prod_{b != a} (a - b), exact
        for (int b = 0; b <= P; ++b)
            if (b != a) den *= (double)(a - b);
        w[a] = (CT)(1.0 / den) * (pre[a] * suf[a]);
    }
}

// The weights of the masses M_{j+e} in the partial integral of a node in
// cell j whose stencil weights are w: the weights above the node summed down
// to e for e >= 0, minus the weights below summed up to e for e < 0, stored
// at g[e + LO + 1] for e = -LO .. P-LO-1, with g[0] = g[P+1] = 0.
template <typename T, int P>
__device__ inline void outward_sums(const T *w, T *g)
{
    constexpr int LO = (P - 1) / 2;
    g[0] = g[P + 1] = (T)0;
    T acc = (T)0;
#pragma unroll
    for (int e = P - LO - 1; e >= 0; --e) {
        acc += w[LO + 1 + e];
        g[e + LO + 1] = acc;
    }
    acc = (T)0;
#pragma unroll
    for (int e = -LO; e < 0; ++e) {
        acc += w[LO + e];
        g[e + LO + 1] = -acc;
    }
}

// The shift of a uniform run as one stencil on cell values.  With every cell
// of size h, the partial integral of the node in cell j is the fixed
// combination sum_e g_e M_{j+e} (outward_sums), so the destination mass
// M_j + ell(j+1) - ell(j) weighs M_{j+d} by [d == 0] + g_{d-1} - g_d,
// d = -LO .. P-LO, and dividing by h gives the shifted cell value as the same
// combination of the values Q_{j+d}: cc[d + LO].  The weights sum to one
// (the g terms telescope), which is the shift's conservation.
template <typename CT, int P>
__device__ inline void uniform_stencil(CT th, CT *cc)
{
    constexpr int LO = (P - 1) / 2;
    CT w[P + 1], g[P + 2];
    uniform_weights<CT, P>(th, w);
    outward_sums<CT, P>(w, g);
#pragma unroll
    for (int d = 0; d <= P; ++d) cc[d] = (d == LO ? (CT)1 : (CT)0) + g[d] - g[d + 1];
}

// Their derivatives with respect to x (theta over the cell size dx, 1/dx =
// dxinv), in FP64 as the cell-record form gives them.
template <typename CT, int P>
__device__ inline void uniform_dweights(CT th, double dxinv, double *dw)
{
    constexpr int LO = (P - 1) / 2;
    CT t[P + 1], pre[P + 1], suf[P + 1], dpre[P + 1], dsuf[P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) t[a] = th - (CT)(a - LO);
    pre[0] = (CT)1;
    dpre[0] = (CT)0;
#pragma unroll
    for (int a = 1; a <= P; ++a) {
        pre[a] = pre[a - 1] * t[a - 1];
        dpre[a] = dpre[a - 1] * t[a - 1] + pre[a - 1];
    }
    suf[P] = (CT)1;
    dsuf[P] = (CT)0;
#pragma unroll
    for (int a = P - 1; a >= 0; --a) {
        suf[a] = suf[a + 1] * t[a + 1];
        dsuf[a] = dsuf[a + 1] * t[a + 1] + suf[a + 1];
    }
#pragma unroll
    for (int a = 0; a <= P; ++a) {
        double den = 1.0;
        for (int b = 0; b <= P; ++b)
            if (b != a) den *= (double)(a - b);
        dw[a] = (double)((CT)(1.0 / den) * (dpre[a] * suf[a] + pre[a] * dsuf[a])) * dxinv;
    }
}

// Extended source index g = c + k n of node e of a row (any integer e; the
// node is wrapped into the row with its period count kx).  The plan uses it
// for the two end nodes of every tile; the step kernel evaluates the same
// arithmetic inline, in batches.
__device__ inline int64_t node_locate(const double *x, int n, const MeshTab &tb,
                                      const RowShift &rs, int e, double &xt, int &cell)
{
    int kx = 0;
    if (e < 0) { e += n; kx = -1; }
    while (e >= n) { e -= n; kx += 1; }
    const double bsc = tb.scal[0], bx0 = tb.scal[2];
    const NodePos np = node_pos(x[e], rs, x[0], x[n], bsc, bx0, tb.nb);
    int c = cell_from_bucket(tb.bucket[np.b], tb.bnext[np.b], np.xt);
    if (np.xt >= tb.bnext[np.b].y) c = cell_walk(x, n, c, np.xt);
    xt = np.xt;
    cell = c;
    return (int64_t)c + (rs.kf0 + np.dk + kx) * (int64_t)n;
}

__device__ inline int64_t node_index(const double *x, int n, const MeshTab &tb,
                                     const RowShift &rs, double len, int e)
{
    double xt;
    int c;
    (void)len;
    return node_locate(x, n, tb, rs, e, xt, c);
}

// Non-uniform cells (MeshTab::nonu) among the extended source indices [a, b)
// of a periodic row of n cells.
__device__ inline int64_t nonu_count(const int32_t *pre, int n, int64_t a, int64_t b)
{
    auto upto = [&](int64_t i) {
        const int64_t k = i >= 0 ? i / n : -((-i + n - 1) / n);
        return k * (int64_t)pre[n] + pre[i - k * n];
    };
    return upto(b) - upto(a);
}

// ---- limited reconstructions of the bulk shift (Section 3.1, App. A) ----
//
// Both are handed to the shift as the cubic
//   ell(theta) = theta (A + theta (B + theta C)),
// the integral of q_c from the cell's left node to x_c + theta dx_c, so that
// ell(1) = M_c.

// PPM mesh weights of cell j from the sizes h_{j-1}, h_j, h_{j+1}, h_{j+2}
// (App. A with the neighbouring sizes summed, Colella & Woodward Eq. 1.6):
//   delta_j   = d1 (a_{j+1} - a_j) + d2 (a_j - a_{j-1})
//   a_{j+1/2} = a_j + e1 (a_{j+1} - a_j) + e2 delta_{j+1} + e3 delta_j
struct PpmW {
    double d1, d2, e1, e2, e3;
};

__device__ inline PpmW ppm_weights(double hm, double h0, double hp, double hpp)
{
    PpmW w;
    const double f = h0 / (hm + h0 + hp);
    w.d1 = f * (2.0 * hm + h0) / (hp + h0);
    w.d2 = f * (h0 + 2.0 * hp) / (hm + h0);
    const double inv = 1.0 / (hm + h0 + hp + hpp);
    const double w1 = 2.0 * hp * h0 / (h0 + hp) *
                      ((hm + h0) / (2.0 * h0 + hp) - (hpp + hp) / (2.0 * hp + h0));
    w.e1 = h0 / (h0 + hp) + w1 * inv;
    w.e2 = -h0 * (hm + h0) / (2.0 * h0 + hp) * inv;
    w.e3 = hp * (hp + hpp) / (h0 + 2.0 * hp) * inv;
    return w;
}

// Limited slope delta_j: zero at an extremum of the averages, otherwise at
// most twice either one-sided difference, with the unlimited slope's sign.
template <typename CT>
__device__ inline CT ppm_delta(CT qm, CT q0, CT qp, CT d1, CT d2)
{
    const CT up = qp - q0, dn = q0 - qm;
    const CT d = d1 * up + d2 * dn;
    const CT mag = fmin(fabs(d), (CT)2 * fmin(fabs(up), fabs(dn)));
    return up * dn <= (CT)0 ? (CT)0 : copysign(mag, d);
}

// Constrained parabola of a cell (average a, interface values L and R, size
// h) as the cubic ell(theta).  An extremum is flat; an overshooting side is
// pulled in until the parabola is monotone.
template <typename CT>
__device__ inline void ppm_cubic(CT a, CT L, CT R, CT h, CT &A, CT &B, CT &C)
{
    if ((R - a) * (a - L) <= (CT)0) {
        L = a;
        R = a;
    } else {
        const CT dq = R - L, qa = a - (CT)0.5 * (L + R);
        const CT d6 = dq * dq * (CT)(1.0 / 6.0);
        if (dq * qa > d6) L = (CT)3 * a - (CT)2 * R;
        else if (-d6 > dq * qa) R = (CT)3 * a - (CT)2 * L;
    }
    const CT q6 = (CT)6 * a - (CT)3 * (L + R);
    A = h * L;
    B = (CT)0.5 * h * (R - L + q6);
    C = h * q6 * (CT)(-1.0 / 3.0);
}

// PLM cell (mass M, size h, van Leer slope from the averages and the
// reciprocal centre gaps) as the cubic ell(theta) with C = 0.
template <typename CT>
__device__ inline void plm_cubic(CT qm, CT q0, CT qp, CT gm, CT gp, CT M, CT h,
                                 CT &A, CT &B)
{
    const CT dp = (qp - q0) * gp, dm = (q0 - qm) * gm;
    const CT sig = (dp * dm <= (CT)0) ? (CT)0 : harmonic2(dp, dm);
    const CT kap = (CT)0.5 * sig * h * h;
    A = M - kap;
    B = kap;
}

// Stencil half-width of a limited reconstruction (cells a side).
template <int R> struct LimHalo { static constexpr int lo = R == kReconPLM ? 1 : 2; };

// Partial integral of the limited reconstruction of cell c at xh, from global
// memory in FP64 (direct path).
template <typename TQ, int R>
__device__ __attribute__((noinline)) double lim_partial_global(const double *x,
                                                               const TQ *q, int n,
                                                               int c, double xh)
{
    constexpr int LO = LimHalo<R>::lo;
    double qv[2 * LO + 1], h[2 * LO + 2];
#pragma unroll
    for (int a = 0; a <= 2 * LO; ++a) qv[a] = (double)q[wrapi(c - LO + a, n)];
#pragma unroll
    for (int a = 0; a <= 2 * LO + 1; ++a) {
        const int m = wrapi(c - LO + a, n);
        h[a] = x[m + 1] - x[m];
    }
    const double h0 = h[LO];
    const double th = (xh - x[c]) / h0;
    double A, B, C = 0.0;
    if constexpr (R == kReconPLM) {
        // reciprocal centre gaps (c-1, c) and (c, c+1)
        const double gm = 2.0 / (h[0] + h[1]), gp = 2.0 / (h[1] + h[2]);
        plm_cubic<double>(qv[0], qv[1], qv[2], gm, gp, qv[1] * h0, h0, A, B);
    } else {
        // limited slopes of cells c-1, c, c+1, then the interfaces c-1/2, c+1/2
        double d[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const PpmW w = ppm_weights(h[k], h[k + 1], h[k + 2], h[k + 3]);
            d[k] = ppm_delta<double>(qv[k], qv[k + 1], qv[k + 2], w.d1, w.d2);
        }
        const PpmW wl = ppm_weights(h[0], h[1], h[2], h[3]);
        const PpmW wr = ppm_weights(h[1], h[2], h[3], h[4]);
        const double L = qv[1] + wl.e1 * (qv[2] - qv[1]) + wl.e2 * d[1] + wl.e3 * d[0];
        const double Rv = qv[2] + wr.e1 * (qv[3] - qv[2]) + wr.e2 * d[2] + wr.e3 * d[1];
        ppm_cubic<double>(qv[2], L, Rv, h0, A, B, C);
    }
    return th * (A + th * (B + th * C));
}

// The same for PPM with the shared mesh's FP64 weights tables (tb.ppmd: d1,
// d2, e1, e2, e3 of every cell, the values ppm_weights gives from the same
// cell sizes) instead of forming the weights of five cells per node.
template <typename TQ>
__device__ __attribute__((noinline)) double ppm_partial_tab(const MeshTab &tb, const double *x,
                                                            const TQ *q, int n, int c,
                                                            double xh)
{
    double qv[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) qv[a] = (double)q[wrapi(c - 2 + a, n)];
    const int cm = wrapi(c - 1, n), cp = wrapi(c + 1, n);
    const double *pw = tb.ppmd;
    const double h0 = x[c + 1] - x[c];
    const double th = (xh - x[c]) / h0;
    const double d0 = ppm_delta<double>(qv[0], qv[1], qv[2], pw[cm], pw[n + cm]);
    const double d1 = ppm_delta<double>(qv[1], qv[2], qv[3], pw[c], pw[n + c]);
    const double d2 = ppm_delta<double>(qv[2], qv[3], qv[4], pw[cp], pw[n + cp]);
    const double L = qv[1] + pw[2 * n + cm] * (qv[2] - qv[1]) + pw[3 * n + cm] * d1 +
                     pw[4 * n + cm] * d0;
    const double Rv = qv[2] + pw[2 * n + c] * (qv[3] - qv[2]) + pw[3 * n + c] * d2 +
                      pw[4 * n + c] * d1;
    double A, B, C;
    ppm_cubic<double>(qv[2], L, Rv, h0, A, B, C);
    return th * (A + th * (B + th * C));
}

} // namespace dev
} // namespace ram
