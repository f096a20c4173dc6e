// ram_step_shared.hip -- the RAM step on rows that share one mesh (gfx950).
//
// Same computation as k_step (bulk shift of Section 3, Steps 1-3, then the
// residual upwind step), specialised for a mesh shared by every row, which is
// the polar-disk layout: rows are radii, the shared mesh is the azimuthal one.
// What the specialisation buys:
//
//   * the source window of every tile is planned once per call (k_plan: the
//     shift of a row is the same at every step of a call), so a tile reads
//     its window bounds with one scalar load and issues the window, residual-
//     velocity and mesh loads before any search;
//   * the source cell of a shifted node takes one bucket record (lower-bound
//     cell and the next two nodes) and the stencil one cell record (x_c, 1/dx_c,
//     normalised node offsets, reciprocal Lagrange denominators): two
//     dependent loads after the node itself;
//   * tiles away from the row seam skip all periodic index wrapping.
#include "ram_device.h"

#include <type_traits>

namespace ram {
namespace {

using namespace dev;

constexpr int kWinSh = 1536;                    // LDS window capacity, cells
constexpr int kWinRegs = kWinSh / kBlock;       // window cells per thread

template <typename M, typename A, typename CT>
struct ShLds {
    static constexpr size_t win = sizeof(M) * kWinSh + sizeof(A) * (kWinSh + 1);
    static constexpr size_t res = 2 * sizeof(CT) * kStepNodes;
    static constexpr size_t uni = win > res ? win : res;
};

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

// Source cell of xh: the bucket's lower-bound cell plus the nodes passed
// (two are in the record; more only on meshes finer than the buckets).
__device__ inline int cell_of(const double *x, int n, const MeshTab &tb,
                              double bsc, double xh)
{
    int b = (int)((xh - x[0]) * bsc);
    b = min(max(b, 0), tb.nb - 1);
    int c = tb.bucket[b];
    const double2 nx = tb.bnext[b];
    c += (xh >= nx.x) ? 1 : 0;
    if (xh >= nx.y) {
        c += 1;
        while (c + 1 < n && x[c + 1] <= xh) ++c;
    }
    return c;
}

// Shifted node e (any integer; e is wrapped into the row with its period
// count) -> extended source index g and the Lagrange weights of its stencil.
template <typename WT, int P>
__device__ inline int64_t node_eval(const double *x, int n, const MeshTab &tb,
                                    double bsc, double invlen, double len,
                                    double s, double xe, int kx, WT *w)
{
    const double xt = xe - s;
    const double kf = floor((xt - x[0]) * invlen);
    double xh = xt - kf * len;
    int64_t k = (int64_t)kf;
    if (xh >= x[n]) { xh -= len; k += 1; }
    else if (xh < x[0]) { xh += len; k -= 1; }
    const int c = cell_of(x, n, tb, bsc, xh);
    const CellRec<WT> &r = RecT<WT>::get(tb)[c];
    const WT th = (WT)((xh - r.xc) * r.dxinv);
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
    return (int64_t)c + (k + kx) * (int64_t)n;
}

// Window plan: extended source index of each tile's first node minus lo, and
// the window length (or -1 when it exceeds the LDS capacity).
template <int P>
__global__ __launch_bounds__(256) void k_plan(StepArgs a, int64_t *wlo_out,
                                              int32_t *w_out)
{
    constexpr int LO = (P - 1) / 2;
    const int64_t tile = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const Rows &R = a.rows;
    if (tile >= R.n_tiles) return;
    const int n = (int)R.n_cols;
    const int64_t tpr = (n + R.tile - 1) / R.tile;
    const int64_t row = tile / tpr;
    const int i0 = (int)(tile - row * tpr) * R.tile;
    const int H = a.dv ? 2 : 0;
    const int nd = min(R.tile, n - i0);
    const double *x = R.edges;
    const double len = x[n] - x[0];
    const double s = a.v0[row] * a.dt;
    const double bsc = R.tab.scal[0], invlen = R.tab.scal[1];
    int64_t g[2];
    for (int side = 0; side < 2; ++side) {
        int e = side == 0 ? i0 - H : i0 + nd + H;
        int kx = 0;
        if (e < 0) { e += n; kx = -1; }
        while (e >= n) { e -= n; kx += 1; }
        float w[P + 1];
        g[side] = node_eval<float, P>(x, n, R.tab, bsc, invlen, len, s, x[e], kx, w);
    }
    const int64_t wide = g[1] - g[0] + P;
    wlo_out[tile] = g[0] - LO;
    w_out[tile] = (wide >= P && wide <= kWinSh) ? (int32_t)wide : -1;
}

// Periodic index for j in [-n, 2n).
__device__ inline int wrap1(int j, int n)
{
    return j < 0 ? j + n : (j >= n ? j - n : j);
}

template <typename TQ, int P, int S, int H>
__global__ __launch_bounds__(kBlock) void k_step_sh(StepArgs a)
{
    using AC = Acc<S>;
    using M = typename AC::M;
    using A = typename AC::A;
    using CT = TQ;                       // arithmetic after the prefix sums
    using L = ShLds<M, A, CT>;
    constexpr int LO = (P - 1) / 2;
    constexpr int NI = kItems;
    constexpr int WCAP = kWinSh;

    __shared__ int sjc[kStepNodes];      // window index of each node's cell
    __shared__ CT sell[kStepNodes];      // partial integral C~(xh) - C(c)
    __shared__ A swt[kBlock / 64];
    __shared__ __attribute__((aligned(16))) unsigned char su[L::uni];
    __shared__ int s_flag;
    M *sm = (M *)su;                                 // window masses
    A *sp = (A *)(su + sizeof(M) * WCAP);            // exclusive prefix
    int64_t *sg = (int64_t *)su;                     // direct path: node indices
    CT *sq = (CT *)su;                               // shifted state
    CT *sf = sq + kStepNodes;                        // face fluxes

    const Rows &R = a.rows;
    const MeshTab &tb = R.tab;
    const int n = (int)R.n_cols;
    const int tpr = (n + R.tile - 1) / R.tile;
    const int row = (int)(blockIdx.x / (unsigned)tpr);
    const int i0 = ((int)blockIdx.x - row * tpr) * R.tile;
    const int nd = min(R.tile, n - i0);
    const int NC = nd + 2 * H;
    const int NE = NC + 1;
    const bool inner = (i0 - H >= 0) && (i0 + nd + H < n);
    const double *x = R.edges;
    const int64_t qoff = (int64_t)row * n;
    const TQ *q = (const TQ *)a.q_in + qoff;
    TQ *qo = (TQ *)a.q_out + qoff;
    TQ *qmid = a.q_mid ? (TQ *)a.q_mid + qoff : nullptr;
    const double s = a.v0[row] * a.dt;
    const double len = x[n] - x[0];
    const double bsc = tb.scal[0], invlen = tb.scal[1];
    const int64_t wlo = a.plan_wlo[blockIdx.x];
    const int W = a.plan_w[blockIdx.x];
    const int t = threadIdx.x;

    // ---- loads that do not depend on the search, issued first ------------
    double xe[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int ei = t + k * kBlock;
        const int e = i0 - H + ei;
        xe[k] = ei < NE ? x[inner ? e : wrap1(e, n)] : 0.0;
    }
    // window start inside the row: wlo mod n, without a 64-bit division in
    // the common case of a window at most one period away
    int base = 0;
    if (W > 0) {
        const int64_t kk = wlo >= 0 ? wlo / n : -((-wlo + n - 1) / n);
        base = (int)(wlo - kk * n);
    }
    const bool wsmall = W + base <= 2 * n;
    M wq[kWinRegs], wd[kWinRegs];
#pragma unroll
    for (int r = 0; r < kWinRegs; ++r) {
        const int j = t + r * kBlock;
        if (j < W) {
            int mm = base + j;
            if (wsmall) mm = mm >= n ? mm - n : mm;
            else mm = wrap_small(mm, n);
            wq[r] = (M)q[mm];
            wd[r] = TabT<M>::dx(tb)[mm];
        }
    }

    // ---- (A) shifted nodes: source index and stencil weights -------------
    int64_t g[NI];
    CT w[NI][P + 1];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int ei = t + k * kBlock;
        g[k] = 0;
        if (ei < NE) {
            const int e = i0 - H + ei;
            const int kx = e < 0 ? -1 : (e >= n ? 1 : 0);
            g[k] = node_eval<CT, P>(x, n, tb, bsc, invlen, len, s, xe[k], kx, w[k]);
            const int64_t jc = g[k] - wlo;
            ok = ok && jc >= LO && jc + P - LO <= W;
        }
    }
    if (t == 0) s_flag = W > 0 ? 1 : 0;
    __syncthreads();
    if (!ok) s_flag = 0;
    // ---- (B) window masses and the block scan ------------------------------
#pragma unroll
    for (int r = 0; r < kWinRegs; ++r) {
        const int j = t + r * kBlock;
        if (j < W) sm[j] = wq[r] * wd[r];
    }
    __syncthreads();
    const bool windowed = s_flag != 0;
    if (windowed) {
        const int per = (W + kBlock - 1) / kBlock;
        const int j0 = min(W, t * per);
        const int j1 = min(W, j0 + per);
        M mine[kWinRegs];
        A run = AC::zero();
#pragma unroll
        for (int r = 0; r < kWinRegs; ++r) {
            if (j0 + r < j1) {
                mine[r] = sm[j0 + r];
                run = AC::add(run, mine[r]);
            }
        }
        A total;
        A acc = block_exscan_dpp<AC>(run, swt, total);
#pragma unroll
        for (int r = 0; r < kWinRegs; ++r) {
            if (j0 + r < j1) {
                sp[j0 + r] = acc;
                acc = AC::add(acc, mine[r]);
            }
        }
        if (t == 0) sp[W] = total;
        __syncthreads();
        // ---- (C) partial integrals of the interpolated cumulative ----------
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int ei = t + k * kBlock;
            if (ei < NE) {
                const int jc = (int)(g[k] - wlo);
                const A pc = sp[jc];
                CT ell = (CT)0;
#pragma unroll
                for (int b = 0; b <= P; ++b)
                    if (b != LO) ell += w[k][b] * (CT)AC::diff(sp[jc - LO + b], pc);
                sell[ei] = ell;
                sjc[ei] = jc;
            }
        }
    } else {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int ei = t + k * kBlock;
            if (ei < NE) {
                sg[ei] = g[k];
                sell[ei] = (CT)direct_partial<TQ, P>(x, q, n, len, s, invlen,
                                                     i0 - H + ei, g[k]);
            }
        }
    }

    // residual inputs, fetched while the partial integrals settle
    const CT dt = (CT)a.dt;
    TQ dvr[NI];
    CT dxl[NI], dxr[NI], h0[NI], h1[NI], h2[NI], dxi[NI];
    if (H) {
        const TQ *dv = (const TQ *)a.dv + qoff;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int u = t + k * kBlock;
            if (u < nd + 1) {                        // face f = i0+u
                const int f = i0 + u;
                const int fm = inner ? f - 1 : wrap1(f - 1, n);
                const int fp = inner ? f : wrap1(f, n);
                const int fmm = inner ? f - 2 : wrap1(f - 2, n);
                const int fpp = inner ? f + 1 : wrap1(f + 1, n);
                dvr[k] = dv[fp];
                dxl[k] = TabT<CT>::dx(tb)[fm];
                dxr[k] = TabT<CT>::dx(tb)[fp];
                h0[k] = TabT<CT>::hinv(tb)[fmm];     // gap (f-2, f-1)
                h1[k] = TabT<CT>::hinv(tb)[fm];      // gap (f-1, f)
                h2[k] = TabT<CT>::hinv(tb)[fp];      // gap (f, f+1)
                (void)fpp;
            }
            if (u < nd) dxi[k] = TabT<CT>::dxinv(tb)[i0 + u];
        }
    }
    __syncthreads();

    // ---- (D) destination masses, Step 3 ------------------------------------
    CT qs[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int ci = t + k * kBlock;
        qs[k] = (CT)0;
        if (ci < NC) {
            const int c0 = i0 - H + ci;
            const int cell = inner ? c0 : wrap1(c0, n);
            CT mp;
            if (windowed) {
                const int ja = sjc[ci], jb = sjc[ci + 1];
                const CT whole = (jb - ja == 1) ? (CT)sm[ja] : (CT)AC::diff(sp[jb], sp[ja]);
                mp = whole + (sell[ci + 1] - sell[ci]);
            } else {
                mp = (CT)(direct_whole<TQ>(x, q, n, sg[ci], sg[ci + 1]) +
                          ((double)sell[ci + 1] - (double)sell[ci]));
            }
            qs[k] = mp * TabT<CT>::dxinv(tb)[cell];
            if (H == 0) qo[cell] = (TQ)qs[k];
            else if (qmid && ci >= H && ci < H + nd) qmid[cell] = (TQ)qs[k];
        }
    }
    if (H == 0) return;
    __syncthreads();   // the window bytes become the residual's arrays
#pragma unroll
    for (int k = 0; k < NI; ++k)
        if (t + k * kBlock < NC) sq[t + k * kBlock] = qs[k];
    __syncthreads();

    // ---- (E) fluxes on faces i0 .. i0+nd, with the upwind cell's slope -----
    // face i0+u lies between cells i0+u-1 (state index u+1) and i0+u (u+2)
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int u = t + k * kBlock;
        if (u < nd + 1) {
            const CT v = (CT)dvr[k];
            const bool up = v >= (CT)0;
            const int c = up ? u + 1 : u + 2;             // upwind cell, state index
            const CT qm = sq[c - 1], q0 = sq[c], qp = sq[c + 1];
            const CT hpl = up ? h1[k] : h2[k];
            const CT hmi = up ? h0[k] : h1[k];
            const CT dp = (qp - q0) * hpl;
            const CT dm = (q0 - qm) * hmi;
            const CT sig = (dp * dm <= (CT)0) ? (CT)0 : harmonic2(dp, dm);
            const CT half = up ? (CT)0.5 * (dxl[k] - v * dt) : (CT)-0.5 * (dxr[k] + v * dt);
            sf[u] = v * (q0 + sig * half);
        }
    }
    __syncthreads();
    // ---- (F) conservative update --------------------------------------------
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int u = t + k * kBlock;
        if (u < nd) qo[i0 + u] = (TQ)(sq[u + 2] - dt * (sf[u + 1] - sf[u]) * dxi[k]);
    }
}

template <typename TQ, int P, int H>
hipError_t step_sh_h(const StepArgs &a, int scan, hipStream_t st)
{
    const dim3 g((unsigned)a.rows.n_tiles), b(kBlock);
    switch (scan) {
    case kScanF64: hipLaunchKernelGGL((k_step_sh<TQ, P, kScanF64, H>), g, b, 0, st, a); break;
    case kScanTwoSum: hipLaunchKernelGGL((k_step_sh<TQ, P, kScanTwoSum, H>), g, b, 0, st, a); break;
    default: hipLaunchKernelGGL((k_step_sh<TQ, P, kScanF32, H>), g, b, 0, st, a); break;
    }
    return hipGetLastError();
}

template <typename TQ, int P>
hipError_t step_sh_scan(const StepArgs &a, int scan, hipStream_t st)
{
    if (a.dv) return step_sh_h<TQ, P, 2>(a, scan, st);
    return step_sh_h<TQ, P, 0>(a, scan, st);
}

template <typename TQ>
hipError_t step_sh_order(const StepArgs &a, int scan, int order, hipStream_t st)
{
    switch (order) {
    case 1: return step_sh_scan<TQ, 1>(a, scan, st);
    case 3: return step_sh_scan<TQ, 3>(a, scan, st);
    default: return step_sh_scan<TQ, 5>(a, scan, st);
    }
}

} // namespace

hipError_t launch_plan(const StepArgs &a, int order, int64_t *wlo, int32_t *w,
                       hipStream_t stream)
{
    const unsigned grid = (unsigned)((a.rows.n_tiles + 255) / 256);
    switch (order) {
    case 1: hipLaunchKernelGGL(k_plan<1>, dim3(grid), dim3(256), 0, stream, a, wlo, w); break;
    case 3: hipLaunchKernelGGL(k_plan<3>, dim3(grid), dim3(256), 0, stream, a, wlo, w); break;
    default: hipLaunchKernelGGL(k_plan<5>, dim3(grid), dim3(256), 0, stream, a, wlo, w); break;
    }
    return hipGetLastError();
}

hipError_t launch_step_shared(const StepArgs &a, bool f64, int scan, int order,
                              hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    if (f64) return step_sh_order<double>(a, kScanF64, order, stream);
    return step_sh_order<float>(a, scan, order, stream);
}

} // namespace ram
