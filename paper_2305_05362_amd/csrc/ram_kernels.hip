// ram_kernels.hip -- forward HIP kernels of the RAM advection step (gfx950).
//
// Rows are independent periodic lines (paper Section 2).  Every kernel works
// on tiles of consecutive cells of one row, one workgroup (kBlock threads =
// four wave64) per tile, with row-major coalesced HBM access.
//
//   k_step       bulk shift (Section 3, Steps 1-3), optionally fused with the
//                residual upwind step (Eq. splitting_second).  Per tile, with
//                one shifted node per thread:
//                (A) x~ = x - v0 dt is wrapped into the period and its source
//                    cell found (Eq. condition_p) -- through the mesh's bucket
//                    index when the mesh is shared, by binary search when
//                    every row has its own mesh; the Lagrange weights of the
//                    node's degree-p stencil stay in registers;
//                (B) the tile's source window is staged in LDS as cell masses
//                    M = Q dx (Eq. Qmass_i) and turned into an exclusive prefix
//                    (the cumulative integral) by a block scan in FP64,
//                    compensated FP32 or plain FP32;
//                (C) each node's partial integral of the reconstruction is the
//                    Lagrange interpolant of the window cumulative;
//                (D) destination mass = whole source cells in between + two
//                    partial integrals (Eq. mass_shift_algo), times 1/dx
//                    (Eq. step3);
//                (E-G) fused residual: van Leer slopes (Section 3.1), upwind
//                    swept-interval face fluxes and the conservative update,
//                    on the shifted state still in LDS (two-cell halo a side).
//                Windows wider than the LDS capacity take a direct path that
//                sums the masses from global memory.
//   k_residual   the residual step alone.
//   k_mesh_prep  mesh-only tables of a shared mesh.
//   k_tiles_prep tile table of a ragged batch.
#include "ram_device.h"

#include <algorithm>

#include <type_traits>

namespace ram {
namespace {

using namespace dev;


// Lagrange weights of the stencil nodes c-LO .. c-LO+P at xh, in WT.
// Shared meshes use the per-cell stencil table: node offsets and reciprocal
// denominators in units of dx_c, so only theta = (xh - x_c)/dx_c is formed in
// FP64 and every factor is O(1).  Per-row meshes form the weights from the
// nodes directly.
template <typename WT, int P>
__device__ inline void stencil_weights(const double *x, int n, double len,
                                       const Rows &R, int c, double xh, WT *w)
{
    constexpr int LO = (P - 1) / 2;
    if (!R.has_tab) {
        double X[P + 1], wd[P + 1];
#pragma unroll
        for (int a = 0; a <= P; ++a) X[a] = node_x(x, n, len, c - LO + a);
        lagrange_weights<P>(xh, X, wd);
#pragma unroll
        for (int a = 0; a <= P; ++a) w[a] = (WT)wd[a];
        return;
    }
    const WT *st;
    if constexpr (std::is_same<WT, double>::value) st = R.tab.stc + c * (2 * (P + 1));
    else st = R.tab.stcf + c * (2 * (P + 1));
    const WT th = (WT)((xh - x[c]) * R.tab.dxinv[c]);
    WT t[P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) t[a] = th - st[a];
    // products of all t but one, from prefix and suffix products
    WT pre[P + 1], suf[P + 1];
    pre[0] = (WT)1;
#pragma unroll
    for (int a = 1; a <= P; ++a) pre[a] = pre[a - 1] * t[a - 1];
    suf[P] = (WT)1;
#pragma unroll
    for (int a = P - 1; a >= 0; --a) suf[a] = suf[a + 1] * t[a + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) w[a] = st[P + 1 + a] * (pre[a] * suf[a]);
}


// ---------------------------------------------------------------------------
// bulk shift, optionally fused with the residual step
// ---------------------------------------------------------------------------

constexpr int kWinStep = 1536;      // LDS window capacity of k_step, cells

// LDS of k_step.  The window (masses + prefix) is dead once the destination
// masses are formed, so the shifted state, slopes and fluxes of the fused
// residual reuse its bytes; the node indices of the exact-window path use
// them before the window is loaded.
template <typename M, typename A, typename D, typename CT>
struct StepLds {
    static constexpr size_t win = sizeof(M) * kWinStep + sizeof(A) * (kWinStep + 1);
    static constexpr size_t res = 3 * sizeof(CT) * kStepNodes;
    static constexpr size_t nodes = sizeof(int64_t) * kStepNodes;
    // per-row meshes, before the window is loaded: the window's node
    // coordinates (FP64) and their periods relative to the first
    static constexpr size_t stage = (sizeof(double) + sizeof(short)) * (kWinStep + 1);
    static constexpr size_t uni0 = win > res ? win : res;
    static constexpr size_t uni1 = uni0 > nodes ? uni0 : nodes;
    static constexpr size_t uni = uni1 > stage ? uni1 : stage;
};

template <typename TQ, int P, int S>
__global__ __launch_bounds__(kBlock) void k_step(StepArgs a)
{
    using AC = Acc<S>;
    using M = typename AC::M;
    using A = typename AC::A;
    using D = typename std::conditional<std::is_same<TQ, double>::value, double,
                                        typename AC::D>::type;
    using CT = TQ;                     // arithmetic type of the state updates
    using L = StepLds<M, A, D, CT>;
    constexpr int LO = (P - 1) / 2;
    constexpr int NI = kItems;

    __shared__ int sjc[kStepNodes];    // window index of each node's cell
    __shared__ D sell[kStepNodes];     // partial integral C~(xh) - C(c)
    __shared__ A swt[kBlock / 64];
    __shared__ __attribute__((aligned(16))) unsigned char su[L::uni];
    __shared__ int s_flag;             // 1: window path usable
    __shared__ long long s_wlo, s_whi;
    M *sm = (M *)su;                                     // window masses
    A *sp = (A *)(su + sizeof(M) * kWinStep);            // exclusive prefix
    int64_t *sg = (int64_t *)su;                         // node indices
    CT *sq = (CT *)su;                                   // shifted state
    CT *ssig = sq + kStepNodes;                          // van Leer slopes
    CT *sf = ssig + kStepNodes;                          // face fluxes

    const Rows &R = a.rows;
    Tile ti;
    if (!get_tile(R, blockIdx.x, ti)) return;
    const int n = ti.n;
    if (n < P + 1) return;
    const int H = a.dv ? 2 : 0;                 // residual halo
    const int i0 = ti.i0;
    const int nd = min(R.tile, n - i0);         // cells this tile writes
    const int NC = nd + 2 * H;                  // shifted cells
    const int NE = NC + 1;                      // shifted nodes (<= kStepNodes)
    const double *x = ti.x;
    const TQ *q = (const TQ *)a.q_in + ti.qoff;
    TQ *qo = (TQ *)a.q_out + ti.qoff;
    TQ *qmid = a.q_mid ? (TQ *)a.q_mid + ti.qoff : nullptr;
    const double s = a.v0[ti.row] * a.dt;
    const double len = x[n] - x[0];
    const int t = threadIdx.x;
    const bool tab = R.has_tab != 0;
    const double bsc = tab ? R.tab.scal[0] : 0.0;
    const double invlen = tab ? R.tab.scal[1] : 1.0 / len;

    // residual velocity of the faces this thread will need, fetched early
    const TQ *dv = H ? (const TQ *)a.dv + ti.qoff : nullptr;
    TQ dvr[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int f = t + k * kBlock;
        dvr[k] = (H && f < nd + 1) ? dv[wrap_small(i0 + f, n)] : (TQ)0;
    }

    // conservative window from the bucket index (shared mesh): the first and
    // last shifted nodes' buckets, widened by one bucket and the stencil
    if (tab && t < 2) {
        int e = t == 0 ? i0 - H : i0 - H + NE - 1;
        int kx = 0;
        if (e < 0) { e += n; kx = -1; }
        while (e >= n) { e -= n; kx += 1; }
        double xh;
        int64_t k;
        shifted_node_inv(x, n, s, e, invlen, len, xh, k);
        int b = (int)((xh - x[0]) * bsc);
        b = min(max(b, 0), R.tab.nb - 1);
        int64_t gb;
        if (t == 0) {
            gb = (int64_t)R.tab.bucket[max(b - 1, 0)] + (k + kx) * (int64_t)n;
            s_wlo = gb - LO - 1;
        } else {
            gb = (int64_t)R.tab.bucket[min(b + 2, R.tab.nb - 1)] + (k + kx) * (int64_t)n;
            if (b + 2 >= R.tab.nb) gb = (int64_t)n + (k + kx) * (int64_t)n;
            s_whi = gb - LO + P + 2;
        }
    }
    if (t == 0) s_flag = 1;

    // Per-row meshes: the tile's window from its two end nodes (global
    // searches by two threads), then the window's node coordinates staged in
    // LDS, where every node finds its cell and its stencil nodes.
    double *sxs = (double *)su;                          // window nodes (FP64)
    short *skq = (short *)(su + sizeof(double) * (kWinStep + 1));   // periods
    if (!tab) {
        if (t < 2) {
            int e = t == 0 ? i0 - H : i0 - H + NE - 1;
            int kx = 0;
            if (e < 0) { e += n; kx = -1; }
            while (e >= n) { e -= n; kx += 1; }
            double xh;
            int64_t k;
            shifted_node_inv(x, n, s, e, invlen, len, xh, k);
            const int64_t gg = (int64_t)find_cell(x, n, xh) + (k + kx) * (int64_t)n;
            if (t == 0) s_wlo = gg - LO;
            else s_whi = gg - LO + P;
        }
        __syncthreads();
    }
    int64_t pwlo = 0, pk0 = 0;
    bool stage = false;
    int pW = 0;
    if (!tab) {
        pwlo = s_wlo;
        pk0 = pwlo >= 0 ? pwlo / n : -((-pwlo + n - 1) / n);   // period of wlo
        stage = s_whi - pwlo >= P && s_whi - pwlo <= kWinStep;
        pW = stage ? (int)(s_whi - pwlo) : 0;
    }
    if (stage) {
        const int pbase = (int)(pwlo - pk0 * n);
        for (int j = t; j <= pW; j += kBlock) {
            int m = pbase + j, kq = 0;
            while (m >= n) { m -= n; ++kq; }
            sxs[j] = x[m];
            skq[j] = (short)kq;
        }
        __syncthreads();
    }

    // (A) shifted nodes e = i0 - H + t + k kBlock: cell and stencil weights
    int64_t g[NI];
    TQ w[NI][P + 1];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int ei = t + k * kBlock;
        g[k] = 0;
        if (ei < NE) {
            int e = i0 - H + ei;
            int kx = 0;
            if (e < 0) { e += n; kx = -1; }
            while (e >= n) { e -= n; kx += 1; }
            double xh;
            int64_t kk;
            shifted_node_inv(x, n, s, e, invlen, len, xh, kk);
            bool done = false;
            if (stage) {
                // the last window cell whose left node is at or below the
                // shifted node, comparing (period, coordinate) pairs exactly
                const int dk = (int)(kk + kx - pk0);
                auto le = [&](int j) {
                    const int kj = skq[j];
                    return kj < dk || (kj == dk && sxs[j] <= xh);
                };
                int lo = 0, hi = pW + 1;
                if (le(0)) {
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (le(mid)) lo = mid;
                        else hi = mid;
                    }
                    if (lo - LO >= 0 && lo - LO + P <= pW) {
                        g[k] = pwlo + lo;
                        const double xc = sxs[lo];
                        const int kc = skq[lo];
                        double X[P + 1];
#pragma unroll
                        for (int b = 0; b <= P; ++b) {
                            const int jb = lo - LO + b;
                            X[b] = (sxs[jb] - xc) + (double)(skq[jb] - kc) * len;
                        }
                        lagrange_rel<TQ, P>(xh - xc, X, w[k]);
                        done = true;
                    }
                }
            }
            if (!done) {
                const int c = tab ? find_cell_tab(x, n, R.tab, bsc, xh) : find_cell(x, n, xh);
                g[k] = (int64_t)c + (kk + kx) * (int64_t)n;
                stencil_weights<TQ, P>(x, n, len, R, c, xh, w[k]);
            }
        }
    }
    __syncthreads();
    const int64_t wlo = s_wlo;
    const int64_t wide = s_whi - s_wlo;
    // every node's stencil must lie inside the window (else: direct path)
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        if (t + k * kBlock < NE) {
            const int64_t jc = g[k] - wlo;
            if (jc < LO || jc + P - LO > wide) s_flag = 0;
        }
    }
    if (wide > kWinStep || wide < P) s_flag = 0;
    __syncthreads();
    const bool windowed = s_flag != 0;

    if (windowed) {
        const int W = (int)wide;
        const int base = wrapi(wlo, n);
        // (B) window masses and the block scan into the cumulative
        for (int j = t; j < W; j += kBlock) {
            const int mm = wrap_small(base + j, n);
            if (tab) sm[j] = (M)q[mm] * TabT<M>::dx(R.tab)[mm];
            else sm[j] = AC::template mass<TQ>(q[mm], x[mm + 1] - x[mm]);
        }
        __syncthreads();
        const int per = (W + kBlock - 1) / kBlock;
        const int j0 = min(W, t * per);
        const int j1 = min(W, j0 + per);
        A run = AC::zero();
        for (int j = j0; j < j1; ++j) run = AC::add(run, sm[j]);
        A total;
        A acc = block_exscan_dpp<AC>(run, swt, total);
        for (int j = j0; j < j1; ++j) {
            sp[j] = acc;
            acc = AC::add(acc, sm[j]);
        }
        if (t == 0) sp[W] = total;
        __syncthreads();
        // (C) partial integrals from the interpolated window cumulative
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int ei = t + k * kBlock;
            if (ei < NE) {
                const int jc = (int)(g[k] - wlo);
                const A pc = sp[jc];
                D ell = (D)0;
#pragma unroll
                for (int b = 0; b <= P; ++b)
                    if (b != LO) ell += (D)w[k][b] * (D)AC::diff(sp[jc - LO + b], pc);
                sell[ei] = ell;
                sjc[ei] = jc;
            }
        }
    } else {
        // direct path: masses summed from global memory in FP64
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int ei = t + k * kBlock;
            if (ei < NE) {
                sg[ei] = g[k];
                sell[ei] = (D)direct_partial<TQ, P>(x, q, n, len, s, invlen,
                                                    i0 - H + ei, g[k]);
            }
        }
    }
    __syncthreads();

    // (D) destination masses and Step 3
    CT qs[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int ci = t + k * kBlock;
        qs[k] = (CT)0;
        if (ci < NC) {
            const int cell = wrap_small(i0 - H + ci, n);
            D mp;
            if (windowed) {
                const int ja = sjc[ci], jb = sjc[ci + 1];
                const D whole = (jb - ja == 1) ? (D)sm[ja] : (D)AC::diff(sp[jb], sp[ja]);
                mp = whole + (sell[ci + 1] - sell[ci]);
            } else {
                const double wh = direct_whole<TQ>(x, q, n, sg[ci], sg[ci + 1]);
                mp = (D)(wh + ((double)sell[ci + 1] - (double)sell[ci]));
            }
            if (tab) qs[k] = (CT)(mp * (D)TabT<D>::dxinv(R.tab)[cell]);
            else qs[k] = (CT)(mp / (D)(x[cell + 1] - x[cell]));
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

    // (E) van Leer slopes of cells i0-1 .. i0+nd (state index +1)
    const CT dt = (CT)a.dt;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int u = t + k * kBlock;
        if (u < nd + 2) {
            const int cm = wrap_small(i0 - 2 + u, n);
            const int c0 = wrap_small(i0 - 1 + u, n);
            CT hp, hm;
            if (tab) {
                hp = TabT<CT>::hinv(R.tab)[c0];
                hm = TabT<CT>::hinv(R.tab)[cm];
            } else {
                hp = (CT)(1.0 / centre_gap(x, n, len, c0));
                hm = (CT)(1.0 / centre_gap(x, n, len, cm));
            }
            const CT dp = (sq[u + 2] - sq[u + 1]) * hp;
            const CT dm = (sq[u + 1] - sq[u]) * hm;
            ssig[u] = (dp * dm <= (CT)0) ? (CT)0 : harmonic2(dp, dm);
        }
    }
    __syncthreads();
    // (F) fluxes on faces i0 .. i0+nd (face f between cells f-1 and f)
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int u = t + k * kBlock;
        if (u < nd + 1) {
            const int f = wrap_small(i0 + u, n);
            const CT v = (CT)dvr[k];
            CT qf;
            if (v >= (CT)0) {
                const int c = wrap_small(i0 + u - 1, n);
                const CT dxu = tab ? TabT<CT>::dx(R.tab)[c] : (CT)(x[c + 1] - x[c]);
                qf = sq[u + 1] + (CT)0.5 * ssig[u] * (dxu - v * dt);
            } else {
                const CT dxu = tab ? TabT<CT>::dx(R.tab)[f] : (CT)(x[f + 1] - x[f]);
                qf = sq[u + 2] - (CT)0.5 * ssig[u + 1] * (dxu + v * dt);
            }
            sf[u] = v * qf;
        }
    }
    __syncthreads();
    // (G) conservative update of the tile's own cells
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int u = t + k * kBlock;
        if (u < nd) {
            const int i = i0 + u;
            const CT inv = tab ? TabT<CT>::dxinv(R.tab)[i] : (CT)(1.0 / (x[i + 1] - x[i]));
            qo[i] = (TQ)(sq[u + 2] - dt * (sf[u + 1] - sf[u]) * inv);
        }
    }
}

// ---------------------------------------------------------------------------
// residual step alone
// ---------------------------------------------------------------------------

template <typename TQ>
__global__ __launch_bounds__(kBlock) void k_residual(ResidualArgs a)
{
    // Staged once (index j <-> cell i0-2+j, and face i0-2+j between cells
    // j-1 and j): the state, the face velocities and the mesh data (dx,
    // 1/centre gap, 1/dx); every lane issues its loads before the first LDS
    // store.  Then one face per lane (fluxes on faces i0 .. i0+nd, with the
    // upwind cell's van Leer slope) and one cell per lane (the conservative
    // update), lane-consecutive in LDS, so no access conflicts on a bank.
    using CT = TQ;
    using CT2 = typename TabT<CT>::T2;
    constexpr int NP = kStepNodes + 8;
    __shared__ __attribute__((aligned(16))) CT sq[NP];
    __shared__ __attribute__((aligned(16))) CT sdx[NP];
    __shared__ __attribute__((aligned(16))) CT shv[NP];
    __shared__ __attribute__((aligned(16))) CT sdi[NP];
    __shared__ __attribute__((aligned(16))) CT sf[NP];

    const Rows &R = a.rows;
    Tile ti;
    if (!get_tile(R, blockIdx.x, ti)) return;
    const int n = ti.n;
    const double *x = ti.x;
    const TQ *q = (const TQ *)a.q_in + ti.qoff;
    const TQ *dv = (const TQ *)a.dv + ti.qoff;
    TQ *qo = (TQ *)a.q_out + ti.qoff;
    const CT dt = (CT)a.dt;
    const int i0 = ti.i0;
    const int nd = min(R.tile, n - i0);
    const bool tab = R.has_tab != 0;
    const bool inner = (i0 - 2 >= 0) && (i0 + nd + 2 < n);
    const int t = threadIdx.x;
    const double len = x[n] - x[0];
    CT vq[kItems], vv[kItems], vdi[kItems];
    CT2 vr[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int j = min(t + k * kBlock, nd + 3);
        const int c = inner ? i0 - 2 + j : wrap_small(i0 - 2 + j, n);
        vq[k] = (CT)q[c];
        vv[k] = (CT)dv[c];
        if (tab) {
            vr[k] = TabT<CT>::rr(R.tab)[c];
            vdi[k] = TabT<CT>::dxinv(R.tab)[c];
        }
    }
    CT vd[kItems];                       // face velocity of the face j (cell j's left)
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int j = t + k * kBlock;
        if (j < nd + 4) {
            const int c = inner ? i0 - 2 + j : wrap_small(i0 - 2 + j, n);
            if (!tab) {
                const double d = x[c + 1] - x[c];
                vr[k].x = (CT)d;
                vr[k].y = (CT)(1.0 / centre_gap(x, n, len, c));
                vdi[k] = (CT)(1.0 / d);
            }
            sq[j] = vq[k];
            sdx[j] = vr[k].x;
            shv[j] = vr[k].y;
            sdi[j] = vdi[k];
        }
        vd[k] = vv[k];
    }
    __syncthreads();
    // face f (0 .. nd) lies between cells f+1 and f+2; its velocity is the
    // one staged with cell f+2
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int f = t + k * kBlock - 2;
        if (f >= 0 && f <= nd) {
            const CT v = vd[k];
            const bool up = v >= (CT)0;
            const int c = up ? f + 1 : f + 2;             // upwind cell
            const CT qm = sq[c - 1], q0 = sq[c], qp = sq[c + 1];
            const CT dp = (qp - q0) * shv[c];
            const CT dm = (q0 - qm) * shv[c - 1];
            const CT sg = (dp * dm <= (CT)0) ? (CT)0 : harmonic2(dp, dm);
            const CT qf = up ? q0 + (CT)0.5 * sg * (sdx[c] - v * dt)
                             : q0 - (CT)0.5 * sg * (sdx[c] + v * dt);
            sf[f] = v * qf;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int u = t + k * kBlock;
        if (u < nd) qo[i0 + u] = (TQ)(sq[u + 2] - dt * (sf[u + 1] - sf[u]) * sdi[u + 2]);
    }
}

// ---------------------------------------------------------------------------
// mesh-only tables of a shared mesh
// ---------------------------------------------------------------------------

struct MeshTabW {
    double *dx, *dxinv, *hinv, *stc;
    float *dxf, *dxinvf, *hinvf, *stcf;
    int32_t *bucket;
    double2 *bnext;
    int32_t nb;
    double *scal;
    CellRec<float> *crf;
    CellRec<double> *crd;
    float2 *rrf;
    float *stp;
    double2 *rrd;
    double2 *stpd;
    float *stdv;
    double *ppmd;
    float *ppmf;
    int32_t *nonu;
    int32_t *nonu_min;
};

template <int P>
__global__ __launch_bounds__(256) void k_mesh_prep(const double *x, int n, MeshTabW T)
{
    constexpr int LO = (P - 1) / 2;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const double len = x[n] - x[0];
    if (j < n) {
        const double dx = x[j + 1] - x[j];
        const double h = centre_gap(x, n, len, j);
        T.dx[j] = dx;
        T.dxinv[j] = 1.0 / dx;
        T.hinv[j] = 1.0 / h;
        T.dxf[j] = (float)dx;
        T.dxinvf[j] = (float)(1.0 / dx);
        T.hinvf[j] = (float)(1.0 / h);
        T.rrf[j] = make_float2((float)dx, (float)(1.0 / h));
        T.rrd[j] = make_double2(dx, 1.0 / h);
        double th[P + 1];
        const double xc = x[j];
        for (int a = 0; a <= P; ++a) th[a] = (node_x(x, n, len, j - LO + a) - xc) / dx;
        // the cell's own edges, exactly (the FP32 streaming kernel relies on it)
        th[LO] = 0.0;
        th[LO + 1] = 1.0;
        double *st = T.stc + j * (2 * (P + 1));
        float *sf = T.stcf + j * (2 * (P + 1));
        CellRec<float> rf;
        CellRec<double> rd;
        rf.xc = rd.xc = xc;
        rf.dxinv = rd.dxinv = 1.0 / dx;
        for (int a = 0; a < 6; ++a) {
            rf.th[a] = rf.rd[a] = 0.0f;
            rd.th[a] = rd.rd[a] = 0.0;
        }
        for (int a = 0; a <= P; ++a) {
            double den = 1.0;
            for (int b = 0; b <= P; ++b)
                if (b != a) den *= th[a] - th[b];
            st[a] = th[a];
            st[P + 1 + a] = 1.0 / den;
            sf[a] = (float)th[a];
            sf[P + 1 + a] = (float)(1.0 / den);
            rf.th[a] = (float)th[a];
            rf.rd[a] = (float)(1.0 / den);
            rd.th[a] = th[a];
            rd.rd[a] = 1.0 / den;
        }
        T.crf[j] = rf;
        T.crd[j] = rd;
        {
            float v[9];
            int k = 0;
            for (int a = 0; a <= P; ++a)
                if (a != LO && a != LO + 1) v[k++] = rf.th[a];
            for (int a = 0; a <= P; ++a)
                if (a != LO) v[k++] = rf.rd[a];
            for (; k < 9; ++k) v[k] = 0.0f;
            float4 *p4 = (float4 *)T.stp;
            p4[j] = make_float4(v[0], v[1], v[2], v[3]);
            p4[n + j] = make_float4(v[4], v[5], v[6], v[7]);
            T.stp[8 * n + j] = v[8];
        }
        {
            // FP64: the cell's left edge and 1/dx, then the same values, in
            // pairs (six planes of double2)
            double v[12];
            int k = 0;
            v[k++] = xc;
            v[k++] = 1.0 / dx;
            for (int a = 0; a <= P; ++a)
                if (a != LO && a != LO + 1) v[k++] = rd.th[a];
            for (int a = 0; a <= P; ++a)
                if (a != LO) v[k++] = rd.rd[a];
            for (; k < 12; ++k) v[k] = 0.0;
            for (int pl = 0; pl < 6; ++pl) T.stpd[pl * n + j] = make_double2(v[2 * pl], v[2 * pl + 1]);
            // the same offsets and denominators as FP32 deviations from those
            // of equally spaced nodes (offset b - LO, denominator 1 / prod_{a != b}
            // (b - a)): th_b - (b - LO), and rd_b / rd_eq_b - 1
            float dv9[9];
            int m = 0;
            for (int a = 0; a <= P; ++a)
                if (a != LO && a != LO + 1) dv9[m++] = (float)(rd.th[a] - (double)(a - LO));
            for (int a = 0; a <= P; ++a) {
                if (a == LO) continue;
                double eq = 1.0;
                for (int b = 0; b <= P; ++b)
                    if (b != a) eq *= (double)(a - b);
                dv9[m++] = (float)(rd.rd[a] * eq - 1.0);
            }
            for (; m < 9; ++m) dv9[m] = 0.0f;
            float4 *d4 = (float4 *)T.stdv;
            d4[j] = make_float4(dv9[0], dv9[1], dv9[2], dv9[3]);
            d4[n + j] = make_float4(dv9[4], dv9[5], dv9[6], dv9[7]);
            T.stdv[8 * n + j] = dv9[8];
        }
        const PpmW pw = ppm_weights(x[wrap_small(j - 1, n) + 1] - x[wrap_small(j - 1, n)], dx,
                                    x[wrap_small(j + 1, n) + 1] - x[wrap_small(j + 1, n)],
                                    x[wrap_small(j + 2, n) + 1] - x[wrap_small(j + 2, n)]);
        const double pv[5] = {pw.d1, pw.d2, pw.e1, pw.e2, pw.e3};
        for (int k = 0; k < 5; ++k) {
            T.ppmd[k * n + j] = pv[k];
            T.ppmf[k * n + j] = (float)pv[k];
        }
    }
    if (j < T.nb) {
        // lower-bound cell of bucket j, taken a hair below the bucket start so
        // that a bucket number rounded up by one still bounds the cell from
        // below; then the next two nodes (+inf past the last cell)
        const double w = len / (double)T.nb;
        const int c0 = find_cell(x, n, x[0] + ((double)j - 1e-6) * w);
        T.bucket[j] = c0;
        const double inf = __builtin_huge_val();
        T.bnext[j] = make_double2(c0 + 1 < n ? x[c0 + 1] : inf, c0 + 2 < n ? x[c0 + 2] : inf);
    }
    if (j == 0) {
        T.scal[0] = (double)T.nb / len;
        T.scal[1] = 1.0 / len;
        T.scal[2] = x[0] * ((double)T.nb / len);
    }
}

// Uniform runs of a shared mesh: prefix counts of the cells whose size
// differs from the largest (nonu) and from the smallest (nonu_min) by more
// than kUniformTol of it.  One workgroup of 1024 threads: both sizes by a
// coalesced pass and block reductions; then each of the 16 waves takes one
// contiguous segment of the row, counts its flagged cells, and after one
// scan of the 16 counts writes its segment's prefix 64 cells at a time from
// one ballot per flag (no barrier inside the segment loops).
__global__ __launch_bounds__(1024) void k_mesh_uniform(const double *x, int n, int32_t *nonu,
                                                       int32_t *nonu_min)
{
    __shared__ double smax[16], smin[16];
    __shared__ int32_t soff[2][17];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    double mx = 0.0, mn = __builtin_huge_val();
#pragma unroll 8
    for (int j = t; j < n; j += 1024) {
        const double d = x[j + 1] - x[j];
        mx = fmax(mx, d);
        mn = fmin(mn, d);
    }
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, o, 64));
        mn = fmin(mn, __shfl_xor(mn, o, 64));
    }
    if (lane == 0) {
        smax[wv] = mx;
        smin[wv] = mn;
    }
    __syncthreads();
    double hx = smax[0], hn = smin[0];
    for (int w = 1; w < 16; ++w) {
        hx = fmax(hx, smax[w]);
        hn = fmin(hn, smin[w]);
    }
    auto off_max = [&](double d) { return fabs(d - hx) > kUniformTol * hx; };
    auto off_min = [&](double d) { return fabs(d - hn) > kUniformTol * hn; };
    const int seg = (n + 15) / 16;
    const int a0 = min(n, wv * seg), a1 = min(n, a0 + seg);
    int32_t cx = 0, cn = 0;
#pragma unroll 4
    for (int j = a0 + lane; j < a1; j += 64) {
        const double d = x[j + 1] - x[j];
        cx += off_max(d) ? 1 : 0;
        cn += off_min(d) ? 1 : 0;
    }
    for (int o = 32; o > 0; o >>= 1) {
        cx += __shfl_xor(cx, o, 64);
        cn += __shfl_xor(cn, o, 64);
    }
    if (lane == 0) {
        soff[0][wv + 1] = cx;
        soff[1][wv + 1] = cn;
    }
    __syncthreads();
    if (t == 0) {
        soff[0][0] = soff[1][0] = 0;
        for (int w = 1; w <= 16; ++w) {
            soff[0][w] += soff[0][w - 1];
            soff[1][w] += soff[1][w - 1];
        }
    }
    __syncthreads();
    int32_t bx = soff[0][wv], bn = soff[1][wv];
    const uint64_t below = (1ull << lane) - 1ull;
    for (int j0 = a0; j0 < a1; j0 += 64) {
        const int j = j0 + lane;
        bool fx = false, fn = false;
        if (j < a1) {
            const double d = x[j + 1] - x[j];
            fx = off_max(d);
            fn = off_min(d);
        }
        const uint64_t mbx = __ballot(fx), mbn = __ballot(fn);
        if (j < a1) {
            nonu[j] = bx + __popcll(mbx & below);
            nonu_min[j] = bn + __popcll(mbn & below);
        }
        bx += __popcll(mbx);
        bn += __popcll(mbn);
    }
    if (t == 0) {
        nonu[n] = soff[0][16];
        nonu_min[n] = soff[1][16];
    }
}

// ---------------------------------------------------------------------------
// ragged-row tile table: tile_ptr[r] = sum_{r'<r} ceil(N_r'/tile) and
// tile_row[t] = row of tile t.  One workgroup of 1024 threads.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(1024) void k_tiles_prep(const int64_t *row_ptr,
                                                     int64_t n_rows, int tile,
                                                     int64_t *tile_ptr,
                                                     int32_t *tile_row)
{
    __shared__ int64_t stot[1024];
    const int64_t per = (n_rows + 1023) / 1024;
    const int64_t r0 = min(n_rows, (int64_t)threadIdx.x * per);
    const int64_t r1 = min(n_rows, r0 + per);
    int64_t run = 0;
    for (int64_t r = r0; r < r1; ++r)
        run += (row_ptr[r + 1] - row_ptr[r] + tile - 1) / tile;
    stot[threadIdx.x] = run;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t o = threadIdx.x >= (unsigned)d ? stot[threadIdx.x - d] : 0;
        __syncthreads();
        stot[threadIdx.x] += o;
        __syncthreads();
    }
    int64_t acc = stot[threadIdx.x] - run;
    for (int64_t r = r0; r < r1; ++r) {
        tile_ptr[r] = acc;
        const int64_t nt = (row_ptr[r + 1] - row_ptr[r] + tile - 1) / tile;
        for (int64_t k = 0; k < nt; ++k) tile_row[acc + k] = (int32_t)r;
        acc += nt;
    }
    if (threadIdx.x == 1023) tile_ptr[n_rows] = stot[1023];
}

template <typename TQ, int P>
hipError_t step_scan(const StepArgs &a, int scan, hipStream_t st)
{
    const dim3 g((unsigned)a.rows.n_tiles), b(kBlock);
    switch (scan) {
    case kScanF64:
    case kSumDirect: hipLaunchKernelGGL((k_step<TQ, P, kScanF64>), g, b, 0, st, a); break;
    case kScanTwoSum: hipLaunchKernelGGL((k_step<TQ, P, kScanTwoSum>), g, b, 0, st, a); break;
    default: hipLaunchKernelGGL((k_step<TQ, P, kScanF32>), g, b, 0, st, a); break;
    }
    return hipGetLastError();
}

template <typename TQ>
hipError_t step_order(const StepArgs &a, int scan, int order, hipStream_t st)
{
    switch (order) {
    case 1: return step_scan<TQ, 1>(a, scan, st);
    case 3: return step_scan<TQ, 3>(a, scan, st);
    default: return step_scan<TQ, 5>(a, scan, st);
    }
}

size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

} // namespace

size_t mesh_tab_bytes(int64_t n, int order)
{
    const int64_t nb = 4 * n;
    return 3 * al256(8 * n) + 3 * al256(4 * n) + al256(8 * n * 2 * (order + 1)) +
           al256(4 * n * 2 * (order + 1)) + al256(4 * nb) + al256(16 * nb) + al256(16) +
           al256(sizeof(CellRec<float>) * n) + al256(sizeof(CellRec<double>) * n) +
           al256(8 * n) + al256(36 * n) + al256(16 * n) + al256(96 * n) + al256(36 * n) + al256(40 * n) +
           al256(20 * n) +
           2 * al256(4 * (n + 1));
}

hipError_t launch_mesh_prep(const double *x, int64_t n, int order, void *mem,
                            MeshTab &tab, hipStream_t stream, bool uniform)
{
    char *p = (char *)mem;
    MeshTabW w;
    w.dx = (double *)p; p += al256(8 * n);
    w.dxinv = (double *)p; p += al256(8 * n);
    w.hinv = (double *)p; p += al256(8 * n);
    w.dxf = (float *)p; p += al256(4 * n);
    w.dxinvf = (float *)p; p += al256(4 * n);
    w.hinvf = (float *)p; p += al256(4 * n);
    w.stc = (double *)p; p += al256(8 * n * 2 * (order + 1));
    w.stcf = (float *)p; p += al256(4 * n * 2 * (order + 1));
    w.bucket = (int32_t *)p; p += al256(4 * 4 * n);
    w.nb = (int32_t)(4 * n);
    w.bnext = (double2 *)p; p += al256(16 * 4 * n);
    w.scal = (double *)p; p += al256(16);
    w.crf = (CellRec<float> *)p; p += al256(sizeof(CellRec<float>) * n);
    w.crd = (CellRec<double> *)p; p += al256(sizeof(CellRec<double>) * n);
    w.rrf = (float2 *)p; p += al256(8 * n);
    w.stp = (float *)p; p += al256(36 * n);
    w.rrd = (double2 *)p; p += al256(16 * n);
    w.stpd = (double2 *)p; p += al256(96 * n);
    w.stdv = (float *)p; p += al256(36 * n);
    w.ppmd = (double *)p; p += al256(40 * n);
    w.ppmf = (float *)p; p += al256(20 * n);
    w.nonu = (int32_t *)p; p += al256(4 * (n + 1));
    w.nonu_min = (int32_t *)p;
    tab.dx = w.dx; tab.dxinv = w.dxinv; tab.hinv = w.hinv; tab.stc = w.stc;
    tab.dxf = w.dxf; tab.dxinvf = w.dxinvf; tab.hinvf = w.hinvf; tab.stcf = w.stcf;
    tab.bucket = w.bucket;
    tab.nb = w.nb;
    tab.scal = w.scal;
    tab.bnext = w.bnext;
    tab.crf = w.crf;
    tab.crd = w.crd;
    tab.rrf = w.rrf;
    tab.stp = w.stp;
    tab.rrd = w.rrd;
    tab.stpd = w.stpd;
    tab.stdv = w.stdv;
    tab.ppmd = w.ppmd;
    tab.ppmf = w.ppmf;
    tab.nonu = uniform ? w.nonu : nullptr;
    tab.nonu_min = uniform ? w.nonu_min : nullptr;
    // one wave per workgroup, so that the cells' tables (the first n threads,
    // FP64 divisions) spread over every CU
    const unsigned grid = (unsigned)((w.nb + 63) / 64);
    switch (order) {
    case 1: hipLaunchKernelGGL(k_mesh_prep<1>, dim3(grid), dim3(64), 0, stream, x, (int)n, w); break;
    case 3: hipLaunchKernelGGL(k_mesh_prep<3>, dim3(grid), dim3(64), 0, stream, x, (int)n, w); break;
    default: hipLaunchKernelGGL(k_mesh_prep<5>, dim3(grid), dim3(64), 0, stream, x, (int)n, w); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !uniform) return e;
    hipLaunchKernelGGL(k_mesh_uniform, dim3(1), dim3(1024), 0, stream, x, (int)n, w.nonu,
                       w.nonu_min);
    return hipGetLastError();
}

hipError_t launch_tiles_prep(const int64_t *row_ptr, int64_t n_rows, int tile,
                             int64_t *tile_ptr, int32_t *tile_row,
                             hipStream_t stream)
{
    hipLaunchKernelGGL(k_tiles_prep, dim3(1), dim3(1024), 0, stream, row_ptr,
                       n_rows, tile, tile_ptr, tile_row);
    return hipGetLastError();
}

hipError_t launch_step(const StepArgs &a, bool f64, int scan, int order,
                       hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    if (a.rag.rec) {
        if (f64) return hipErrorInvalidValue;
        return launch_step_rag(a, order, scan, stream);
    }
    if (f64) return step_order<double>(a, kScanF64, order, stream);
    return step_order<float>(a, scan, order, stream);
}

hipError_t launch_residual(const ResidualArgs &a, bool f64, hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    // the staged window (tile + 4 cells) must fit kItems slots a lane
    if (a.rows.tile > kResTile) return hipErrorInvalidValue;
    const dim3 grid((unsigned)a.rows.n_tiles), block(kBlock);
    if (f64)
        hipLaunchKernelGGL(k_residual<double>, grid, block, 0, stream, a);
    else
        hipLaunchKernelGGL(k_residual<float>, grid, block, 0, stream, a);
    return hipGetLastError();
}

// Plain copy kernel (16-byte words, then the tail bytes): also usable inside
// a captured graph, where it keeps copy nodes out.
__global__ __launch_bounds__(256) void k_copy(const unsigned char *src, unsigned char *dst,
                                              int64_t bytes)
{
    const int64_t nw = bytes / 16;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = i0; i < nw; i += stride)
        ((uint4 *)dst)[i] = ((const uint4 *)src)[i];
    for (int64_t b = nw * 16 + i0; b < bytes; b += stride) dst[b] = src[b];
}

hipError_t launch_copy(const void *src, void *dst, int64_t bytes,
                       hipStream_t stream)
{
    if (bytes <= 0) return hipSuccess;
    if ((((uintptr_t)src | (uintptr_t)dst) & 15) != 0)
        return hipMemcpyAsync(dst, src, (size_t)bytes, hipMemcpyDeviceToDevice, stream);
    const int64_t nw = (bytes + 15) / 16;
    const unsigned grid = (unsigned)std::min<int64_t>((nw + 255) / 256, 8192);
    hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, stream,
                       (const unsigned char *)src, (unsigned char *)dst, bytes);
    return hipGetLastError();
}

} // namespace ram
