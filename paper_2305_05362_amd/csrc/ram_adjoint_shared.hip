// ram_adjoint_shared.hip -- one RAM step backwards on rows sharing a mesh.
//
// The step is Q^n --shift--> Q^{n+1/2} --residual--> Q^{n+1}.  Given the
// gradient Qbar^{n+1}, one tile of destination cells [i0, i0+nd) does, in one
// pass:
//
//   (1) the residual adjoint (transpose of the upwind step's Jacobian at
//       Q^{n+1/2}): Qbar^{n+1/2} on the tile's cells, and dvbar += on its
//       faces -- slopes, face states and fluxes transposed over a two-cell
//       halo; limiter derivative 0 where the one-sided slopes differ in sign,
//       the dv >= 0 branch at dv = 0;
//   (2) the shift adjoint.  With V_e the interpolated cumulative at shifted
//       node e and M'_i = V_{i+1} - V_i, the transpose scatters
//       Vbar_e = Mbar'_{e-1} - Mbar'_e through each node's Lagrange weights
//       onto the window's node cumulative (Cbar), and the source masses are
//       the suffix sums Mbar_m = sum_{j > m} Cbar_j (a DPP block scan).
//       Source cells shared with the neighbouring tiles (the p cells of each
//       boundary node's stencil) go to a per-tile side buffer, summed per
//       cell in a fixed order by a second kernel; every other cell is
//       written once;
//   (3) v0bar += dt * sum_e -Vbar_e q~(x~_e), with q~ the reconstruction
//       (derivative of the interpolated cumulative of Q^n) at the shifted
//       node: one term per tile, summed per row in tile order afterwards.
//
// FP64 results are the same in every run: the Cbar scatter goes in p+1
// passes, one stencil offset each, in which the nodes that share a source
// cell (and so a target) are summed in node order by the first of them; the
// FP32 state's scatter uses LDS atomics (FP64) instead.
//
// Tiles whose source window does not fit in LDS gather instead: each window
// cell telescopes the tile's Vbar down to one Mbar' plus the few stencils
// that straddle it, with the weights recomputed from global memory.
#include "ram_device.h"
#include "ram_adjoint_dev.h"

#include <type_traits>

namespace ram {
namespace {

using namespace dev;

constexpr int kWinA = 1536;             // LDS window capacity, cells

__device__ inline int wrap1a(int j, int n)
{
    return j < 0 ? j + n : (j >= n ? j - n : j);
}

// Eight consecutive values of an LDS array from index 4t (16-byte aligned):
// 16-byte reads, lane-consecutive, so the banks serve them without conflict
// (eight 4-byte reads four words apart per lane would conflict 8-way).
template <typename T>
__device__ inline void lds_read8(const T *p, T (&o)[8])
{
    static_assert(sizeof(T) == 4 || sizeof(T) == 8 || sizeof(T) == 16, "element size");
    if constexpr (sizeof(T) == 4) {
        const float4 a = ((const float4 *)p)[0], b = ((const float4 *)p)[1];
        const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int i = 0; i < 8; ++i) o[i] = __builtin_bit_cast(T, v[i]);
    } else if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double2 a = ((const double2 *)p)[i];
            o[2 * i] = __builtin_bit_cast(T, a.x);
            o[2 * i + 1] = __builtin_bit_cast(T, a.y);
        }
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) o[i] = p[i];
    }
}

// Window cell j (of W) of a tile: cells only this tile's window holds go to
// the state, the window's first and last p cells to the tile's side buffer.
template <typename TQ, int P>
__device__ inline void put_cell_any(TQ *qbi, TQ *edge, int mm, int j, int W, TQ v)
{
    if (j >= P && j < W - P) qbi[mm] = v;
    else if (j < P) edge[j] = v;
    else edge[P + j - max(P, W - P)] = v;
}

template <typename CT>
struct AdjLds {
    using CT2 = typename TabT<CT>::T2;
    static constexpr int NP = kStepNodes + 8;
    static constexpr size_t res = (4 * sizeof(CT) + sizeof(CT2)) * NP;
    // Cbar and the window masses; for an FP64 state also each node's window
    // index and one pass's terms (the ordered scatter)
    static constexpr bool ordered = sizeof(CT) == 8;
    static constexpr size_t win = 2 * sizeof(double) * (kWinA + 1) +
                                  (ordered ? (sizeof(int) + sizeof(double)) * kStepNodes : 0);
    static constexpr size_t nodes = 2 * sizeof(int64_t) * kStepNodes;
    static constexpr size_t u0 = res > win ? res : win;
    static constexpr size_t uni = u0 > nodes ? u0 : nodes;
};

template <typename TQ, int P, bool RES>
__global__ __launch_bounds__(kBlock) void k_adj_sh(StepAdjArgs a)
{
    using CT = TQ;
    using ACD = Acc<kScanF64>;
    using L = AdjLds<CT>;
    constexpr int LO = (P - 1) / 2;
    constexpr int NI = kItems;

    using CT2 = typename TabT<CT>::T2;
    constexpr int NP = L::NP;
    __shared__ CT smb[kStepNodes];               // Mbar' of the tile's cells
    __shared__ double sedge[kItems][kBlock / 64]; // q~ of each wave's first lane
    __shared__ double swt[kBlock / 64];
    __shared__ double sred[kBlock / 64];
    __shared__ __attribute__((aligned(16))) unsigned char su[L::uni];
    __shared__ int s_flag;
    // residual-adjoint staging, index j <-> cell (and face) i0-2+j
    CT *sqh = (CT *)su;                          // Q^{n+1/2}
    CT *sqb = sqh + NP;                          // Qbar^{n+1}
    CT *sdi = sqb + NP;                          // 1/dx
    CT *sdv = sdi + NP;                          // dv of face i0-2+j
    CT2 *srr = (CT2 *)(sdv + NP);                // (dx, 1/centre gap)
    // shift-adjoint arrays
    double *scb = (double *)su;                  // Cbar on window nodes
    double *spm = scb + (kWinA + 1);             // masses of the Q^n window
    int *sjn = (int *)(spm + (kWinA + 1));       // ordered scatter: node window index
    double *sct = (double *)(sjn + kStepNodes);  //   and the pass's term per node
    // direct path
    int64_t *sgd = (int64_t *)su;

    const Rows &R = a.rows;
    const MeshTab &tb = R.tab;
    const int n = (int)R.n_cols;
    const int tpr = (n + R.tile - 1) / R.tile;
    const int row = (int)(blockIdx.x / (unsigned)tpr);
    const int i0 = ((int)blockIdx.x - row * tpr) * R.tile;
    const int nd = min(R.tile, n - i0);
    const int NE = nd + 1;
    const bool inner = (i0 - 2 >= 0) && (i0 + nd + 2 < n);
    const double *x = R.edges;
    const int64_t qoff = (int64_t)row * n;
    const TQ *qbo = (const TQ *)a.qbar_out + qoff;
    TQ *qbi = (TQ *)a.qbar_in + qoff;
    const TQ *qf = a.q_fwd ? (const TQ *)a.q_fwd + qoff : nullptr;
    const bool want_v0 = a.v0bar != nullptr && qf != nullptr;
    const double s = a.v0[row] * a.dt;
    const double len = x[n] - x[0];
    const RowShift rs = row_shift(s, len, tb.scal[1]);
    const int64_t wlo = a.plan_wlo[blockIdx.x];
    const int W = a.plan_w[blockIdx.x];
    const int t = threadIdx.x;
    TQ *edge = (TQ *)a.edge + (int64_t)blockIdx.x * (2 * P);
    auto wr = [&](int j) { return inner ? j : wrap1a(j, n); };
    const CT dt = (CT)a.dt;

    // ---- (1) residual adjoint: Mbar' of the tile's cells -------------------
    // Staged once: Q^{n+1/2}, Qbar^{n+1}, mesh records and dv of cells/faces
    // i0-2 .. i0+nd+1; then every thread takes four consecutive cells and
    // forms, from its window of cells a-2..a+5 and faces a-1..a+5 in
    // registers, the face fluxes' adjoints, the limiter derivatives and the
    // cells' Qbar^{n+1/2} (and dvbar of its four faces).
    if (RES) {
        const TQ *qh = (const TQ *)a.q_half + qoff;
        const TQ *dv = (const TQ *)a.dv + qoff;
        TQ *dvb = a.dvbar ? (TQ *)a.dvbar + qoff : nullptr;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int j = t + k * kBlock;
            if (j < nd + 4) {
                const int c = wr(i0 - 2 + j);
                sqh[j] = (CT)qh[c];
                sqb[j] = (CT)qbo[c];
                sdi[j] = TabT<CT>::dxinv(tb)[c];
                sdv[j] = (CT)dv[c];
                srr[j] = TabT<CT>::rr(tb)[c];
            }
        }
        __syncthreads();
        const int u0 = 4 * t;                        // first cell of the thread
        if (u0 < nd) {
            CT q[8], qb[8], di[8], dx[8], hv[8], vv[7], v8[8];
            CT2 r8[8];
            lds_read8(sqh + u0, q);
            lds_read8(sqb + u0, qb);
            lds_read8(sdi + u0, di);
            lds_read8(srr + u0, r8);
            lds_read8(sdv + u0, v8);
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                dx[w] = r8[w].x;
                hv[w] = r8[w].y;
            }
#pragma unroll
            for (int f = 0; f < 7; ++f) vv[f] = v8[f + 1];
            // faces a-1+f, between window cells f and f+1
            CT fbar[7], qsb[7], scs[7], half[7];
            bool up[7];
#pragma unroll
            for (int f = 0; f < 7; ++f) {
                const CT v = vv[f];
                up[f] = v >= (CT)0;
                fbar[f] = dt * (qb[f + 1] * di[f + 1] - qb[f] * di[f]);
                half[f] = up[f] ? (CT)0.5 * (dx[f] - v * dt) : (CT)-0.5 * (dx[f + 1] + v * dt);
                qsb[f] = fbar[f] * v;
                scs[f] = qsb[f] * half[f];
            }
            // window cells 1..6: slope, limiter derivatives (times the gap
            // inverses), and the slope adjoint each receives
            CT sg[8], da[8], db[8], sb[8];
#pragma unroll
            for (int w = 1; w <= 6; ++w) {
                const CT ap = (q[w + 1] - q[w]) * hv[w];
                const CT bm = (q[w] - q[w - 1]) * hv[w - 1];
                sg[w] = da[w] = db[w] = (CT)0;
                if (ap * bm > (CT)0) {
                    const CT sm = ap + bm;
                    const CT inv = (CT)1 / (sm * sm);
                    da[w] = (CT)2 * bm * bm * inv * hv[w];
                    db[w] = (CT)2 * ap * ap * inv * hv[w - 1];
                    sg[w] = harmonic2(ap, bm);
                }
                sb[w] = (up[w - 1] ? (CT)0 : scs[w - 1]) + (up[w] ? scs[w] : (CT)0);
            }
#pragma unroll
            for (int w = 2; w <= 5; ++w) {
                const int u = u0 + w - 2;
                if (u < nd) {
                    CT gs = qb[w];
                    if (!up[w - 1]) gs += qsb[w - 1];
                    if (up[w]) gs += qsb[w];
                    gs += sb[w - 1] * da[w - 1] + sb[w] * (db[w] - da[w]) - sb[w + 1] * db[w + 1];
                    smb[u] = gs * di[w];
                    if (dvb) {
                        // face i0+u = window face w-1, upwind cell w-1 or w
                        const int f = w - 1;
                        const int cu = up[f] ? f : f + 1;
                        const CT v = vv[f];
                        const CT qs = q[cu] + sg[cu] * half[f];
                        dvb[i0 + u] = (TQ)((CT)dvb[i0 + u] +
                                           fbar[f] * (qs - (CT)0.5 * sg[cu] * v * dt));
                    }
                }
            }
        }
    } else {
        // fixed slots, so that every thread's loads are in flight together
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int u = t + k * kBlock;
            if (u < nd) smb[u] = (CT)qbo[i0 + u] * TabT<CT>::dxinv(tb)[i0 + u];
        }
    }
    __syncthreads();

    // ---- (2) a uniform tile ---------------------------------------------------
    // FP32; the window plan found the tile's nodes and window in one uniform
    // run of the mesh: node e sits in window cell LO + e at the plan's theta,
    // and the shift is the forward kernel's stencil Q'_i = sum_d cc_d Q_{i+d}
    // (window index i + d for destination cell i).  Its transpose gathers
    // sum_d cc_d Mbar'_{j-d} for window cell j (times dx: the source value's
    // gradient), with no search, scatter or scan; v0bar's telescoped sum
    // -sum_i Mbar'_i (q~_{i+1} - q~_i) takes q~_{i+1} - q~_i =
    // sum_d (d cc_d / d theta) Q^n_{i+d}.  The window's first and last p
    // cells are shared with the neighbouring tiles and accumulated with
    // atomics after the zeroing pass, as in the general path.
    if constexpr (sizeof(TQ) == 4) {
        const float thu = __int_as_float(a.plan_w[2 * R.n_tiles + blockIdx.x]);
        if (thu >= 0.0f && W > 0 && W <= kWinA) {
            // window cells in fixed slots (W = nd + P <= NI * kBlock + P), so
            // that each thread's loads are issued together; one cell size
            const int base = a.plan_w[R.n_tiles + blockIdx.x];   // wlo mod n
            constexpr int NS = NI + (P + kBlock - 1) / kBlock;
            double *sw = (double *)su;                           // Q^n of the window
            const double dx0 = TabT<double>::dx(tb)[base];
            int mms[NS];
            double qw[NS];
#pragma unroll
            for (int r = 0; r < NS; ++r) {
                const int j = t + r * kBlock;
                const int mm = base + j;
                mms[r] = j < W ? (mm >= n ? wrap_small(mm, n) : mm) : 0;
                if (want_v0 && j < W) qw[r] = (double)qf[mms[r]];
            }
            double cs[P + 1];
            uniform_stencil<double, P>((double)thu, cs);
#pragma unroll
            for (int r = 0; r < NS; ++r) {
                const int j = t + r * kBlock;
                if (j < W) {
                    double acc = 0.0;
#pragma unroll
                    for (int d = 0; d <= P; ++d) {
                        const int i = j - d;
                        if (i >= 0 && i < nd) acc += cs[d] * (double)smb[i];
                    }
                    const double val = acc * dx0;
                    put_cell_any<TQ, P>(qbi, edge, mms[r], j, W, (TQ)val);
                }
            }
            if (want_v0) {
#pragma unroll
                for (int r = 0; r < NS; ++r) {
                    const int j = t + r * kBlock;
                    if (j < W) sw[j] = qw[r];
                }
                double dw[P + 1], gd[P + 2], dd[P + 1];
                uniform_dweights<double, P>((double)thu, 1.0, dw);
                outward_sums<double, P>(dw, gd);
#pragma unroll
                for (int d = 0; d <= P; ++d) dd[d] = gd[d] - gd[d + 1];
                __syncthreads();
                double vpart = 0.0;
#pragma unroll
                for (int k = 0; k < NI; ++k) {
                    const int u = t + k * kBlock;
                    if (u < nd) {
                        double dq = 0.0;
#pragma unroll
                        for (int d = 0; d <= P; ++d) dq += dd[d] * sw[u + d];
                        vpart -= (double)smb[u] * dq;
                    }
                }
                for (int d = 32; d >= 1; d >>= 1) vpart += __shfl_xor(vpart, d);
                if ((t & 63) == 0) sred[t >> 6] = vpart;
                __syncthreads();
                if (t == 0) {
                    double tot = 0.0;
                    for (int wv = 0; wv < kBlock / 64; ++wv) tot += sred[wv];
                    a.v0part[blockIdx.x] = a.dt * tot;
                }
            }
            return;
        }
    }

    // ---- (2) shifted nodes, tile-local Vbar ---------------------------------
    int64_t g[NI];
    CT w[NI][P + 1];
    double vb[NI], xh[NI];
    int cc[NI];
    bool ok = true;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int e = t + k * kBlock;
        g[k] = 0;
        vb[k] = 0.0;
        if (e < NE) {
            const int en = i0 + e;
            const int kx = en >= n ? 1 : 0;
            const double xe = x[en >= n ? en - n : en];
            g[k] = node_eval_adj<CT, P>(x, n, tb, rs, len, xe, kx, w[k], cc[k],
                                        xh[k]);
        }
        if (e < NE) {
            vb[k] = (e >= 1 ? (double)smb[e - 1] : 0.0) - (e <= nd - 1 ? (double)smb[e] : 0.0);
            const int64_t jc = g[k] - wlo;
            ok = ok && jc >= LO && jc + P - LO <= W;
        }
    }
    if (t == 0) s_flag = (W > 0 && W <= kWinA) ? 1 : 0;
    __syncthreads();
    if (!ok) s_flag = 0;
    __syncthreads();
    const bool windowed = s_flag != 0;
    double qt[NI];                               // q~ at the thread's nodes
#pragma unroll
    for (int k = 0; k < NI; ++k) qt[k] = 0.0;

    if (windowed) {
        // ---- Cbar scatter --------------------------------------------------
        for (int j = t; j <= W; j += kBlock) scb[j] = 0.0;
        const int base = a.plan_w[R.n_tiles + blockIdx.x];   // wlo mod n
        // forward window masses for the reconstruction at the nodes
        if (want_v0) {
            for (int j = t; j < W; j += kBlock) {
                int mm = base + j;
                mm = mm >= n ? wrap_small(mm, n) : mm;
                spm[j] = (double)qf[mm] * TabT<double>::dx(tb)[mm];
            }
        }
        __syncthreads();
        // V_e = C(g) + sum_{a != lo} w_a (C(g-lo+a) - C(g)): the node's own
        // cumulative enters with weight exactly one, so the suffix sums of
        // cells below the stencil telescope without the weights' rounding
        if constexpr (L::ordered) {
            double part[NI];
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                const int e = t + k * kBlock;
                part[k] = 0.0;
                if (e < NE) {
                    sjn[e] = (int)(g[k] - wlo);
#pragma unroll
                    for (int b = 0; b <= P; ++b)
                        if (b != LO) part[k] += (double)w[k][b] * vb[k];
                }
            }
            // pass b: node e's term goes to window node jc_e - lo + b; the
            // targets rise with e, equal only for nodes in one source cell
#pragma unroll
            for (int b = 0; b <= P; ++b) {
#pragma unroll
                for (int k = 0; k < NI; ++k) {
                    const int e = t + k * kBlock;
                    if (e < NE) sct[e] = b == LO ? vb[k] - part[k] : (double)w[k][b] * vb[k];
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < NI; ++k) {
                    const int e = t + k * kBlock;
                    if (e < NE && (e == 0 || sjn[e - 1] != sjn[e])) {
                        const int jc = sjn[e];
                        double sum = sct[e];
                        for (int f = e + 1; f < NE && sjn[f] == jc; ++f) sum += sct[f];
                        scb[jc - LO + b] += sum;
                    }
                }
                __syncthreads();
            }
        } else {
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                if (t + k * kBlock < NE) {
                    const int jc = (int)(g[k] - wlo);
                    double part = 0.0;
#pragma unroll
                    for (int b = 0; b <= P; ++b) {
                        if (b == LO) continue;
                        const double c = (double)w[k][b] * vb[k];
                        atomicAdd(&scb[jc - LO + b], c);
                        part += c;
                    }
                    atomicAdd(&scb[jc], vb[k] - part);
                }
            }
            __syncthreads();
        }
        // ---- suffix sums over the window nodes -----------------------------
        const int NN = W + 1;
        const int per = (NN + kBlock - 1) / kBlock;
        const int j0 = min(NN, t * per), j1 = min(NN, j0 + per);
        double mine[8], run = 0.0;
#pragma unroll
        for (int r = 0; r < 8; ++r)
            if (j0 + r < j1) {
                mine[r] = scb[j0 + r];
                run += mine[r];
            }
        double total;
        double acc = block_exscan_dpp<ACD>(run, swt, total);
        // S(cell j) = total - sum_{node <= j} Cbar
#pragma unroll
        for (int r = 0; r < 8; ++r)
            if (j0 + r < j1) {
                acc += mine[r];
                scb[j0 + r] = total - acc;
            }
        __syncthreads();
        // ---- Qbar = dx * S: interior cells once, shared cells by atomics ---
        for (int j = t; j < W; j += kBlock) {
            int mm = base + j;
            mm = mm >= n ? wrap_small(mm, n) : mm;
            const double val = scb[j] * TabT<double>::dx(tb)[mm];
            put_cell_any<TQ, P>(qbi, edge, mm, j, W, (TQ)val);
        }
        // reconstruction q~ at the nodes: sum_b w'_b (C(g-lo+b) - C(g)) / dx_c,
        // the differences summed from the masses next to the node
        if (want_v0) {
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                const int e = t + k * kBlock;
                if (e < NE) {
                    const int jc = (int)(g[k] - wlo);
                    double dwd[P + 1];
                    node_dweights<CT, P>(tb, cc[k], xh[k], dwd);
                    double dq = 0.0, up = 0.0, dn = 0.0;
#pragma unroll
                    for (int b = LO + 1; b <= P; ++b) {
                        up += spm[jc + b - LO - 1];
                        dq += dwd[b] * up;
                    }
#pragma unroll
                    for (int b = LO - 1; b >= 0; --b) {
                        dn += spm[jc - LO + b];
                        dq -= dwd[b] * dn;
                    }
                    qt[k] = dq;
                }
            }
        }
    } else {
        // ---- direct path: gather per window cell ---------------------------
        double *svb = (double *)(sgd + kStepNodes);
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            if (t + k * kBlock < NE) {
                sgd[t + k * kBlock] = g[k];
                svb[t + k * kBlock] = vb[k];
            }
        }
        __syncthreads();
        // window bounds from the plan: this tile's first cell and the next
        // tile's (the row's first tile one period on, for the last tile), so
        // the shared cells are exactly the ones the zeroing pass cleared
        const int64_t wl = wlo;
        const bool last = i0 + nd >= n;
        const int64_t wend =
            (last ? a.plan_wlo[blockIdx.x - (tpr - 1)] + n : a.plan_wlo[blockIdx.x + 1]) + P;
        const int Wd = (int)(wend - wl);
        for (int j = t; j < Wd; j += kBlock) {
            const int64_t target = wl + j + LO;
            int lo = 0, hi = NE;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (sgd[mid] > target) hi = mid; else lo = mid + 1;
            }
            double S = (lo >= 1 && lo <= nd) ? (double)smb[lo - 1] : 0.0;
            for (int e = lo - 1; e >= 0 && sgd[e] > target - P; --e) {
                const int en = i0 + e;
                const int kx = en >= n ? 1 : 0;
                double ww[P + 1], xh2;
                int c2;
                node_eval_adj<double, P>(x, n, tb, rs, len, x[en >= n ? en - n : en], kx,
                                         ww, c2, xh2);
                // the share of the node's weights on cumulative nodes above
                // the cell, with the node's own weight taken as one minus the
                // others (the form the windowed scatter uses)
                const int bmin = (int)min((int64_t)P, max((int64_t)1, target - sgd[e] + 1));
                double h = 0.0;
                if (bmin > LO) {
                    for (int b = P; b >= bmin; --b) h += ww[b];
                } else {
                    for (int b = 0; b < bmin; ++b) h += ww[b];
                    h = 1.0 - h;
                }
                S += svb[e] * h;
            }
            const int mm = wrapi(wl + j, n);
            const double val = S * TabT<double>::dx(tb)[mm];
            put_cell_any<TQ, P>(qbi, edge, mm, j, Wd, (TQ)val);
        }
        if (want_v0) {
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                const int e = t + k * kBlock;
                if (e < NE) {
                    double dwd[P + 1];
                    node_dweights<CT, P>(tb, cc[k], xh[k], dwd);
                    qt[k] = direct_qtilde<TQ, P>(x, qf, n, dwd, cc[k]);
                }
            }
        }
    }
    // ---- (3) v0bar ------------------------------------------------------------
    // dV_e/ds = -q~_e; with Vbar_e = Mbar'_{e-1} - Mbar'_e the tile's sum
    // telescopes to -sum_i Mbar'_i (q~_{i+1} - q~_i), which keeps the
    // cancellation between neighbouring nodes inside one FP64 difference
    if (want_v0) {
        // q~ of node e+1: the next lane's, or across a wave boundary the
        // next wave's first lane (the last thread's next node is thread 0's
        // next item)
        double qn[NI];
#pragma unroll
        for (int k = 0; k < NI; ++k) qn[k] = __shfl_down(qt[k], 1);
        const int lane = t & 63, wv = t >> 6;
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < NI; ++k) sedge[k][wv] = qt[k];
        }
        __syncthreads();
        if (lane == 63) {
#pragma unroll
            for (int k = 0; k < NI; ++k)
                qn[k] = wv + 1 < kBlock / 64 ? sedge[k][wv + 1]
                                             : (k + 1 < NI ? sedge[k + 1][0] : 0.0);
        }
        double vpart = 0.0;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int u = t + k * kBlock;
            if (u < nd) vpart -= (double)smb[u] * (qn[k] - qt[k]);
        }
        for (int d = 32; d >= 1; d >>= 1) vpart += __shfl_xor(vpart, d);
        if ((t & 63) == 0) sred[t >> 6] = vpart;
        __syncthreads();
        if (t == 0) {
            double tot = 0.0;
            for (int wv = 0; wv < kBlock / 64; ++wv) tot += sred[wv];
            a.v0part[blockIdx.x] = a.dt * tot;
        }
    }
}

template <typename TQ, int P>
hipError_t adj_order(const StepAdjArgs &a, hipStream_t st)
{
    const dim3 g((unsigned)a.rows.n_tiles), b(kBlock);
    if (a.dv) hipLaunchKernelGGL((k_adj_sh<TQ, P, true>), g, b, 0, st, a);
    else hipLaunchKernelGGL((k_adj_sh<TQ, P, false>), g, b, 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_edge_sum(a.rows, a.plan_wlo, a.edge, a.qbar_in, sizeof(TQ) == 8, P, st);
    if (e != hipSuccess || !(a.v0bar && a.q_fwd)) return e;
    return launch_v0_reduce(a.rows, a.v0part, a.v0bar, st);
}

template <typename TQ>
hipError_t adj_dispatch(const StepAdjArgs &a, int order, hipStream_t st)
{
    switch (order) {
    case 1: return adj_order<TQ, 1>(a, st);
    case 3: return adj_order<TQ, 3>(a, st);
    default: return adj_order<TQ, 5>(a, st);
    }
}

} // namespace

hipError_t launch_step_adjoint_shared(const StepAdjArgs &a, bool f64, int order,
                                      hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    if (f64) return adj_dispatch<double>(a, order, stream);
    return adj_dispatch<float>(a, order, stream);
}

} // namespace ram
