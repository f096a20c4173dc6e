// ram_adjoint_fast.hip -- one RAM step backwards for an FP32 state on rows
// that share a mesh, one tile of kFastTile destination cells a wave, on the
// forward's per-call tile plan (k_plan_fast, no halo: a tile's nodes are
// i0 .. i0+nd and its window the source cells of their stencils).
//
// The step is Q^n --shift--> Q^{n+1/2} --residual--> Q^{n+1}.  Given
// Qbar^{n+1}, a tile does (the same algebra as k_adj_sh):
//
//   (1) the residual's transpose on its cells, four consecutive cells a lane
//       with their two-cell neighbourhoods in registers (the cells' states
//       and gradients through the wave's LDS, the halo from global memory):
//       Qbar^{n+1/2} of the cells and the dvbar terms of their left faces;
//   (2) the shift's transpose onto the window (Section 3, Steps 1-3, Eq.
//       mass_shift_algo transposed):
//       * a tile in a uniform run of the mesh (every node in the next source
//         cell at one theta; the plan's stencil cc) gathers
//         Qbar^n_j = sum_d cc_d Qbar^{n+1/2}_{j-d}: no search, no scatter;
//       * another tile scatters Vbar_e = Mbar'_{e-1} - Mbar'_e (Mbar' the
//         destination masses' gradient) through each node's Lagrange weights
//         onto the window's cumulative nodes (FP64 LDS atomics; the node's
//         own weight taken as one minus the others), sums them from the top
//         (a DPP suffix scan, FP64) into the window masses' gradient, and
//         multiplies by the cell sizes;
//       the p cells at each end of a window are shared with the neighbouring
//       tile: each tile stores its terms for them in a side buffer, and a
//       second kernel adds up, cell by cell, the terms of every tile whose
//       window holds the cell (no atomics; the same sum in every run);
//   (3) v0bar: -dt sum_i Mbar'_i (q~_{i+1} - q~_i) with q~ the
//       reconstruction (x-derivative of the interpolated cumulative of Q^n)
//       at the shifted nodes: a fixed stencil on Q^n in a uniform run, the
//       weights' derivatives on the window masses (FP64) elsewhere; one term
//       a tile, summed per row in tile order afterwards.
//
// A tile whose window exceeds the LDS (or wraps a short row more than once)
// locates its nodes itself and gathers each window cell's gradient from the
// few stencils that straddle it (the telescoped form of k_adj_sh's direct
// path).
#include "ram_device.h"
#include "ram_adjoint_dev.h"
#include "ram_wave.h"

namespace ram {
namespace {

using namespace dev;

constexpr int kFT = kFastTile;
constexpr int kStage = kFT + 8;          // staged cells of one array (cell c at c + 4)
constexpr int kPadQ = 8;                 // zeros around a uniform tile's Qbar^{n+1/2} (>= p)
constexpr int kSwOff = 288;              // a uniform tile's window values, LDS floats
constexpr size_t kGenU = 8 * (kFastWin + 8);   // bytes: staging, FP64 window, Cbar or node data
constexpr int kGenShareA = 4;            // other tiles: a grid of a quarter of the tiles

static_assert(2 * kPadQ + kFT <= kSwOff, "uniform LDS layout");
static_assert(kSwOff + kFT + 16 <= 3 * kStage, "uniform LDS layout");
static_assert(3 * kStage * 4 <= kGenU && 16 * kFastNodes <= kGenU, "general LDS layout");

// Eight values of an LDS array from index i (i even): 8 + 16 + 8 bytes.
__device__ __forceinline__ void lds8(const float *s, int i, float (&o)[8])
{
    const float2 a = *(const float2 *)(s + i);
    const float4 b = *(const float4 *)(s + i + 2);
    const float2 c = *(const float2 *)(s + i + 6);
    o[0] = a.x; o[1] = a.y;
    o[2] = b.x; o[3] = b.y; o[4] = b.z; o[5] = b.w;
    o[6] = c.x; o[7] = c.y;
}

__device__ __forceinline__ void f4(const float4 &v, float *o)
{
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}

// Sum of a double over the wave.
__device__ __forceinline__ double wave_sum(double v)
{
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    return v;
}

// The residual step's transpose on four consecutive cells a .. a+3 (Section
// 3.1 reading: the upwind flux with the van Leer slope and the swept-interval
// average; the limiter's derivative is 0 where the one-sided slopes differ in
// sign, the dv >= 0 branch taken at dv = 0), from cells a-2 .. a+5 (index w):
// the state the residual read q, the gradient of its result qb, 1/dx di, dx,
// the inverse centre gaps hv (cell w to w+1), and the velocities v8 of their
// left faces.  gs: the gradient of the shifted state on the four cells; fb:
// the dv gradient terms of their left faces.
__device__ __forceinline__ void residual_adj4(const float (&q)[8], const float (&qb)[8],
                                              const float (&di)[8], const float (&dx)[8],
                                              const float (&hv)[8], const float (&v8)[8],
                                              float dt, float (&gs)[4], float (&fb)[4])
{
    // faces a-1+f, between cells f and f+1
    float fbar[7], qsb[7], scs[7], half[7], vv[7];
    bool up[7];
#pragma unroll
    for (int f = 0; f < 7; ++f) {
        const float v = v8[f + 1];
        vv[f] = v;
        up[f] = v >= 0.0f;
        fbar[f] = dt * (qb[f + 1] * di[f + 1] - qb[f] * di[f]);
        half[f] = up[f] ? 0.5f * (dx[f] - v * dt) : -0.5f * (dx[f + 1] + v * dt);
        qsb[f] = fbar[f] * v;
        scs[f] = qsb[f] * half[f];
    }
    // cells 1 .. 6: slope, limiter derivatives (times the gap inverses), and
    // the slope gradient each receives
    float sg[8], da[8], db[8], sb[8];
#pragma unroll
    for (int w = 1; w <= 6; ++w) {
        const float ap = (q[w + 1] - q[w]) * hv[w];
        const float bm = (q[w] - q[w - 1]) * hv[w - 1];
        sg[w] = da[w] = db[w] = 0.0f;
        if (ap * bm > 0.0f) {
            const float sm = ap + bm;
            const float inv = 1.0f / (sm * sm);
            da[w] = 2.0f * bm * bm * inv * hv[w];
            db[w] = 2.0f * ap * ap * inv * hv[w - 1];
            sg[w] = harmonic2(ap, bm);
        }
        sb[w] = (up[w - 1] ? 0.0f : scs[w - 1]) + (up[w] ? scs[w] : 0.0f);
    }
#pragma unroll
    for (int w = 2; w <= 5; ++w) {
        float g = qb[w];
        if (!up[w - 1]) g += qsb[w - 1];
        if (up[w]) g += qsb[w];
        g += sb[w - 1] * da[w - 1] + sb[w] * (db[w] - da[w]) - sb[w + 1] * db[w + 1];
        gs[w - 2] = g;
        // the cell's left face (face w-1), upwind cell w-1 or w
        const int f = w - 1;
        const int cu = up[f] ? f : f + 1;
        const float qs = q[cu] + sg[cu] * half[f];
        fb[w - 2] = fbar[f] * (qs - 0.5f * sg[cu] * vv[f] * dt);
    }
}

// What the residual's transpose reads for a lane's four cells: states and
// gradients of the cells (and of the tile's two-cell halo a side), their
// faces' velocities and, for a searching tile, their geometry.
struct ResIn {
    float4 qb4, qh4, dv4, fb4;
    float2 qbL, qbR, qhL, qhR, dvL, dvR;
};

template <bool RES>
__device__ __forceinline__ ResIn res_load(const StepAdjArgs &a, int64_t qoff, int n, int i0,
                                          int nd, int cl, bool want_dvb)
{
    ResIn r;
    const float *qbo = (const float *)a.qbar_out + qoff;
    r.qb4 = *(const float4 *)(qbo + i0 + cl);
    if constexpr (RES) {
        // halo cells i0-2, i0-1 and i0+nd, i0+nd+1 (the row is a multiple of
        // four cells: 8-byte aligned pairs that do not straddle its end)
        const int hl = i0 >= 2 ? i0 - 2 : i0 - 2 + n;
        const int hr = i0 + nd < n ? i0 + nd : 0;
        const float *qh = (const float *)a.q_half + qoff;
        const float *dv = (const float *)a.dv + qoff;
        r.qh4 = *(const float4 *)(qh + i0 + cl);
        r.dv4 = *(const float4 *)(dv + i0 + cl);
        r.fb4 = want_dvb ? *(const float4 *)((const float *)a.dvbar + qoff + i0 + cl)
                         : make_float4(0.f, 0.f, 0.f, 0.f);
        r.qbL = *(const float2 *)(qbo + hl);
        r.qbR = *(const float2 *)(qbo + hr);
        r.qhL = *(const float2 *)(qh + hl);
        r.qhR = *(const float2 *)(qh + hr);
        r.dvL = *(const float2 *)(dv + hl);
        r.dvR = *(const float2 *)(dv + hr);
    }
    return r;
}

// Stage the states through the wave's LDS (cell c of the tile at c + 4 of
// each of three arrays) and read back each lane's cells a-2 .. a+5.
__device__ __forceinline__ void res_stage(const ResIn &r, float *st, int cl, int nd, int t,
                                          float (&q)[8], float (&qb)[8], float (&v8)[8])
{
    float *sqh = st, *sqb = st + kStage, *sdv = st + 2 * kStage;
    *(float4 *)(sqh + 4 + cl) = r.qh4;
    *(float4 *)(sqb + 4 + cl) = r.qb4;
    *(float4 *)(sdv + 4 + cl) = r.dv4;
    if (t == 0) {
        *(float2 *)(sqh + 2) = r.qhL;
        *(float2 *)(sqb + 2) = r.qbL;
        *(float2 *)(sdv + 2) = r.dvL;
        *(float2 *)(sqh + nd + 4) = r.qhR;
        *(float2 *)(sqb + nd + 4) = r.qbR;
        *(float2 *)(sdv + nd + 4) = r.dvR;
    }
    wave_sync();
    lds8(sqh, cl + 2, q);
    lds8(sqb, cl + 2, qb);
    lds8(sdv, cl + 2, v8);
}

// Store the gradient v of window cell j (of W; row cell `cell`): a cell only
// this tile's window holds goes to the state, the window's first p cells
// (head) and its last p (tail; the two overlap-free when W < 2p) to the
// tile's side buffer, for k_adjf_edges.  One store a lane, whichever it is.
template <int P>
__device__ __forceinline__ void put_cell(float *qbi, float *edge, int cell, int j, int W, float v)
{
    float *dst;
    if (j >= P && j < W - P) dst = qbi + cell;
    else if (j < P) dst = edge + j;
    else dst = edge + P + (j - max(P, W - P));
    *dst = v;
}

// ---------------------------------------------------------------------------
// A tile in a uniform run (k_plan_fast: nodes i0 .. i0+nd in window cells
// LO .. LO+nd at one theta, cells i0-1 .. i0+nd of the run's size).
// ---------------------------------------------------------------------------
template <int P, bool RES, bool V0>
__device__ __forceinline__ void adj_uniform_tile(const StepAdjArgs &a, const FastTile &r,
                                                 float *su, int t)
{
    constexpr int NG = 2;                            // window groups a lane (>= kFT + P + 3 cells)
    const int n = (int)a.rows.n_cols;
    const MeshTab &tb = a.rows.tab;
    const TilePos p = tile_pos(r.pad[0], n, 0);
    const int i0 = p.i0, nd = p.nd, c4 = 4 * t, cl = min(c4, nd - 4);
    const bool live = c4 < nd;
    const int64_t qoff = (int64_t)p.row * n;
    float *qbi = (float *)a.qbar_in + qoff;
    const int W = r.w, base = r.base, a0 = base & ~3, off = base - a0;
    const int gl = (W + off - 1) >> 2;               // last memory-aligned window group
    const bool want_dvb = RES && a.dvbar != nullptr;

    // ---- 1. every load: the cells, their halo and faces; the halo cells'
    // geometry (outside the run's checked cells); the window's values (v0bar)
    const ResIn ri = res_load<RES>(a, qoff, n, i0, nd, cl, want_dvb);
    float4 gL = make_float4(0.f, 0.f, 0.f, 0.f), gR = gL;
    float2 iL = make_float2(0.f, 0.f), iR = iL;
    if constexpr (RES) {
        const int hl = i0 >= 2 ? i0 - 2 : i0 - 2 + n;
        const int hr = i0 + nd < n ? i0 + nd : 0;
        gL = *(const float4 *)(tb.rrf + hl);         // (dx, 1/gap) of cells i0-2, i0-1
        gR = *(const float4 *)(tb.rrf + hr);         // of cells i0+nd, i0+nd+1
        iL = *(const float2 *)(tb.dxinvf + hl);
        iR = *(const float2 *)(tb.dxinvf + hr);
    }
    float wq[NG][4];
    if constexpr (V0) {
        const float *qf = (const float *)a.q_fwd + qoff;
#pragma unroll
        for (int u = 0; u < NG; ++u) {
            int c = a0 + 4 * min(t + u * kLanes, gl);
            c = c >= n ? c - n : c;
            f4(*(const float4 *)(qf + c), wq[u]);
        }
    }

    // ---- 2. the residual's transpose: Qbar^{n+1/2} of the lane's cells -----
    float gs[4];
    if constexpr (RES) {
        float q[8], qb[8], v8[8];
        res_stage(ri, su, cl, nd, t, q, qb, v8);
        float dx[8], hv[8], di[8];
#pragma unroll
        for (int w = 0; w < 8; ++w) {
            dx[w] = r.dx;
            hv[w] = r.hinv;
            di[w] = r.dxinv;
        }
        if (cl == 0) {                               // cell i0-2 and the gap to i0-1
            dx[0] = gL.x;
            hv[0] = gL.y;
            di[0] = iL.x;
        }
        if (cl + 4 == nd) {                          // the gap to i0+nd+1, and that cell
            hv[6] = gR.y;
            dx[7] = gR.z;
            di[7] = iR.y;
        }
        float fb[4];
        residual_adj4(q, qb, di, dx, hv, v8, (float)a.dt, gs, fb);
        if (want_dvb && live)
            *(float4 *)((float *)a.dvbar + qoff + i0 + c4) =
                make_float4(ri.fb4.x + fb[0], ri.fb4.y + fb[1], ri.fb4.z + fb[2], ri.fb4.w + fb[3]);
        wave_sync();                                 // the staged arrays are dead
    } else {
        f4(ri.qb4, gs);
    }

    // ---- 3. Qbar^{n+1/2} at kPadQ + u with zeros around; the window's
    // values at j + off (the memory-aligned groups as loaded)
    float *sq = su, *sw = su + kSwOff;
    if (t < kPadQ) {
        sq[t] = 0.0f;
        sq[kPadQ + nd + t] = 0.0f;
    }
    if (live) *(float4 *)(sq + kPadQ + c4) = make_float4(gs[0], gs[1], gs[2], gs[3]);
    if constexpr (V0) {
#pragma unroll
        for (int u = 0; u < NG; ++u) {
            const int g = t + u * kLanes;
            if (g <= gl) *(float4 *)(sw + 4 * g) = make_float4(wq[u][0], wq[u][1], wq[u][2], wq[u][3]);
        }
    }
    wave_sync();

    // ---- 4. Qbar^n_j = sum_d cc_d Qbar^{n+1/2}_{j-d}, one window cell a lane
    constexpr int NJ = (kFT + P + kLanes - 1) / kLanes;
    float *edge = (float *)a.edge + (int64_t)r.pad[0] * (2 * P);
#pragma unroll
    for (int u = 0; u < NJ; ++u) {
        const int j = t + u * kLanes;
        if (j >= W) continue;
        float acc = 0.0f;
#pragma unroll
        for (int d = 0; d <= P; ++d) acc += r.cc[d] * sq[kPadQ + j - d];
        int c = base + j;
        c = c >= n ? c - n : c;
        put_cell<P>(qbi, edge, c, j, W, acc);
    }

    // ---- 5. v0bar: q~_{i+1} - q~_i = sum_d dd_d Q^n_{i+d}, one cell a lane ----
    if constexpr (V0) {
        double dw[P + 1], gd[P + 2], dd[P + 1];
        uniform_dweights<double, P>((double)__int_as_float(r.pad[1]), 1.0, dw);
        outward_sums<double, P>(dw, gd);
#pragma unroll
        for (int d = 0; d <= P; ++d) dd[d] = gd[d] - gd[d + 1];
        double vp = 0.0;
#pragma unroll
        for (int u = 0; u < kFT / kLanes; ++u) {
            const int i = t + u * kLanes;
            if (i >= nd) continue;
            double dq = 0.0;
#pragma unroll
            for (int d = 0; d <= P; ++d) dq += dd[d] * (double)sw[i + d + off];
            vp -= (double)sq[kPadQ + i] * (double)r.dxinv * dq;
        }
        vp = wave_sum(vp);
        if (t == 0) a.v0part[r.pad[0]] = a.dt * vp;
    }
}

// ---------------------------------------------------------------------------
// The residual's transpose of a searching tile (per-cell geometry): Mbar' =
// Qbar^{n+1/2} / dx of the tile's cells into smb[1 + u] (smb[0] and
// smb[nd + 1] zero: the tile's nodes' Vbar_e = smb[e] - smb[e + 1]).
// ---------------------------------------------------------------------------
template <bool RES, class After, class Store>
__device__ __forceinline__ void res_general(const StepAdjArgs &a, const ResIn &ri,
                                            const float2 (&rr)[8], const float (&dxi)[8],
                                            int64_t qoff, int i0, int nd, int cl, int t,
                                            bool want_dvb, float *st, After after, Store store)
{
    const int c4 = 4 * t;
    float gs[4];
    if constexpr (RES) {
        float q[8], qb[8], v8[8], dx[8], hv[8];
        res_stage(ri, st, cl, nd, t, q, qb, v8);
        after();                                     // loads issued once the staging is read
#pragma unroll
        for (int w = 0; w < 8; ++w) {
            dx[w] = rr[w].x;
            hv[w] = rr[w].y;
        }
        float fb[4];
        residual_adj4(q, qb, dxi, dx, hv, v8, (float)a.dt, gs, fb);
        if (want_dvb && c4 < nd)
            *(float4 *)((float *)a.dvbar + qoff + i0 + c4) =
                make_float4(ri.fb4.x + fb[0], ri.fb4.y + fb[1], ri.fb4.z + fb[2], ri.fb4.w + fb[3]);
    } else {
        after();
        f4(ri.qb4, gs);
    }
    store(gs);
}

// Mbar' = Qbar^{n+1/2} / dx of the lane's four cells into smb[1 + u], with
// smb[0] and smb[nd + 1] zero (FP32 from the FP32 sizes).
__device__ __forceinline__ void store_mb(float *smb, const float (&gs)[4], const float (&dxi)[8],
                                         int nd, int t)
{
    const int c4 = 4 * t;
    if (c4 < nd) {
#pragma unroll
        for (int k = 0; k < 4; ++k) smb[1 + c4 + k] = gs[k] * dxi[2 + k];
    }
    if (t == 0) {
        smb[0] = 0.0f;
        smb[nd + 1] = 0.0f;
    }
}

// Geometry of cells i0+cl-2 .. i0+cl+5: (dx, 1/centre gap) as four 16-byte
// pairs, 1/dx as 8 + 16 + 8 bytes (a multiple of four cells a row: no group
// straddles its end).
__device__ __forceinline__ void load_geom(const MeshTab &tb, int n, int cb, float2 (&rr)[8],
                                          float (&dxi)[8])
{
    auto wr = [&](int c) { return c < 0 ? c + n : (c >= n ? c - n : c); };
#pragma unroll
    for (int pr = 0; pr < 4; ++pr) {
        const float4 r2 = *(const float4 *)(tb.rrf + wr(cb + 2 * pr));
        rr[2 * pr] = make_float2(r2.x, r2.y);
        rr[2 * pr + 1] = make_float2(r2.z, r2.w);
    }
    const float2 d0 = *(const float2 *)(tb.dxinvf + wr(cb));
    const float4 d1 = *(const float4 *)(tb.dxinvf + wr(cb + 2));
    const float2 d2 = *(const float2 *)(tb.dxinvf + wr(cb + 6));
    dxi[0] = d0.x; dxi[1] = d0.y;
    dxi[2] = d1.x; dxi[3] = d1.y; dxi[4] = d1.z; dxi[5] = d1.w;
    dxi[6] = d2.x; dxi[7] = d2.y;
}

// v0bar of a tile from q~ at its nodes (node m = t + 64u in slot u) and Mbar'
// in smb: -dt sum_i Mbar'_i (q~_{i+1} - q~_i), one term a tile.
template <int NS, typename MT>
__device__ __forceinline__ void v0_term(const StepAdjArgs &a, int tile, const double (&qt)[NS],
                                        const MT *smb, int nd, int t)
{
    double vp = 0.0;
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const int m = t + u * kLanes;
        // q~ of node m + 1: the next lane's, lane 63 the next slot's lane 0
        double qn = __shfl_down(qt[u], 1);
        if (u + 1 < NS) {
            const double q0 = __shfl(qt[u + 1 < NS ? u + 1 : u], 0);
            if (t == kLanes - 1) qn = q0;
        }
        if (m < nd) vp -= (double)smb[1 + m] * (qn - qt[u]);
    }
    vp = wave_sum(vp);
    if (t == 0) a.v0part[tile] = a.dt * vp;
}

// ---------------------------------------------------------------------------
// A searching tile whose window fits the LDS: the plan's window index and
// theta of every node, the Lagrange weights from the stencil planes of the
// node's source cell (as the forward's streaming kernel takes them).
// ---------------------------------------------------------------------------
template <int P, bool RES, bool V0>
__device__ __forceinline__ void adj_window_tile(const StepAdjArgs &a, const FastTile &ft,
                                                unsigned char *su, float *smb, int t)
{
    constexpr int LO = (P - 1) / 2;
    constexpr int NS = (kFastNodes + kLanes - 1) / kLanes;   // node slots
    constexpr int NG = 2;                            // window groups a lane loads first
    const MeshTab &tb = a.rows.tab;
    const int n = (int)a.rows.n_cols;
    const TilePos p = tile_pos(ft.pad[0], n, 0);
    const int i0 = p.i0, nd = p.nd, NE = nd + 1, c4 = 4 * t, cl = min(c4, nd - 4);
    const int64_t qoff = (int64_t)p.row * n;
    float *qbi = (float *)a.qbar_in + qoff;
    const int W = ft.w, base = ft.base, a0 = base & ~3, off = base - a0;
    const int gl = (W + off - 1) >> 2;               // last memory-aligned window group
    const bool want_dvb = RES && a.dvbar != nullptr;

    // ---- 1. node plan, the residual's cells and geometry, the window --------
    const float *thp = a.fast.theta + (int64_t)ft.pad[1] * kFastNodes;
    const int16_t *jcp = a.fast.jc + (int64_t)ft.pad[1] * kFastNodes;
    float thv[NS];
    int jv[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const int m = min(t + u * kLanes, kFastNodes - 1);
        thv[u] = thp[m];
        jv[u] = jcp[m];
    }
    const ResIn ri = res_load<RES>(a, qoff, n, i0, nd, cl, want_dvb);
    float2 rr[8];
    float dxi[8];
    if constexpr (RES) {
        load_geom(tb, n, i0 + cl - 2, rr, dxi);
    } else {
        f4(*(const float4 *)(tb.dxinvf + i0 + cl), dxi + 2);
    }
    float wq[NG][4], wd[NG][4];
    const float *qf = V0 ? (const float *)a.q_fwd + qoff : nullptr;
    // the window's values and sizes (v0bar), loaded while the residual runs
    auto load_win = [&]() {
        if constexpr (V0) {
#pragma unroll
            for (int u = 0; u < NG; ++u) {
                int c = a0 + 4 * min(t + u * kLanes, gl);
                c = c >= n ? c - n : c;
                f4(*(const float4 *)(qf + c), wq[u]);
                f4(*(const float4 *)(tb.dxf + c), wd[u]);
            }
        }
    };

    // ---- 2. stencil data of the nodes' source cells (and their 1/dx) --------
    float rth[NS][P + 1], rrd[NS][P + 1], ndi[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        int c = base + jv[u];
        c = c >= n ? c - n : c;
        float v[12];
        f4(((const float4 *)tb.stp)[c], v);
        f4(((const float4 *)tb.stp)[n + c], v + 4);
        v[8] = tb.stp[8 * n + c];
        int k = 0;
#pragma unroll
        for (int b = 0; b <= P; ++b) rth[u][b] = b == LO ? 0.0f : (b == LO + 1 ? 1.0f : v[k++]);
#pragma unroll
        for (int b = 0; b <= P; ++b) rrd[u][b] = b == LO ? 0.0f : v[k++];
        ndi[u] = V0 ? tb.dxinvf[c] : 0.0f;
    }

    // ---- 3. the residual's transpose -> Mbar' ------------------------------------
    res_general<RES>(a, ri, rr, dxi, qoff, i0, nd, cl, t, want_dvb, (float *)su, load_win,
                     [&](const float (&gs)[4]) { store_mb(smb, gs, dxi, nd, t); });
    wave_sync();                                     // staging dead, smb visible

    // ---- 4. q~ at the nodes from the window masses (FP64), v0bar -----------------
    double qt[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) qt[u] = 0.0;
    if constexpr (V0) {
        double *spm = (double *)su;                  // window mass j at spm[j]
#pragma unroll
        for (int u = 0; u < NG; ++u) {
            const int g = t + u * kLanes;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int j = 4 * g + k - off;
                if (g <= gl && j >= 0 && j < W) spm[j] = (double)wq[u][k] * (double)wd[u][k];
            }
        }
        for (int g = t + NG * kLanes; g <= gl; g += kLanes) {     // long windows
            int c = a0 + 4 * g;
            c = c >= n ? c - n : c;
            float vq[4], vd[4];
            f4(*(const float4 *)(qf + c), vq);
            f4(*(const float4 *)(tb.dxf + c), vd);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int j = 4 * g + k - off;
                if (j >= 0 && j < W) spm[j] = (double)vq[k] * (double)vd[k];
            }
        }
        wave_sync();
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            // x-derivatives of the weights other than the own node's (FP32,
            // the product rule through the prefix and suffix products)
            const float th = thv[u];
            float tt[P + 1], pre[P + 1], suf[P + 1], dpre[P + 1], dsuf[P + 1];
#pragma unroll
            for (int b = 0; b <= P; ++b) tt[b] = th - rth[u][b];
            pre[0] = 1.0f;
            dpre[0] = 0.0f;
#pragma unroll
            for (int b = 1; b <= P; ++b) {
                pre[b] = pre[b - 1] * tt[b - 1];
                dpre[b] = dpre[b - 1] * tt[b - 1] + pre[b - 1];
            }
            suf[P] = 1.0f;
            dsuf[P] = 0.0f;
#pragma unroll
            for (int b = P - 1; b >= 0; --b) {
                suf[b] = suf[b + 1] * tt[b + 1];
                dsuf[b] = dsuf[b + 1] * tt[b + 1] + suf[b + 1];
            }
            const int j = jv[u];
            double dq = 0.0, upm = 0.0, dnm = 0.0;
#pragma unroll
            for (int b = LO + 1; b <= P; ++b) {
                upm += spm[j + b - LO - 1];
                dq += (double)(rrd[u][b] * (dpre[b] * suf[b] + pre[b] * dsuf[b])) * upm;
            }
#pragma unroll
            for (int b = LO - 1; b >= 0; --b) {
                dnm += spm[j - LO + b];
                dq -= (double)(rrd[u][b] * (dpre[b] * suf[b] + pre[b] * dsuf[b])) * dnm;
            }
            qt[u] = dq * (double)ndi[u];
        }
        wave_sync();                                 // the masses are dead
    }

    // ---- 5. Cbar: each node's Vbar through its weights (FP64 LDS atomics) --------
    double *scb = (double *)su;                      // window node j at scb[j]
    const int gq = W >> 2;                           // last group of the nodes 0 .. W
    for (int j = t; j < 4 * (gq + 1); j += kLanes) scb[j] = 0.0;
    wave_sync();
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const int m = t + u * kLanes;
        if (m >= NE) continue;
        const float th = thv[u];
        float tt[P + 1], pre[P + 1], suf[P + 1];
#pragma unroll
        for (int b = 0; b <= P; ++b) tt[b] = th - rth[u][b];
        pre[0] = 1.0f;
#pragma unroll
        for (int b = 1; b <= P; ++b) pre[b] = pre[b - 1] * tt[b - 1];
        suf[P] = 1.0f;
#pragma unroll
        for (int b = P - 1; b >= 0; --b) suf[b] = suf[b + 1] * tt[b + 1];
        const double vb = (double)smb[m] - (double)smb[m + 1];
        const int j = jv[u];
        double part = 0.0;
#pragma unroll
        for (int b = 0; b <= P; ++b) {
            if (b == LO) continue;
            const double c = (double)(rrd[u][b] * (pre[b] * suf[b])) * vb;
            atomicAdd(&scb[j - LO + b], c);
            part += c;
        }
        atomicAdd(&scb[j], vb - part);
    }
    wave_sync();

    // ---- 6. sums from the top: Mbar_m = sum_{j > m} Cbar_j = total - incl_m ------
    using AC = Acc<kScanF64>;
    double carry = 0.0;
    for (int s = 0; s * kLanes <= gq; ++s) {
        const int g = t + s * kLanes;
        const bool in = g <= gq;
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        if (in) {
            const double2 a01 = *(const double2 *)(scb + 4 * g);
            const double2 a23 = *(const double2 *)(scb + 4 * g + 2);
            v[0] = a01.x; v[1] = a01.y; v[2] = a23.x; v[3] = a23.y;
        }
        const double tot = (v[0] + v[1]) + (v[2] + v[3]);
        const double inc = wave_inclusive<AC>(tot);
        double e = AC::template dpp<kDppWaveShr1, 0xf, 0xf>(inc);
        if (t == 0) e = 0.0;
        e += carry;
        if (in) {
            double o[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                e += v[k];
                o[k] = e;
            }
            *(double2 *)(scb + 4 * g) = make_double2(o[0], o[1]);
            *(double2 *)(scb + 4 * g + 2) = make_double2(o[2], o[3]);
        }
        carry += lane63(inc);
    }
    wave_sync();

    // ---- 7. Qbar^n = Mbar dx, one window cell a lane --------------------------------
    float *edge = (float *)a.edge + (int64_t)ft.pad[0] * (2 * P);
    for (int j = t; j < W; j += kLanes) {
        int c = base + j;
        c = c >= n ? c - n : c;
        put_cell<P>(qbi, edge, c, j, W, (float)((carry - scb[j]) * (double)tb.dxf[c]));
    }
    if constexpr (V0) v0_term<NS>(a, ft.pad[0], qt, smb, nd, t);
}

// ---------------------------------------------------------------------------
// A tile whose window does not fit (or wraps a short row more than once): the
// nodes located here (FP64 search of the bucket index), each window cell's
// gradient telescoped from the tile's Vbar down to one Mbar' plus the
// stencils that straddle the cell, q~ from global memory.
// ---------------------------------------------------------------------------
// The reconstruction q~ at a node in cell c from global memory: the weights'
// x-derivatives dw on the cumulative differences C(c - lo + b) - C(c), from
// the masses of cells c-lo .. c+p-lo-1 (FP64).
template <int P>
__device__ __forceinline__ double qtilde_global(const double *x, const float *q, int n,
                                                const double (&dw)[P + 1], int c)
{
    constexpr int LO = (P - 1) / 2;
    double m[P];
#pragma unroll
    for (int k = 0; k < P; ++k) m[k] = cell_mass(x, q, n, (int64_t)c - LO + k);
    double dq = 0.0, up = 0.0, dn = 0.0;
#pragma unroll
    for (int b = LO + 1; b <= P; ++b) {
        up += m[b - 1];
        dq += dw[b] * up;
    }
#pragma unroll
    for (int b = LO - 1; b >= 0; --b) {
        dn += m[b];
        dq -= dw[b] * dn;
    }
    return dq;
}

template <int P, bool RES, bool V0>
__device__ __forceinline__ void adj_direct_tile(const StepAdjArgs &a, const FastTile &ft,
                                                unsigned char *su, float *smb, int t)
{
    constexpr int LO = (P - 1) / 2;
    constexpr int NS = (kFastNodes + kLanes - 1) / kLanes;
    const Rows &R = a.rows;
    const MeshTab &tb = R.tab;
    const int n = (int)R.n_cols;
    const int tile = ft.pad[0];
    const TilePos p = tile_pos(tile, n, 0);
    const int i0 = p.i0, nd = p.nd, NE = nd + 1, cl = min(4 * t, nd - 4);
    const int64_t qoff = (int64_t)p.row * n;
    float *qbi = (float *)a.qbar_in + qoff;
    const double *x = R.edges;
    const double len = x[n] - x[0];
    const RowShift rs = row_shift(a.v0[p.row] * a.dt, len, tb.scal[1]);
    const bool want_dvb = RES && a.dvbar != nullptr;

    const ResIn ri = res_load<RES>(a, qoff, n, i0, nd, cl, want_dvb);
    float2 rr[8];
    float dxi[8];
    if constexpr (RES) load_geom(tb, n, i0 + cl - 2, rr, dxi);
    else f4(*(const float4 *)(tb.dxinvf + i0 + cl), dxi + 2);
    res_general<RES>(a, ri, rr, dxi, qoff, i0, nd, cl, t, want_dvb, (float *)su, [] {},
                     [&](const float (&gs)[4]) { store_mb(smb, gs, dxi, nd, t); });
    wave_sync();

    int64_t *sgd = (int64_t *)su;                    // node m's extended source index
    double *svb = (double *)(sgd + kFastNodes);      // and its Vbar
    double qt[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const int m = t + u * kLanes;
        qt[u] = 0.0;
        if (m < NE) {
            const int en = i0 + m;
            const int kx = en >= n ? 1 : 0;
            float w[P + 1];
            double xh;
            int c;
            sgd[m] = node_eval_adj<float, P>(x, n, tb, rs, len, x[en - kx * n], kx, w, c, xh);
            svb[m] = (double)smb[m] - (double)smb[m + 1];
            if constexpr (V0) {
                double dwd[P + 1];
                node_dweights<float, P>(tb, c, xh, dwd);
                qt[u] = qtilde_global<P>(x, (const float *)a.q_fwd + qoff, n, dwd, c);
            }
        }
    }
    wave_sync();
    // the window: this tile's first node's stencil up to the next tile's
    // (the row's first tile one period on, for the last tile of a row)
    const int tpr = (n + kFT - 1) / kFT;
    const bool last = i0 + nd >= n;
    auto wlo_of = [&](int k) {
        const FastTile &r = a.fast.rec[k];
        return (int64_t)(((uint64_t)(uint32_t)r.wlo_hi << 32) | (uint32_t)r.wlo_lo);
    };
    const int64_t wl = wlo_of(tile);
    const int64_t wend = (last ? wlo_of(tile - (tpr - 1)) + n : wlo_of(tile + 1)) + P;
    const int Wd = (int)(wend - wl);
    float *edge = (float *)a.edge + (int64_t)tile * (2 * P);
    for (int j = t; j < Wd; j += kLanes) {
        const int64_t target = wl + j + LO;
        int lo = 0, hi = NE;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sgd[mid] > target) hi = mid; else lo = mid + 1;
        }
        // nodes lo.. lie wholly above the cell: their Vbar telescopes to Mbar'_{lo-1}
        double S = (lo >= 1 && lo <= nd) ? (double)smb[lo] : 0.0;
        for (int e = lo - 1; e >= 0 && sgd[e] > target - P; --e) {
            const int en = i0 + e;
            const int kx = en >= n ? 1 : 0;
            double ww[P + 1], xh2;
            int c2;
            node_eval_adj<double, P>(x, n, tb, rs, len, x[en - kx * n], kx, ww, c2, xh2);
            // the share of the node's weights on cumulative nodes above the
            // cell, the own weight taken as one minus the others
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
        put_cell<P>(qbi, edge, mm, j, Wd, (float)(S * (double)tb.dxf[mm]));
    }
    if constexpr (V0) v0_term<NS>(a, tile, qt, smb, nd, t);
}

// The window cells that several tiles add into: the first p of every tile's
// window (a tile's window ends p cells past the next tile's start).  Boundary
// T (one thread) writes the cells from its window start up to p cells on or
// the next tile's start, each the sum, tile T first and then down, of the
// terms the tiles whose windows hold it stored (head or tail; tile k's window
// is [A_k, A_{k+1} + p), and across the row's ends the row's tiles one period
// away).  Usually two terms; more where a tile's nodes fall in fewer than p
// source cells.
template <int P>
__global__ __launch_bounds__(256) void k_adjf_edges(StepAdjArgs a)
{
    const int64_t tile = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (tile >= a.rows.n_tiles) return;
    const int n = (int)a.rows.n_cols;
    const int tpr = (n + kFT - 1) / kFT;
    const int64_t row = tile / tpr;
    const int k0 = (int)(tile - row * tpr);
    // window start of the row's k-th tile, any k (k mod tpr, one period per wrap)
    auto start = [&](int k, int64_t &id) {
        const int q = k >= 0 ? k / tpr : -((-k + tpr - 1) / tpr);
        id = row * tpr + (k - q * tpr);
        const FastTile &r = a.fast.rec[id];
        const int64_t w = (int64_t)(((uint64_t)(uint32_t)r.wlo_hi << 32) | (uint32_t)r.wlo_lo);
        return w + (int64_t)q * n;
    };
    int64_t idp, id0, idn;
    const int64_t ap = start(k0 - 1, idp), a0 = start(k0, id0), a1 = start(k0 + 1, idn);
    float *qbi = (float *)a.qbar_in + row * n;
    if (a1 - a0 >= P && a0 - ap >= P) {
        // two terms a cell: this tile's head and the previous tile's tail
        // (its window [ap, a0 + p) of at least 2p cells ends its tail there)
        const float *e0 = (const float *)a.edge + id0 * (2 * P);
        const float *ep = (const float *)a.edge + idp * (2 * P);
        float v[P];
#pragma unroll
        for (int k = 0; k < P; ++k) v[k] = (0.0f + e0[k]) + ep[P + k];
#pragma unroll
        for (int k = 0; k < P; ++k) qbi[wrapi(a0 + k, n)] = v[k];
        return;
    }
    const int64_t mend = min(a0 + P, a1);
    for (int64_t m = a0; m < mend; ++m) {
        float sum = 0.0f;
        int64_t at = a0, an = a1, id = id0;
        for (int k = k0; k > k0 - tpr - 1; --k) {
            if (k != k0) {
                an = at;
                at = start(k, id);
            }
            const int64_t W = an - at + P;
            if (at + W <= m) break;
            const int pos = (int)(m - at);
            const float *e = (const float *)a.edge + id * (2 * P);
            sum += pos < P ? e[pos] : e[P + pos - (int)max((int64_t)P, W - P)];
        }
        qbi[wrapi(m, n)] = sum;
    }
}

// ---------------------------------------------------------------------------
// The limited (PLM / PPM) step backwards: the same tiles, plan and edge sums
// with p = 2 lo + 1 (the reconstruction's stencil, lo cells a side).  The
// limited shift is nonlinear in Q, and its transpose is that of its Jacobian
// at Q^n with each limiter differentiated on the branch it takes there (a
// zero slope where the one-sided differences do not share a sign):
//     Qbar_m = dx_m Mbar'_i (m a whole cell of destination i)
//            + sum_e Vbar_e d ell_e / d Q_m   (|c_e - m| <= lo),
// ell_e the partial integral of node e's cell.  Each node's Jacobian row and
// reconstruction value are evaluated in FP64 from the FP32 state and the
// mesh's FP64 tables, at its FP64 position in its cell (the plan gives the
// cell; uniform runs and searching tiles alike), so the limiters take the
// branches the FP64 evaluation takes; the terms accumulate in FP64 in LDS.
// ---------------------------------------------------------------------------

__device__ inline int64_t rec_wlo(const FastTile &r)
{
    return (int64_t)(((uint64_t)(uint32_t)r.wlo_hi << 32) | (uint32_t)r.wlo_lo);
}

// d ell / d Q_{c-lo+j} (j = 0 .. 2 lo) of the limited partial integral of
// cell c (size h) at theta, and the reconstruction's value there, from the
// averages qv of cells c-lo .. c+lo: PLM with the van Leer slope over the
// reciprocal centre gaps; PPM with the limited slopes of cells c-1 .. c+1,
// the interface values c-1/2 and c+1/2 and the constrained parabola (the
// forward's reconstruction of Section 3.1's reading), chained back through
// the branch each limiter takes.
template <int R>
__device__ __forceinline__ void lim_node(const MeshTab &tb, int n, int c, double h, double th,
                                         const double (&qv)[2 * LimHalo<R>::lo + 1],
                                         double (&gw)[2 * LimHalo<R>::lo + 1], double &qval)
{
    if constexpr (R == kReconPLM) {
        const int cm = c == 0 ? n - 1 : c - 1;
        const double gp = tb.hinv[c], gm = tb.hinv[cm];
        const double av = (qv[2] - qv[1]) * gp, bv = (qv[1] - qv[0]) * gm;
        double sig = 0.0, dsa = 0.0, dsb = 0.0;
        if (av * bv > 0.0) {
            const double s2 = (av + bv) * (av + bv);
            sig = 2.0 * av * bv / (av + bv);
            dsa = 2.0 * bv * bv / s2;
            dsb = 2.0 * av * av / s2;
        }
        // ell = Q_c h theta + sigma h^2 (theta^2 - theta) / 2
        const double ks = 0.5 * h * h * (th * th - th);
        gw[0] = -ks * dsb * gm;
        gw[1] = h * th + ks * (dsb * gm - dsa * gp);
        gw[2] = ks * dsa * gp;
        qval = qv[1] + sig * h * (th - 0.5);
    } else {
        // slope weights of cells c-1 .. c+1, interface weights of c-1 and c
        const double *pw = tb.ppmd;
        double d1[3], d2[3], e1[2], e2[2], e3[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            int m = c - 1 + k;
            m = m < 0 ? m + n : (m >= n ? m - n : m);
            d1[k] = pw[m];
            d2[k] = pw[n + m];
            if (k < 2) {
                e1[k] = pw[2 * n + m];
                e2[k] = pw[3 * n + m];
                e3[k] = pw[4 * n + m];
            }
        }
        // limited slopes of cells c-1, c, c+1 and their derivatives with
        // respect to the averages of each slope's cells
        double dl[3], dd[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double up = qv[k + 2] - qv[k + 1], dn = qv[k + 1] - qv[k];
            const double d = d1[k] * up + d2[k] * dn;
            dd[k][0] = dd[k][1] = dd[k][2] = 0.0;
            dl[k] = 0.0;
            if (up * dn > 0.0) {
                dl[k] = copysign(fmin(fabs(d), 2.0 * fmin(fabs(up), fabs(dn))), d);
                if (fabs(d) <= 2.0 * fabs(up) && fabs(d) <= 2.0 * fabs(dn)) {
                    dd[k][0] = -d2[k];
                    dd[k][1] = d2[k] - d1[k];
                    dd[k][2] = d1[k];
                } else if (fabs(up) <= fabs(dn)) {
                    dd[k][1] = -2.0;                 // twice the upper difference
                    dd[k][2] = 2.0;
                } else {
                    dd[k][0] = -2.0;                 // twice the lower difference
                    dd[k][1] = 2.0;
                }
            }
        }
        // interface values c-1/2 and c+1/2 before the constraints
        const double Lr = qv[1] + e1[0] * (qv[2] - qv[1]) + e2[0] * dl[1] + e3[0] * dl[0];
        const double Rr = qv[2] + e1[1] * (qv[3] - qv[2]) + e2[1] * dl[2] + e3[1] * dl[1];
        const double a = qv[2];
        double L = Lr, Rv = Rr;
        int branch = 0;                              // 1 flat, 2 L pulled in, 3 R pulled in
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
        // d ell / d (a, L, R) with q6 expanded, then back through the branch
        const double th2 = th * th, th3 = th2 * th;
        const double ga = h * (3.0 * th2 - 2.0 * th3);
        const double gl = h * (th - 2.0 * th2 + th3);
        const double gr = h * (th3 - th2);
        double ba = ga, bl = gl, br = gr;
        if (branch == 1) { ba = ga + gl + gr; bl = 0.0; br = 0.0; }
        else if (branch == 2) { ba = ga + 3.0 * gl; bl = 0.0; br = gr - 2.0 * gl; }
        else if (branch == 3) { ba = ga + 3.0 * gr; bl = gl - 2.0 * gr; br = 0.0; }
        double gb[5] = {0.0, 0.0, ba, 0.0, 0.0};
        const double bd[3] = {bl * e3[0], bl * e2[0] + br * e3[1], br * e2[1]};
        gb[1] += bl * (1.0 - e1[0]);
        gb[2] += bl * e1[0] + br * (1.0 - e1[1]);
        gb[3] += br * e1[1];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int j = 0; j < 3; ++j) gb[k + j] += bd[k] * dd[k][j];
#pragma unroll
        for (int k = 0; k < 5; ++k) gw[k] = gb[k];
    }
}

// A window of at most kLimTab cells is tabulated in LDS (per cell its limited
// slope, per interface its value and derivatives); wider windows evaluate
// each node's row from global memory, the accumulator in chunks.
constexpr int kLimTab = 320;
constexpr size_t kLimTabI = 8 * (kLimTab + 8);      // bytes: one FP64 value a cell
constexpr size_t kLimTabD = 16 * (kLimTab + 8);     //        four FP32 values a cell
constexpr size_t kLimU0 = 2 * kLimTabI + kLimTabD;  // table and accumulator
constexpr size_t kLimU = kLimU0 > kGenU ? kLimU0 : kGenU;
constexpr size_t kLimStage = 4 * (kLimTab + 16);    // the window's averages

// A window that fits the LDS: per window cell j (one a lane) the limited
// slope (PPM: FP64 value, FP32 derivatives with respect to the averages of
// cells j-1 .. j+1; PLM: the van Leer slope in FP64, its derivatives times
// the gap inverses in FP32) from the FP64 mesh weights, loaded once a cell;
// then (PPM) per interface j+1/2 its value in FP64 and its derivatives with
// respect to cells j-1 .. j+2 in FP32; then per node only LDS reads: the
// constraint branch in FP64 from the average and the two interface values,
// the row through the branch, its terms and the destination's whole cells
// into the FP64 accumulator.  Every branch decision takes FP64 values from
// FP64 weights; the FP32 derivatives only scale terms.
template <int R, int NS>
__device__ __forceinline__ void lim_tab_rows(const StepAdjArgs &a, const MeshTab &tb, int n,
                                             int base, int off, int W, int NE, int nd,
                                             int64_t wl, int t, int (&kv)[NS],
                                             int (&kn)[NS], double (&thv)[NS],
                                             double (&hv)[NS], const float *sqw,
                                             const double *smb, double *tI, float4 *tD,
                                             double *cacc, double &vp)
{
    constexpr int LO = LimHalo<R>::lo;
    constexpr int NT = (kLimTab + kLanes - 1) / kLanes;
    auto cell = [&](int j) { const int c = base + j; return c >= n ? c - n : c; };
    auto qa = [&](int j) { return (double)sqw[j + off]; };
    for (int j = t; j < W; j += kLanes) cacc[j] = 0.0;
    // ---- slopes (cells 1 .. W-2) ----------------------------------------------
    double e1v[NT], e2v[NT], e3v[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        const int j = t + s * kLanes;
        e1v[s] = e2v[s] = e3v[s] = 0.0;
        if (j < 1 || j > W - 2) continue;
        const int c = cell(j);
        const double qm = qa(j - 1), q0 = qa(j), qp = qa(j + 1);
        if constexpr (R == kReconPLM) {
            const double gp = tb.hinv[c], gm = tb.hinv[c == 0 ? n - 1 : c - 1];
            const double av = (qp - q0) * gp, bv = (q0 - qm) * gm;
            double sig = 0.0, dsa = 0.0, dsb = 0.0;
            if (av * bv > 0.0) {
                const double inv = 1.0 / (av + bv);
                sig = 2.0 * av * bv * inv;
                dsa = 2.0 * bv * bv * inv * inv;
                dsb = 2.0 * av * av * inv * inv;
            }
            tI[j] = sig;
            tD[j] = make_float4((float)(dsb * gm), (float)(dsa * gp), 0.0f, 0.0f);
        } else {
            const double *pw = tb.ppmd;
            const double d1 = pw[c], d2 = pw[n + c];
            e1v[s] = pw[2 * n + c];
            e2v[s] = pw[3 * n + c];
            e3v[s] = pw[4 * n + c];
            const double up = qp - q0, dn = q0 - qm;
            const double d = d1 * up + d2 * dn;
            double dl = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
            if (up * dn > 0.0) {
                dl = copysign(fmin(fabs(d), 2.0 * fmin(fabs(up), fabs(dn))), d);
                if (fabs(d) <= 2.0 * fabs(up) && fabs(d) <= 2.0 * fabs(dn)) {
                    g0 = -d2;
                    g1 = d2 - d1;
                    g2 = d1;
                } else if (fabs(up) <= fabs(dn)) {
                    g1 = -2.0;                       // twice the upper difference
                    g2 = 2.0;
                } else {
                    g0 = -2.0;                       // twice the lower difference
                    g1 = 2.0;
                }
            }
            tI[j] = dl;
            tD[j] = make_float4((float)g0, (float)g1, (float)g2, 0.0f);
        }
    }
    wave_sync();
    if constexpr (R == kReconPPM) {
        // ---- interfaces j+1/2 (j = 1 .. W-3), replacing the slopes in place --------
        double Iv[NT];
        float4 Dv[NT];
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            const int j = t + s * kLanes;
            Iv[s] = 0.0;
            Dv[s] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j < 1 || j > W - 3) continue;
            const double dl0 = tI[j], dl1 = tI[j + 1];
            const float4 g0 = tD[j], g1 = tD[j + 1];
            const double e1 = e1v[s], e2 = e2v[s], e3 = e3v[s];
            const double q0 = qa(j), q1 = qa(j + 1);
            Iv[s] = q0 + e1 * (q1 - q0) + e2 * dl1 + e3 * dl0;
            Dv[s] = make_float4((float)(e3 * g0.x),
                                (float)(1.0 - e1 + e3 * g0.y + e2 * g1.x),
                                (float)(e1 + e3 * g0.z + e2 * g1.y),
                                (float)(e2 * g1.z));
        }
        wave_sync();
#pragma unroll
        for (int s = 0; s < NT; ++s) {
            const int j = t + s * kLanes;
            if (j < 1 || j > W - 3) continue;
            tI[j] = Iv[s];
            tD[j] = Dv[s];
        }
        wave_sync();
    }
    // ---- nodes (slot 0 each trip, the slots moved down after it) ------------------
#pragma unroll 1
    for (int u = 0; u < NS; ++u) {
        const int m = t + u * kLanes;
        const int k = kv[0], kne = kn[0];
        const double h = hv[0], th = thv[0];
        slot_down(kv);
        slot_down(kn);
        slot_down(hv);
        slot_down(thv);
        if (m >= NE) continue;
        double gw[2 * LO + 1], qval;
        if constexpr (R == kReconPLM) {
            const double sig = tI[k];
            const float4 ab = tD[k];
            const double ks = 0.5 * h * h * (th * th - th);
            gw[0] = -ks * (double)ab.x;
            gw[1] = h * th + ks * ((double)ab.x - (double)ab.y);
            gw[2] = ks * (double)ab.y;
            qval = qa(k) + sig * h * (th - 0.5);
        } else {
            const double av = qa(k);
            const double Lr = tI[k - 1], Rr = tI[k];
            const float4 dL = tD[k - 1], dR = tD[k];
            double L = Lr, Rv = Rr;
            int branch = 0;                          // 1 flat, 2 L pulled in, 3 R pulled in
            if ((Rv - av) * (av - L) <= 0.0) {
                L = av;
                Rv = av;
                branch = 1;
            } else {
                const double dq = Rv - L, qd = av - 0.5 * (L + Rv);
                if (dq * qd > dq * dq / 6.0) { L = 3.0 * av - 2.0 * Rv; branch = 2; }
                else if (-dq * dq / 6.0 > dq * qd) { Rv = 3.0 * av - 2.0 * L; branch = 3; }
            }
            const double q6 = 6.0 * av - 3.0 * (L + Rv);
            qval = L + th * (Rv - L) + q6 * th * (1.0 - th);
            const double th2 = th * th, th3 = th2 * th;
            const double ga = h * (3.0 * th2 - 2.0 * th3);
            const double gl = h * (th - 2.0 * th2 + th3);
            const double gr = h * (th3 - th2);
            double ba = ga, bl = gl, br = gr;
            if (branch == 1) { ba = ga + gl + gr; bl = 0.0; br = 0.0; }
            else if (branch == 2) { ba = ga + 3.0 * gl; bl = 0.0; br = gr - 2.0 * gl; }
            else if (branch == 3) { ba = ga + 3.0 * gr; bl = gl - 2.0 * gr; br = 0.0; }
            // cells k-2 .. k+2: the left interface's derivatives cover k-2 .. k+1,
            // the right one's k-1 .. k+2
            gw[0] = bl * (double)dL.x;
            gw[1] = bl * (double)dL.y + br * (double)dR.x;
            gw[2] = ba + bl * (double)dL.z + br * (double)dR.y;
            gw[3] = bl * (double)dL.w + br * (double)dR.z;
            gw[4] = br * (double)dR.w;
        }
        const double vb = smb[m] - smb[m + 1];
        vp -= vb * qval;
#pragma unroll
        for (int j = 0; j <= 2 * LO; ++j) atomicAdd(&cacc[k - LO + j], vb * gw[j]);
        if (m < nd) {
            // destination m's whole cells: window cells k .. kn - 1
            const double mb = smb[m + 1];
            for (int j = k; j < kne; ++j) {
                const double dxj = j == k ? h : tb.dx[wrapi(wl + j, n)];
                atomicAdd(&cacc[j], mb * dxj);
            }
        }
    }
    wave_sync();
}

// One tile of the limited step backwards (any kind: the uniform runs save
// only the search, every node's Jacobian row is evaluated).
template <int R, bool RES, bool V0>
__device__ __forceinline__ void lim_tile(const StepAdjArgs &a, const FastTile &ft,
                                         unsigned char *su, float *sqw, double *smb, int t)
{
    constexpr int LO = LimHalo<R>::lo;
    constexpr int P = 2 * LO + 1;
    constexpr int NS = (kFastNodes + kLanes - 1) / kLanes;
    constexpr int NG = (kLimTab + 3 + 4 * kLanes - 1) / (4 * kLanes);    // window groups a lane
    constexpr int kCh = (int)(kLimU / 8) - 8;        // window cells a chunk of the accumulator
    const Rows &Rw = a.rows;
    const MeshTab &tb = Rw.tab;
    const int n = (int)Rw.n_cols;
    const int tile = ft.pad[0];
    const TilePos p = tile_pos(tile, n, 0);
    const int i0 = p.i0, nd = p.nd, NE = nd + 1, c4 = 4 * t, cl = min(c4, nd - 4);
    const int64_t qoff = (int64_t)p.row * n;
    const float *qf = (const float *)a.q_fwd + qoff;
    float *qbi = (float *)a.qbar_in + qoff;
    const double *x = Rw.edges;
    const double x0 = x[0], xN = x[n], len = xN - x0;
    const RowShift rs = row_shift(a.v0[p.row] * a.dt, len, tb.scal[1]);
    const bool uniform = ft.kind == kFastUniform;
    // the plan locates the nodes; the window fits the table
    const bool planned =
        uniform || (ft.kind == kFastWindow && ft.base + ft.w + 3 < 2 * n && ft.w <= kFastWin);
    // the window: this tile's first node's stencil up to the next tile's
    // (the row's first tile one period on, for the last tile of a row)
    const int tpr = (n + kFT - 1) / kFT;
    const int64_t wl = rec_wlo(a.fast.rec[tile]);
    const int64_t wend =
        (i0 + nd >= n ? rec_wlo(a.fast.rec[tile - (tpr - 1)]) + n : rec_wlo(a.fast.rec[tile + 1])) +
        P;
    const int W = (int)(wend - wl);
    const bool windowed = planned && W <= kLimTab;
    const int base = ft.base, a0 = base & ~3, off = base - a0;
    const int gl = (W + off - 1) >> 2;

    // ---- 1. the residual's transpose (or the gradient as given): Mbar' in FP64
    const bool want_dvb = RES && a.dvbar != nullptr;
    const ResIn ri = res_load<RES>(a, qoff, n, i0, nd, cl, want_dvb);
    float2 rr[8];
    float dxi[8];
    if constexpr (RES) load_geom(tb, n, i0 + cl - 2, rr, dxi);
    const double2 di01 = *(const double2 *)(tb.dxinv + i0 + cl);
    const double2 di23 = *(const double2 *)(tb.dxinv + i0 + cl + 2);
    float wq[NG][4];
    auto load_win = [&]() {
        if (windowed) {
#pragma unroll
            for (int u = 0; u < NG; ++u) {
                int c = a0 + 4 * min(t + u * kLanes, gl);
                c = c >= n ? c - n : c;
                f4(*(const float4 *)(qf + c), wq[u]);
            }
        }
    };
    res_general<RES>(a, ri, rr, dxi, qoff, i0, nd, cl, t, want_dvb, (float *)su, load_win,
                     [&](const float (&gs)[4]) {
                         const double di[4] = {di01.x, di01.y, di23.x, di23.y};
                         if (c4 < nd) {
#pragma unroll
                             for (int k = 0; k < 4; ++k) smb[1 + c4 + k] = (double)gs[k] * di[k];
                         }
                         if (t == 0) {
                             smb[0] = 0.0;
                             smb[nd + 1] = 0.0;
                         }
                     });
    // the window's averages at j + off (memory-aligned groups as loaded)
    if (windowed) {
#pragma unroll
        for (int u = 0; u < NG; ++u) {
            const int g = t + u * kLanes;
            if (g <= gl)
                *(float4 *)(sqw + 4 * g) = make_float4(wq[u][0], wq[u][1], wq[u][2], wq[u][3]);
        }
    }
    wave_sync();                                     // staging dead; smb, averages visible

    // ---- 2. every node's window index, cell and FP64 position in the cell ---------
    const int16_t *jcp =
        planned && !uniform ? a.fast.jc + (int64_t)ft.pad[1] * kFastNodes : nullptr;
    int kv[NS], cv[NS];
    double thv[NS], hv[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const int m = min(t + u * kLanes, NE - 1);
        const int e = i0 + m;
        const int kx = e >= n ? 1 : 0;
        const NodePos np = node_pos(x[e - kx * n], rs, x0, xN, tb.scal[0], tb.scal[2], tb.nb);
        int c, k;
        if (planned) {
            k = uniform ? LO + m : (int)jcp[m];
            c = base + k;
            c = c >= n ? c - n : c;
        } else {
            const double2 nx = tb.bnext[np.b];
            c = cell_from_bucket(tb.bucket[np.b], nx, np.xt);
            if (np.xt >= nx.y) c = cell_walk(x, n, c, np.xt);
            const int64_t g = (int64_t)c + (rs.kf0 + np.dk + kx) * (int64_t)n;
            k = (int)(g - wl);
        }
        const double h = tb.dx[c];
        double d = np.xt - x[c];
        d = d > 0.5 * len ? d - len : (d < -0.5 * len ? d + len : d);
        kv[u] = k;
        cv[u] = c;
        thv[u] = d * tb.dxinv[c];
        hv[u] = h;
    }
    // the next node's window index (node m + 1: the next lane, lane 63 the next slot's lane 0)
    int kn[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        kn[u] = __shfl_down(kv[u], 1);
        if (u + 1 < NS) {
            const int k0 = __shfl(kv[u + 1 < NS ? u + 1 : u], 0);
            if (t == kLanes - 1) kn[u] = k0;
        }
    }

    double vp = 0.0;
    float *edge = (float *)a.edge + (int64_t)tile * (2 * P);
    if (windowed) {
        lim_tab_rows<R>(a, tb, n, base, off, W, NE, nd, wl, t, kv, kn, thv, hv, sqw, smb,
                        (double *)su, (float4 *)(su + kLimTabI),
                        (double *)(su + kLimTabI + kLimTabD), vp);
        const double *cacc = (const double *)(su + kLimTabI + kLimTabD);
        for (int j = t; j < W; j += kLanes)
            put_cell<P>(qbi, edge, wrapi(wl + j, n), j, W, (float)cacc[j]);
        if constexpr (V0) {
            vp = wave_sum(vp);
            if (t == 0) a.v0part[tile] = a.dt * vp;
        }
        return;
    }

    // ---- 3. Jacobian rows through Vbar, and the whole cells, chunk by chunk -------
    // (one node slot at a time: each row is a long FP64 chain; v0bar as
    // -sum_e Vbar_e q~_e, one term a node)
    double *cacc = (double *)su;
    for (int c0 = 0; c0 < W; c0 += kCh) {
        const int cw = min(kCh, W - c0);
        for (int j = t; j < cw; j += kLanes) cacc[j] = 0.0;
        wave_sync();
        int ku[NS], cu[NS], knu[NS];
        double hu[NS], thu[NS];
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            ku[u] = kv[u];
            cu[u] = cv[u];
            knu[u] = kn[u];
            hu[u] = hv[u];
            thu[u] = thv[u];
        }
#pragma unroll 1
        for (int u = 0; u < NS; ++u) {
            const int m = t + u * kLanes;
            const int k = ku[0], c = cu[0], kne = knu[0];
            const double h = hu[0], th = thu[0];
            slot_down(ku);
            slot_down(cu);
            slot_down(knu);
            slot_down(hu);
            slot_down(thu);
            double qv[P];
#pragma unroll
            for (int j = 0; j < P; ++j) {
                if (windowed) {
                    qv[j] = (double)sqw[k - LO + j + off];
                } else {
                    int mm = c - LO + j;
                    mm = mm < 0 ? mm + n : (mm >= n ? mm - n : mm);
                    qv[j] = (double)qf[mm];
                }
            }
            double gw[P], qval;
            lim_node<R>(tb, n, c, h, th, qv, gw, qval);
            if (m < NE) {
                const double vb = smb[m] - smb[m + 1];
                if (c0 == 0) vp -= vb * qval;
#pragma unroll
                for (int j = 0; j < P; ++j) {
                    const int jj = k - LO + j - c0;
                    if (jj >= 0 && jj < cw) atomicAdd(&cacc[jj], vb * gw[j]);
                }
                // destination m's whole cells: window cells k .. kn - 1
                if (m < nd) {
                    const double mb = smb[m + 1];
                    for (int j = max(k, c0); j < min(kne, c0 + cw); ++j) {
                        const double dxj = j == k ? h : tb.dx[wrapi(wl + j, n)];
                        atomicAdd(&cacc[j - c0], mb * dxj);
                    }
                }
            }
        }
        wave_sync();
        for (int j = t; j < cw; j += kLanes)
            put_cell<P>(qbi, edge, wrapi(wl + c0 + j, n), c0 + j, W, (float)cacc[j]);
        wave_sync();
    }
    if constexpr (V0) {
        vp = wave_sum(vp);
        if (t == 0) a.v0part[tile] = a.dt * vp;
    }
}

// Every tile in tile order, one a workgroup of one wave (the LDS a tile
// needs, not four tiles' worth, sets how many share a CU).
template <int R, bool RES, bool V0>
__global__ __launch_bounds__(kLanes) void k_ladj(StepAdjArgs a)
{
    __shared__ __attribute__((aligned(16))) unsigned char su[kLimU];
    __shared__ __attribute__((aligned(16))) float sqw[kLimStage / 4];
    __shared__ __attribute__((aligned(16))) double smb[kFT + 8];
    const int i = (int)blockIdx.x;
    if (i >= (int)a.rows.n_tiles) return;
    const FastTile r = load_rec(a.fast.rec, i);
    lim_tile<R, RES, V0>(a, r, su, sqw, smb, (int)threadIdx.x);
}

template <int R, bool RES, bool V0>
hipError_t ladj_kernels(const StepAdjArgs &a, hipStream_t st)
{
    constexpr int P = 2 * LimHalo<R>::lo + 1;
    const int64_t nt = a.rows.n_tiles;
    hipLaunchKernelGGL((k_ladj<R, RES, V0>), dim3((unsigned)nt), dim3(kLanes), 0, st, a);
    hipLaunchKernelGGL((k_adjf_edges<P>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !V0) return e;
    return launch_v0_reduce(a.rows, a.v0part, a.v0bar, st);
}

template <int R>
hipError_t ladj_r(const StepAdjArgs &a, hipStream_t st)
{
    const bool v0 = a.v0bar != nullptr;
    if (a.dv) return v0 ? ladj_kernels<R, true, true>(a, st) : ladj_kernels<R, true, false>(a, st);
    return v0 ? ladj_kernels<R, false, true>(a, st) : ladj_kernels<R, false, false>(a, st);
}

// The uniform tiles (the compacted list's first part), one a wave.
template <int P, bool RES, bool V0>
__global__ __launch_bounds__(kBlock) void k_adjf_uni(StepAdjArgs a)
{
    __shared__ __attribute__((aligned(16))) float su[kWaves][3 * kStage];
    const int wid = wave_id();
    const int i = (int)blockIdx.x * kWaves + wid;
    if (i >= a.fast.totals[0]) return;
    const FastTile r = load_rec(a.fast.rec + a.rows.n_tiles, i);
    adj_uniform_tile<P, RES, V0>(a, r, su[wid], (int)threadIdx.x % kLanes);
}

// The other tiles: waves stepping through the rest of the list.
template <int P, bool RES, bool V0>
__global__ __launch_bounds__(kBlock) void k_adjf_gen(StepAdjArgs a)
{
    __shared__ __attribute__((aligned(16))) unsigned char su[kWaves][kGenU];
    __shared__ __attribute__((aligned(16))) float smb[kWaves][kFT + 8];
    const int wid = wave_id();
    const int nt = (int)a.rows.n_tiles;
    const int n = (int)a.rows.n_cols;
    const int t = (int)threadIdx.x % kLanes;
    const int stride = (int)gridDim.x * kWaves;
    for (int i = a.fast.totals[0] + (int)blockIdx.x * kWaves + wid; i < nt; i += stride) {
        const FastTile r = load_rec(a.fast.rec + nt, i);
        if (r.kind == kFastWindow && r.base + r.w + 3 < 2 * n)
            adj_window_tile<P, RES, V0>(a, r, su[wid], smb[wid], t);
        else
            adj_direct_tile<P, RES, V0>(a, r, su[wid], smb[wid], t);
        wave_sync();                                 // the next tile reuses the LDS
    }
}

template <int P, bool RES, bool V0>
hipError_t adjf_kernels(const StepAdjArgs &a, hipStream_t st)
{
    const int64_t nt = a.rows.n_tiles;
    const dim3 b(kBlock);
    const dim3 gu((unsigned)((nt + kWaves - 1) / kWaves));
    const dim3 gg((unsigned)((nt + kWaves * kGenShareA - 1) / (kWaves * kGenShareA)));
    if (const ForkJoin *fj = capture_fork) {
        // inside a captured loop: the two kinds of tile (disjoint outputs and
        // partials) as parallel graph branches, joined before the edges pass
        hipError_t e = hipEventRecord(fj->fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(fj->side, fj->fork, 0);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_adjf_gen<P, RES, V0>), gg, b, 0, fj->side, a);
        e = hipEventRecord(fj->join, fj->side);
        hipLaunchKernelGGL((k_adjf_uni<P, RES, V0>), gu, b, 0, st, a);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, fj->join, 0);
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL((k_adjf_uni<P, RES, V0>), gu, b, 0, st, a);
        hipLaunchKernelGGL((k_adjf_gen<P, RES, V0>), gg, b, 0, st, a);
    }
    hipLaunchKernelGGL((k_adjf_edges<P>), dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !V0) return e;
    return launch_v0_reduce(a.rows, a.v0part, a.v0bar, st);
}

template <int P>
hipError_t adjf_p(const StepAdjArgs &a, hipStream_t st)
{
    const bool v0 = a.v0bar != nullptr && a.q_fwd != nullptr;
    if (a.dv) return v0 ? adjf_kernels<P, true, true>(a, st) : adjf_kernels<P, true, false>(a, st);
    return v0 ? adjf_kernels<P, false, true>(a, st) : adjf_kernels<P, false, false>(a, st);
}

} // namespace

hipError_t launch_step_limited_adjoint_fast(const StepAdjArgs &a, int recon, hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    if (a.rows.tile != kFastTile || a.rows.n_cols % 4 != 0 || a.rows.n_cols < kFastTile + 8 ||
        a.rows.n_tiles > INT32_MAX / 2 || !a.edge || !a.q_fwd)
        return hipErrorInvalidValue;
    return recon == kReconPLM ? ladj_r<kReconPLM>(a, stream) : ladj_r<kReconPPM>(a, stream);
}

hipError_t launch_step_adjoint_fast(const StepAdjArgs &a, int order, hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    if (a.rows.tile != kFastTile || a.rows.n_cols % 4 != 0 || a.rows.n_cols < kFastTile + 8 ||
        a.rows.n_tiles > INT32_MAX / 2 || !a.edge)
        return hipErrorInvalidValue;
    switch (order) {
    case 1: return adjf_p<1>(a, stream);
    case 3: return adjf_p<3>(a, stream);
    default: return adjf_p<5>(a, stream);
    }
}

} // namespace ram
