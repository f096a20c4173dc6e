// ram_step_fast.hip -- the FP32 RAM step on rows that share one mesh, with the
// cumulative differences summed directly from the window masses (gfx950).
//
// Same computation as k_step_sh with direct sums (bulk shift of Section 3,
// Steps 1-3, Eqs. Qmass_i, condition_p, mass_shift_algo, step3, then the
// residual upwind step with the van Leer slope of Section 3.1), laid out for
// streaming rather than for the node search:
//
//   * one tile of kFastTile = 256 destination cells per wave, four
//     consecutive cells a lane, whose residual-velocity loads and final
//     stores are 16-byte vector accesses; each wave has its own LDS and never
//     waits on the other waves of its workgroup (no workgroup barrier);
//   * everything about a tile that does not change between steps is planned
//     once per call: its source window, whether it lies in one of the mesh's
//     uniform runs (then the stencil weights and the run's geometry), the
//     records sorted into the uniform tiles and the others, and for the
//     others each shifted node's window index and position in its cell;
//   * a tile in a uniform run (every node of the tile in the next source cell
//     at one theta) needs no search and no masses: the shifted value of a
//     cell is a fixed (P+1)-point stencil on the window's cell values.  Those
//     tiles run in their own kernel (k_step_uni, 26 registers, eight waves a
//     SIMD) as straight-line code: the window and face loads issued together,
//     the window through the wave's LDS once, each lane reading the thirteen
//     values its eight cells need (its four and the residual's two-cell halo
//     a side) with 16-byte LDS reads, and the residual on registers;
//   * the other tiles (k_step_gen) stage the window masses M = Q dx in LDS,
//     read their nodes' planned window index and theta, then each node's
//     stencil record for its Lagrange weights and partial integral, then the
//     destination masses one cell per lane, and the same register residual on
//     four consecutive cells; a tile whose window exceeds the LDS capacity
//     sums from global memory.
// Tiles of 256 cells keep the searching tiles to the cells near the mesh's
// non-uniform stretches.
#include "ram_device.h"
#include "ram_wave.h"

#include <type_traits>

namespace ram {
namespace {

using namespace dev;

constexpr int kFT = kFastTile;                      // destination cells per tile (wave)
constexpr int kFPad = 16;                           // slack for vector over-reads

// LDS of one wave.  The window (values or masses), the direct path's extended
// node indices and the shifted state share bytes (the wave moves from one to
// the next after a wave-level fence); node partials and their window indices
// have arrays of their own.
struct WaveLds {
    static constexpr int nodes = kFT + 5 + 3;       // up to 261 nodes, padded
    static constexpr size_t win = sizeof(float) * (kFastWin + kFPad);
    static constexpr size_t gidx = sizeof(int64_t) * nodes;
    static constexpr size_t shifted = sizeof(float) * (kFT + 4 + kFPad);
    static constexpr size_t u0 = win > gidx ? win : gidx;
    static constexpr size_t u = u0 > shifted ? u0 : shifted;
    // the prefix modes keep the window's cumulative (8-byte values: FP64, or
    // a two-sum pair) instead of its masses
    static constexpr size_t pre = 8 * (kFastWin + 16);
    static constexpr size_t u_pre = pre > u ? pre : u;
};
template <int S> constexpr size_t wave_lds_bytes()
{
    return S == kSumDirect ? WaveLds::u : WaveLds::u_pre;
}


// The record of one tile: which path, its window, and for a uniform tile the
// stencil and the run's geometry.  One thread per tile; the node search is the
// shared-mesh one of the step kernels (bucket index, Eq. condition_p).
template <int P>
__global__ __launch_bounds__(64) void k_plan_fast(StepArgs a, FastTile *out)
{
    constexpr int LO = (P - 1) / 2;
    const int64_t tile = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const Rows &R = a.rows;
    if (tile >= R.n_tiles) return;
    const int n = (int)R.n_cols;
    const int64_t tpr = (n + kFT - 1) / kFT;
    const int64_t row = tile / tpr;
    const int i0 = (int)(tile - row * tpr) * kFT;
    const int H = a.dv ? 2 : 0;
    const int nd = min(kFT, n - i0);
    const double *x = R.edges;
    const double len = x[n] - x[0];
    const RowShift rs = row_shift(a.v0[row] * a.dt, len, R.tab.scal[1]);
    double xt0;
    int c0;
    const int64_t g0 = node_locate(x, n, R.tab, rs, i0 - H, xt0, c0);
    const int64_t g1 = node_index(x, n, R.tab, rs, len, i0 + nd + H);
    const int64_t wide = g1 - g0 + P;
    const int64_t wlo = g0 - LO;
    FastTile ft;
    ft.kind = kFastWindow;
    ft.w = (wide >= P && wide <= kFastWin) ? (int)wide : -1;
    const int64_t kk = wlo >= 0 ? wlo / n : -((-wlo + n - 1) / n);
    ft.base = (int)(wlo - kk * n);
    ft.wlo_lo = (int32_t)(uint32_t)((uint64_t)wlo & 0xffffffffull);
    ft.wlo_hi = (int32_t)((uint64_t)wlo >> 32);
    for (int d = 0; d < 6; ++d) ft.cc[d] = 0.0f;
    ft.dx = ft.hinv = ft.dxinv = 0.0f;
    ft.pad[0] = (int32_t)tile;
    ft.pad[1] = -1;
    if (ft.w < 0) ft.kind = kFastDirect;
    // uniform: the cells on both sides of the tile's nodes and its whole source
    // window lie in one uniform run of the mesh, and the window holds one
    // source cell per node plus the stencil, so node i0 - H + k sits in window
    // cell LO + k at the first node's theta (rows shorter than a full tile's
    // window stay with the other kernel, whose windows may wrap many times)
    auto in_run = [&](const int32_t *pre) {
        return nonu_count(pre, n, i0 - H - 1, i0 + nd + H + 1) == 0 &&
               nonu_count(pre, n, wlo, wlo + wide) == 0;
    };
    if (ft.kind == kFastWindow && R.tab.nonu && wide == nd + 2 * H + P &&
        n >= kFT + 2 * H + P && (in_run(R.tab.nonu) || in_run(R.tab.nonu_min))) {
        ft.kind = kFastUniform;
        const double th = (xt0 - x[c0]) * R.tab.dxinv[c0];
        double cc[P + 1];
        uniform_stencil<double, P>(th, cc);
        for (int d = 0; d <= P; ++d) ft.cc[d] = (float)cc[d];
        ft.pad[1] = __float_as_int((float)th);
        const float2 rr = R.tab.rrf[i0];
        ft.dx = rr.x;
        ft.hinv = rr.y;
        ft.dxinv = R.tab.dxinvf[i0];
    }
    out[tile] = ft;
}


// Residual step on four consecutive cells of a lane from the shifted state
// s[0..7] of cells i0+4l-2 .. i0+4l+5 (Section 3.1's upwind step with the van
// Leer slope, the face state the upwind linear profile averaged over the
// interval the face velocity sweeps in dt): fluxes on the
// five faces i0+4l .. i0+4l+4 with the upwind cell's van Leer slope and the
// swept-interval average, then the conservative update of the four cells.
// rr(c) gives (dx, 1/centre gap to the right) of s-index c, dxi(k) 1/dx of
// own cell k.
template <typename RR, typename DXI>
__device__ __forceinline__ void residual4(const float *s, const float *dvv, float dt, RR rr,
                                          DXI dxi, float *out)
{
    float F[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const float v = dvv[k];
        const bool up = v >= 0.0f;
        // upwind cell: s-index k+1 (left of the face) or k+2
        const float qm = up ? s[k] : s[k + 1];
        const float q0 = up ? s[k + 1] : s[k + 2];
        const float qp = up ? s[k + 2] : s[k + 3];
        const float2 rc = up ? rr(k + 1) : rr(k + 2);
        const float gm = up ? rr(k).y : rr(k + 1).y;
        const float dp = (qp - q0) * rc.y;
        const float dm = (q0 - qm) * gm;
        const float sig = (dp * dm <= 0.0f) ? 0.0f : harmonic2(dp, dm);
        const float half = up ? 0.5f * (rc.x - v * dt) : -0.5f * (rc.x + v * dt);
        F[k] = v * (q0 + sig * half);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = s[k + 2] - dt * (F[k + 1] - F[k]) * dxi(k);
}


// Residual velocity of faces i0+4l .. i0+4l+4 of a row (face n is face 0);
// lanes past the tile read its last faces again (every load issued, no
// branch).
template <bool VEC>
__device__ __forceinline__ void load_faces(const float *dvp, int n, int i0, int nd, int c4,
                                           float *dvv)
{
    const int cc = min(c4, nd - 1);
    if constexpr (VEC) {
        const float4 v4 = ld_at<float4>(dvp + i0, 4u * (uint32_t)(cc & ~3));
        dvv[0] = v4.x;
        dvv[1] = v4.y;
        dvv[2] = v4.z;
        dvv[3] = v4.w;
    } else {
        // faces up to the tile's right face i0 + nd
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int f = i0 + min(cc + k, nd);
            dvv[k] = dvp[f >= n ? f - n : f];
        }
    }
    const int f4 = i0 + min(cc + 4, nd);
    dvv[4] = dvp[f4 >= n ? f4 - n : f4];
}

template <bool VEC>
__device__ __forceinline__ void store_cells(float *qo, int i0, int nd, int c4, const float *o)
{
    if (c4 >= nd) return;
    if constexpr (VEC) {
        st_at<float4>(qo + i0, 4u * (uint32_t)c4, make_float4(o[0], o[1], o[2], o[3]));
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (c4 + k < nd) qo[i0 + c4 + k] = o[k];
    }
}



// ---------------------------------------------------------------------------
// A tile in a uniform run of the mesh: straight-line code (clamped indices
// instead of guards), the window's and the faces' loads issued together.
// ---------------------------------------------------------------------------

constexpr int kUniWin = 5 * kLanes + 16;            // window slots + over-read slack, floats

// A tile in a uniform run.  VEC: rows of a multiple of four cells (16-byte
// aligned vector loads of the residual velocity, vector stores of the
// result).  Rows need at least kFT + 2H + P cells (k_plan_fast sends shorter
// ones to the other path), so a window wraps the row at most once.
template <int P, int H, bool VEC>
__device__ __forceinline__ void uniform_tile(const StepArgs &a, const FastTile &r, float *sw,
                                             int t)
{
    constexpr int NV = 4 + 2 * H;                    // shifted cells a lane reads
    constexpr int NW = (NV + P + 3) / 4 * 4;         // window values, whole float4s
    constexpr int NUW = (kFT + 2 * H + P + kLanes - 1) / kLanes;  // window slots a lane
    static_assert(NUW * kLanes <= kUniWin && 4 * (kLanes - 1) + NW <= kUniWin, "window");
    const int n = (int)a.rows.n_cols;
    const float dt = (float)a.dt;
    const int c4 = 4 * t;
    const TilePos p = tile_pos(r.pad[0], n, H);
    const int64_t qoff = (int64_t)p.row * n;

    // window cells j = t + 64k (clamped into the window: the extra lanes read
    // its last cell again) and face velocities i0+4l .. i0+4l+4 (clamped into
    // the tile, face n is face 0)
    float wv[NUW];
    {
        const float *q = (const float *)a.q_in + qoff;
#pragma unroll
        for (int k = 0; k < NUW; ++k) {
            int mm = r.base + min(t + k * kLanes, r.w - 1);
            mm = mm >= n ? mm - n : mm;
            wv[k] = q[mm];
        }
    }
    float dvv[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if constexpr (H != 0) load_faces<VEC>((const float *)a.dv + qoff, n, p.i0, p.nd, c4, dvv);
#pragma unroll
    for (int k = 0; k < NUW; ++k) sw[t + k * kLanes] = wv[k];
    wave_sync();
    // shifted cells ci = 4l .. 4l+NV-1 of the tile (cell i0-H+ci) from window
    // cells ci .. ci+P
    float win[NW];
#pragma unroll
    for (int v = 0; v < NW / 4; ++v) {
        const float4 w4 = *(const float4 *)(sw + c4 + 4 * v);
        win[4 * v] = w4.x;
        win[4 * v + 1] = w4.y;
        win[4 * v + 2] = w4.z;
        win[4 * v + 3] = w4.w;
    }
    float s[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) {
        float v = 0.0f;
#pragma unroll
        for (int d = 0; d <= P; ++d) v += r.cc[d] * win[c + d];
        s[c] = v;
    }
    float *qo = (float *)a.q_out + qoff;
    if constexpr (H == 0) {
        store_cells<VEC>(qo, p.i0, p.nd, c4, s);
    } else {
        if (a.q_mid && c4 < p.nd) {
            float *qm = (float *)a.q_mid + qoff;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (c4 + k < p.nd) qm[p.i0 + c4 + k] = s[k + 2];
        }
        const float2 g = make_float2(r.dx, r.hinv);
        const float dxi = r.dxinv;
        float o[4];
        residual4(s, dvv, dt, [&](int) { return g; }, [&](int) { return dxi; }, o);
        store_cells<VEC>(qo, p.i0, p.nd, c4, o);
    }
}

// ---------------------------------------------------------------------------
// Every other tile.  Its nodes' source cells do not change between the steps
// of a call, so k_node_plan locates them once (bucket index, Eq.
// condition_p) and keeps each node's window index and theta; per step a wave
// then needs two round trips to memory: the window, node data, faces and
// geometry together, then the source cells' stencil records.
// ---------------------------------------------------------------------------

// The k-th non-uniform tile's nodes (k = list position - totals[0]): window
// index and FP32 theta of nodes i0-H .. i0+nd+H, and in the slots past the
// last node (up to kFastNodes) the last node again, so that whole 16-byte
// groups of slots can be read; a node outside the window (not expected: the
// plan sized it from the end nodes) turns the tile into a direct one, in both
// copies of its record.  One wave per tile.
template <int P>
__global__ __launch_bounds__(kBlock) void k_node_plan(StepArgs a)
{
    constexpr int LO = (P - 1) / 2;
    constexpr int NS = (kFastNodes + kLanes - 1) / kLanes;
    const Rows &R = a.rows;
    const int nu = a.fast.totals[0];
    const int nt = (int)R.n_tiles;
    const int k = (int)blockIdx.x * kWaves + wave_id();
    if (nu + k >= nt) return;
    FastTile *crec = a.fast.rec + nt;
    const FastTile ft = load_rec(crec, nu + k);
    if (ft.kind != kFastWindow) return;
    const int H = a.dv ? 2 : 0;
    const int t = threadIdx.x % kLanes;
    const MeshTab &tb = R.tab;
    const int n = (int)R.n_cols;
    const TilePos tp = tile_pos(ft.pad[0], n, H);
    const int NE = tp.nd + 2 * H + 1;
    const double *x = R.edges;
    const double x0 = x[0], xN = x[n];
    const double len = xN - x0;
    const RowShift rs = row_shift(a.v0[tp.row] * a.dt, len, tb.scal[1]);
    const int64_t wlo = (int64_t)(((uint64_t)(uint32_t)ft.wlo_hi << 32) | (uint32_t)ft.wlo_lo);
    const int jbase = (int)(rs.kf0 * (int64_t)n - wlo);
    float *th = a.fast.theta + (int64_t)k * kFastNodes;
    int16_t *jcw = a.fast.jc + (int64_t)k * kFastNodes;
    bool ok = true;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int m = t + s * kLanes;
        if (m < kFastNodes) {
            int e = tp.i0 - H + min(m, NE - 1);
            const int kx = e < 0 ? -n : (e >= n ? n : 0);
            e -= kx;
            const NodePos np = node_pos(x[e], rs, x0, xN, tb.scal[0], tb.scal[2], tb.nb);
            const double2 nx = tb.bnext[np.b];
            int c = cell_from_bucket(tb.bucket[np.b], nx, np.xt);
            if (np.xt >= nx.y) c = cell_walk(x, n, c, np.xt);
            const CellRec<float> &rc = RecT<float>::get(tb)[c];
            const int j = c + np.dk * n + kx + jbase;
            ok = ok && j >= LO && j + P - LO <= ft.w;
            th[m] = (float)((np.xt - rc.xc) * rc.dxinv);
            jcw[m] = (int16_t)min(max(j, 0), kFastWin);
        }
    }
    if (!__all(ok ? 1 : 0) && t == 0) {
        a.fast.rec[ft.pad[0]].kind = kFastDirect;
        crec[nu + k].kind = kFastDirect;
    }
}

// LDS window of the limited step's searching tiles, in cells: four arrays of
// it (masses; averages, later the cubics' C; slopes or PLM kappa, later A;
// PPM interface values).  Wider windows take the global-memory path.
constexpr int kGenLimWin = 400;
constexpr size_t kGenLimLds = 4 * sizeof(float) * (kGenLimWin + 8);

// A searching tile's window for the limited step (Section 3.1, App. A): the
// window's masses and averages in LDS, then one pass a stage over the window
// cells -- the limited slopes (PPM; PLM: kappa = sigma dx^2 / 2), the PPM
// interface values, each cell's constrained parabola as the cubic
// ell(theta) = theta (A + theta (B + theta C)), B = M - A - C -- with the
// mesh's weights of each cell, then each node's cubic at its planned theta.
// Node m's window index goes to sjc[m], its partial integral to sell[m].
template <int LR, int NS>
__device__ __forceinline__ void lim_window_partials(const StepArgs &a, const MeshTab &tb, int n,
                                                    int base, int W, int NE, int64_t qoff,
                                                    int t, const float (&thv)[NS],
                                                    const int (&jv)[NS], float *su,
                                                    float *sell, short *sjc)
{
    constexpr int CAP = kGenLimWin + 8;
    float *sw = su;                                  // masses
    float *sq = su + CAP;                            // averages, then C
    float *sd = su + 2 * CAP;                        // slopes or kappa, then A
    float *si = su + 3 * CAP;                        // PPM interface values
    const float *q = (const float *)a.q_in + qoff;
    auto cell = [&](int j) { const int c = base + j; return c >= n ? c - n : c; };
    for (int j = t; j < W; j += kLanes) {
        const int c = cell(j);
        const float qv = q[c];
        sq[j] = qv;
        sw[j] = qv * tb.dxf[c];
    }
    wave_sync();
    const float *pw = tb.ppmf;
    for (int j = t; j < W; j += kLanes) {
        if (j < 1 || j > W - 2) continue;
        const int c = cell(j);
        if constexpr (LR == kReconPPM) {
            sd[j] = ppm_delta<float>(sq[j - 1], sq[j], sq[j + 1], pw[c], pw[n + c]);
        } else {
            const float gp = tb.hinvf[c], gm = tb.hinvf[c == 0 ? n - 1 : c - 1];
            const float dp = (sq[j + 1] - sq[j]) * gp, dm = (sq[j] - sq[j - 1]) * gm;
            const float sig = (dp * dm <= 0.0f) ? 0.0f : harmonic2(dp, dm);
            const float h = tb.dxf[c];
            sd[j] = 0.5f * sig * h * h;
        }
    }
    wave_sync();
    if constexpr (LR == kReconPPM) {
        // interface values between window cells j and j+1, j = 1 .. W-3
        for (int j = t; j < W; j += kLanes) {
            if (j < 1 || j > W - 3) continue;
            const int c = cell(j);
            si[j] = sq[j] + pw[2 * n + c] * (sq[j + 1] - sq[j]) + pw[3 * n + c] * sd[j + 1] +
                    pw[4 * n + c] * sd[j];
        }
        wave_sync();
        // constrained parabolas of window cells 2 .. W-3: A into sd, C into sq
        for (int j = t; j < W; j += kLanes) {
            if (j < 2 || j > W - 3) continue;
            float pa, pb, pc;
            ppm_cubic<float>(sq[j], si[j - 1], si[j], tb.dxf[cell(j)], pa, pb, pc);
            sd[j] = pa;
            sq[j] = pc;
        }
        wave_sync();
    }
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const int m = min(t + u * kLanes, NE - 1);
        const int k = jv[u];
        const float th = thv[u];
        float ell;
        if constexpr (LR == kReconPPM) {
            const float pa = sd[k], pc = sq[k];
            const float pb = sw[k] - pa - pc;
            ell = th * (pa + th * (pb + th * pc));
        } else {
            const float kap = sd[k];
            ell = th * (sw[k] - kap + th * kap);
        }
        sell[m] = ell;
        sjc[m] = (short)k;
    }
    wave_sync();
}

// LR != 0: the limited reconstruction LR (PLM / PPM, P its plan order): a
// window of at most kGenLimWin cells is tabulated in LDS (lim_window_partials,
// su then holds kGenLimLds bytes); wider ones take the global-memory path,
// each node's partial integral the limited profile of its cell (Section 3.1).
template <int P, int H, bool VEC, int LR = 0>
__device__ __forceinline__ void general_tile(const StepArgs &a, const FastTile &ft,
                                             unsigned char *su, float *sell, short *sjc, int t)
{
    constexpr int LO = (P - 1) / 2;
    constexpr int NV = 4 + 2 * H;                    // shifted cells a lane reads
    constexpr int NCS = (kFT + 2 * H + kLanes - 1) / kLanes;      // cell slots
    constexpr int NS = (kFT + 2 * H + 1 + kLanes - 1) / kLanes;   // node slots
    const Rows &R = a.rows;
    float *sw = (float *)su;                         // window masses
    int64_t *sg = (int64_t *)su;                     // direct path: node indices
    float *sq = (float *)su;                         // shifted state
    const int k = ft.pad[1];                         // position among the other tiles
    const MeshTab &tb = R.tab;
    const int n = (int)R.n_cols;
    const int c4 = 4 * t;
    const float dt = (float)a.dt;
    const TilePos tp = tile_pos(ft.pad[0], n, H);
    const int row = tp.row, i0 = tp.i0, nd = tp.nd;
    const bool inner = tp.inner;
    const int NC = nd + 2 * H;
    const int NE = NC + 1;
    const int64_t qoff = (int64_t)row * n;
    const float *q = (const float *)a.q_in + qoff;
    float *qo = (float *)a.q_out + qoff;
    float *qmid = a.q_mid ? (float *)a.q_mid + qoff : nullptr;
    const int W = ft.w, base = ft.base;
    const bool windowed = ft.kind == kFastWindow &&
                          (LR == 0 || (ft.w <= kGenLimWin && ft.w + ft.base <= 2 * n));

    if (windowed) {
        // ---- round trip 1: window masses, the nodes' window index and theta
        const float *thp = a.fast.theta + (int64_t)k * kFastNodes;
        const int16_t *jcp = a.fast.jc + (int64_t)k * kFastNodes;
        float thv[NS];
        int jv[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int m = min(t + s * kLanes, NE - 1);
            thv[s] = thp[m];
            jv[s] = jcp[m];
        }
        if constexpr (LR != 0) {
            lim_window_partials<LR, NS>(a, tb, n, base, W, NE, qoff, t, thv, jv, (float *)su,
                                        sell, sjc);
        } else {
        // window masses M = Q dx, four slots of loads at a time, every load
        // issued (clamped into the window) so that no per-slot branch makes
        // the wave wait for each load in turn
        const int nws = (W + kLanes - 1) / kLanes;
        if (W + base <= 2 * n) {
            for (int r0 = 0; r0 < nws; r0 += 4) {
                float wq[4], wd[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    int mm = base + min(t + (r0 + u) * kLanes, W - 1);
                    mm = mm >= n ? mm - n : mm;
                    wq[u] = q[mm];
                    wd[u] = tb.dxf[mm];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (r0 + u < nws) sw[t + (r0 + u) * kLanes] = wq[u] * wd[u];
            }
        } else {
            // rows shorter than the window: it wraps several times
            for (int j = t; j < W; j += kLanes) {
                const int mm = wrap_small(base + j, n);
                sw[j] = q[mm] * tb.dxf[mm];
            }
        }
        wave_sync();
        // ---- round trip 2: each node's stencil record, then its partial
        // integral C~(x) - C(c) from the masses between (summed outward)
        // (the lanes past the last node repeat it: same values, same LDS slot)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int m = min(t + s * kLanes, NE - 1);
            {
                const int j = jv[s];
                int c = base + j;
                c = c >= n ? c - n : c;
                c = c >= n ? wrap_small(c, n) : c;
                const CellRec<float> &rc = RecT<float>::get(tb)[c];
                float wk[P + 1];
                {
                    const float th = thv[s];
                    float tt[P + 1], pre[P + 1], suf[P + 1];
#pragma unroll
                    for (int b = 0; b <= P; ++b) tt[b] = th - rc.th[b];
                    pre[0] = 1.0f;
#pragma unroll
                    for (int b = 1; b <= P; ++b) pre[b] = pre[b - 1] * tt[b - 1];
                    suf[P] = 1.0f;
#pragma unroll
                    for (int b = P - 1; b >= 0; --b) suf[b] = suf[b + 1] * tt[b + 1];
#pragma unroll
                    for (int b = 0; b <= P; ++b) wk[b] = rc.rd[b] * (pre[b] * suf[b]);
                }
                float ell = 0.0f, up = 0.0f, dn = 0.0f;
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
                sell[m] = ell;
                sjc[m] = (short)j;
            }
        }
        wave_sync();
        }
    } else {
        // window wider than the LDS buffer: nodes located here, partial
        // integrals and whole-cell sums from global memory, in FP64
        const double *x = R.edges;
        const double x0 = x[0], xN = x[n];
        const double len = xN - x0;
        const double sh = a.v0[row] * a.dt;
        const RowShift rs = row_shift(sh, len, tb.scal[1]);
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
            if constexpr (LR == kReconPPM)
                sell[m] = (float)ppm_partial_tab<float>(tb, x, q, n, c, np.xt);
            else if constexpr (LR == kReconPLM)
                sell[m] = (float)lim_partial_global<float, LR>(x, q, n, c, np.xt);
            else
                sell[m] = (float)direct_partial<float, P>(x, q, n, len, sh, tb.scal[1], i0 - H + m, g);
        }
        wave_sync();
    }

    // ---- destination cells, one per lane: whole cells + two partials, / dx --
    // (the lanes past the last cell repeat it: same values, same places)
    float qs[NCS];
#pragma unroll
    for (int kk = 0; kk < NCS; ++kk) {
        const int ci = min(t + kk * kLanes, NC - 1);
        {
            const int c0 = i0 - H + ci;
            const int cell = inner ? c0 : wrap1f(c0, n);
            float mp;
            if (windowed) {
                const int ja = sjc[ci], jb = sjc[ci + 1];
                const float m0 = sw[ja], m1 = sw[ja + 1];
                float whole = jb > ja ? m0 : 0.0f;
                whole += jb > ja + 1 ? m1 : 0.0f;
                for (int mm = ja + 2; mm < jb; ++mm) whole += sw[mm];
                mp = whole + (sell[ci + 1] - sell[ci]);
            } else {
                mp = (float)(direct_whole<float>(R.edges, q, n, sg[ci], sg[ci + 1]) +
                             ((double)sell[ci + 1] - (double)sell[ci]));
            }
            qs[kk] = mp * tb.dxinvf[cell];
            if constexpr (H == 0) qo[cell] = qs[kk];
            else if (qmid && ci >= H && ci < H + nd) qmid[cell] = qs[kk];
        }
    }
    if constexpr (H != 0) {
        float dvv[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
        load_faces<VEC>((const float *)a.dv + qoff, n, i0, nd, c4, dvv);
        // per-cell geometry of cells i0+4l-2 .. i0+4l+5: (dx, 1/gap), and 1/dx
        // of the four own cells
        float2 rrv[NV];
        float dxi[4];
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            const int cg = i0 + min(c4, nd - 1) - 2 + c;
            rrv[c] = tb.rrf[wrap1f(cg, n)];
        }
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) dxi[kk] = tb.dxinvf[min(i0 + c4 + kk, n - 1)];
        wave_sync();                                 // the window is dead
#pragma unroll
        for (int kk = 0; kk < NCS; ++kk) sq[min(t + kk * kLanes, NC - 1)] = qs[kk];
        wave_sync();
        if (c4 < nd) {
            float sv[NV];
#pragma unroll
            for (int v = 0; v < NV / 4; ++v) {
                const float4 q4 = *(const float4 *)(sq + c4 + 4 * v);
                sv[4 * v] = q4.x;
                sv[4 * v + 1] = q4.y;
                sv[4 * v + 2] = q4.z;
                sv[4 * v + 3] = q4.w;
            }
            float o[4];
            residual4(sv, dvv, dt, [&](int c) { return rrv[c]; }, [&](int kk) { return dxi[kk]; },
                      o);
            store_cells<VEC>(qo, i0, nd, c4, o);
        }
    }
}

// ---------------------------------------------------------------------------
// A searching tile whose window fits the wave's LDS, on rows of a multiple of
// four cells (16-byte aligned), with every load of a phase in flight at once:
//   1. the nodes' plan (window index, theta), the window's values and cell
//      sizes in 16-byte groups, the faces' residual velocity;
//   2. the window masses into LDS; the stencil data of all the lane's
//      nodes' source cells (three planes of the mesh table);
//   3. each node's Lagrange weights and partial integral (from the masses
//      beside its window cell) into LDS;
//   4. each shifted cell's mass (the whole window cells between its nodes
//      plus the difference of the two partial integrals), while the cell
//      geometry of the residual is on its way;
//   5. the masses through LDS to four consecutive cells a lane and their
//      residual neighbourhoods, the residual, 16-byte stores.
// Nodes and shifted cells go to lanes in turn (node m, cell ci on lane
// m mod 64, counted from the tile's first halo node/cell), so that the LDS
// gathers of neighbouring lanes fall on neighbouring words: four consecutive
// nodes a lane put their gathers 16 bytes apart, eight lanes on each bank.
// The window is stored from the 16-byte boundary at or below its start (LDS
// index j + off for window cell j), so that its groups go in whole.
// ---------------------------------------------------------------------------

// The prefix modes (S other than kSumDirect): the window's exclusive
// cumulative of the masses, in the mode's precision (Acc<S>), at LDS index
// j + off for window cell j and one past the window's last group; partial
// integrals and whole-cell sums are then its differences (only differences:
// the cells below the window start in the first group cancel).  Masses of
// groups g = l + 64 s (s = 0, 1, ...), four a lane: each group's lane totals
// scanned across the wave, the groups before carried on.
template <int S>
__device__ __forceinline__ void wave_prefix(typename Acc<S>::A *sp, const typename Acc<S>::M (&m)[4],
                                            int g, int gl, typename Acc<S>::A &carry)
{
    using AC = Acc<S>;
    using A = typename AC::A;
    const int lane = (int)threadIdx.x % kLanes;
    const bool live = g <= gl;
    A tot = AC::zero();
    if (live) {
#pragma unroll
        for (int k = 0; k < 4; ++k) tot = AC::add(tot, m[k]);
    }
    // inclusive scan of the lane totals over the wave
    const A inc = wave_inclusive<AC>(tot);
    A ex = AC::template dpp<kDppWaveShr1, 0xf, 0xf>(inc);
    if (lane == 0) ex = AC::zero();
    A e = AC::comb(carry, ex);
    if (live) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            sp[4 * g + k] = e;
            e = AC::add(e, m[k]);
        }
        if (g == gl) sp[4 * g + 4] = e;
    }
    carry = AC::comb(carry, lane63(inc));
}

template <int P, int H, int S>
__device__ __forceinline__ void window_tile(const StepArgs &a, const FastTile &ft,
                                            unsigned char *su, float *sell, short *sjc, int t)
{
    using AC = Acc<S == kSumDirect ? kScanF32 : S>;
    using A = typename AC::A;
    using M = typename AC::M;
    constexpr bool kDirect = S == kSumDirect;
    constexpr int LO = (P - 1) / 2;
    constexpr int NG = 2;                            // window groups of 4 a lane loads first
    constexpr int NS = (kFT + 2 * H + 1 + kLanes - 1) / kLanes;   // node slots
    constexpr int NCS = (kFT + 2 * H + kLanes - 1) / kLanes;      // shifted-cell slots
    const Rows &R = a.rows;
    const MeshTab &tb = R.tab;
    const int n = (int)R.n_cols;
    const int c4 = 4 * t;
    const TilePos tp = tile_pos(ft.pad[0], n, H);
    const int i0 = tp.i0, nd = tp.nd;
    const int NC = nd + 2 * H;
    const int64_t qoff = (int64_t)tp.row * n;
    const float *q = (const float *)a.q_in + qoff;
    float *qo = (float *)a.q_out + qoff;
    const int W = ft.w, base = ft.base;
    const int a0 = base & ~3, off = base - a0;
    const int gl = (W + off - 1) >> 2;               // last window group
    float *sw = (float *)su;                         // window mass j at sw[j + off]

    // ---- 1. node plan, window, faces ------------------------------------------
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
    // window values and cell sizes (FP64 sizes for the FP64 prefix)
    constexpr bool kDx64 = S == kScanF64;
    float4 wq[NG], wd[NG];
    double2 wd2[kDx64 ? NG : 1][2];
#pragma unroll
    for (int u = 0; u < NG; ++u) {
        int c = a0 + 4 * min(t + u * kLanes, gl);
        c = c >= n ? c - n : c;
        wq[u] = ld_at<float4>(q, 4u * (uint32_t)c);
        if constexpr (kDx64) {
            wd2[u][0] = ld_at<double2>(tb.dx, 8u * (uint32_t)c);
            wd2[u][1] = ld_at<double2>(tb.dx, 8u * (uint32_t)c + 16u);
        } else {
            wd[u] = ld_at<float4>(tb.dxf, 4u * (uint32_t)c);
        }
    }
    float dvv[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if constexpr (H != 0) load_faces<true>((const float *)a.dv + qoff, n, i0, nd, c4, dvv);
    float4 di4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (H == 0) di4 = *(const float4 *)(tb.dxinvf + i0 + min(c4, nd - 4));
    A *sp = (A *)su;                                 // prefix modes: cumulative at j + off
    if constexpr (kDirect) {
#pragma unroll
        for (int u = 0; u < NG; ++u) {
            const int g = min(t + u * kLanes, gl);
            *(float4 *)(sw + 4 * g) = make_float4(wq[u].x * wd[u].x, wq[u].y * wd[u].y,
                                                  wq[u].z * wd[u].z, wq[u].w * wd[u].w);
        }
        // windows longer than NG groups a lane (compressing stretches of mesh)
        for (int u = NG; u * kLanes <= gl; ++u) {
            const int g = min(t + u * kLanes, gl);
            int c = a0 + 4 * g;
            c = c >= n ? c - n : c;
            const float4 vq = ld_at<float4>(q, 4u * (uint32_t)c);
            const float4 vd = ld_at<float4>(tb.dxf, 4u * (uint32_t)c);
            *(float4 *)(sw + 4 * g) = make_float4(vq.x * vd.x, vq.y * vd.y, vq.z * vd.z, vq.w * vd.w);
        }
    } else {
        A carry = AC::zero();
        auto masses = [&](const float4 &vq, const float4 &vd, const double2 (&v2)[2], M (&m)[4]) {
            if constexpr (kDx64) {
                m[0] = AC::mass(vq.x, v2[0].x);
                m[1] = AC::mass(vq.y, v2[0].y);
                m[2] = AC::mass(vq.z, v2[1].x);
                m[3] = AC::mass(vq.w, v2[1].y);
            } else {
                m[0] = (M)(vq.x * vd.x);
                m[1] = (M)(vq.y * vd.y);
                m[2] = (M)(vq.z * vd.z);
                m[3] = (M)(vq.w * vd.w);
            }
        };
#pragma unroll
        for (int u = 0; u < NG; ++u) {
            if (u * kLanes > gl) break;
            M m[4];
            masses(wq[u], wd[u], wd2[kDx64 ? u : 0], m);
            wave_prefix<S == kSumDirect ? kScanF32 : S>(sp, m, t + u * kLanes, gl, carry);
        }
        for (int u = NG; u * kLanes <= gl; ++u) {
            const int g = min(t + u * kLanes, gl);
            int c = a0 + 4 * g;
            c = c >= n ? c - n : c;
            const float4 vq = *(const float4 *)(q + c);
            float4 vd = make_float4(0.f, 0.f, 0.f, 0.f);
            double2 v2[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
            if constexpr (kDx64) {
                v2[0] = *(const double2 *)(tb.dx + c);
                v2[1] = *(const double2 *)(tb.dx + c + 2);
            } else {
                vd = *(const float4 *)(tb.dxf + c);
            }
            M m[4];
            masses(vq, vd, v2, m);
            wave_prefix<S == kSumDirect ? kScanF32 : S>(sp, m, t + u * kLanes, gl, carry);
        }
    }

    // ---- 2. stencil data of the nodes' source cells, all at once -----------------
    // (planes: neighbouring lanes read neighbouring cells' data; the offsets
    // of the cell's own edges are 0 and 1 exactly, the own node's weight is not
    // needed)
    constexpr int NV = 2 * P - 1;                    // values a cell
    float rth[NS][P + 1], rrd[NS][P + 1];
    const float *stp1 = tb.stp + 4 * n, *stp2 = tb.stp + 8 * n;
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        int c = base + jv[u];
        c = c >= n ? c - n : c;
        float v[12];
        const float4 A = ld_at<float4>(tb.stp, 16u * (uint32_t)c);
        v[0] = A.x; v[1] = A.y; v[2] = A.z; v[3] = A.w;
        if constexpr (NV > 4) {
            const float4 B = ld_at<float4>(stp1, 16u * (uint32_t)c);
            v[4] = B.x; v[5] = B.y; v[6] = B.z; v[7] = B.w;
        }
        if constexpr (NV > 8) v[8] = ld_at<float>(stp2, 4u * (uint32_t)c);
        int k = 0;
#pragma unroll
        for (int b = 0; b <= P; ++b)
            rth[u][b] = b == LO ? 0.0f : (b == LO + 1 ? 1.0f : v[k++]);
#pragma unroll
        for (int b = 0; b <= P; ++b) rrd[u][b] = b == LO ? 0.0f : v[k++];
    }
    wave_sync();                                     // the window masses

    // ---- 3. weights and partial integrals C~(x) - C(c), summed outward ------------
    // (lanes past the last node repeat it: the plan's padding, same slots)
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const float th = thv[u];
        float tt[P + 1], pre[P + 1], suf[P + 1], wk[P + 1];
#pragma unroll
        for (int b = 0; b <= P; ++b) tt[b] = th - rth[u][b];
        pre[0] = 1.0f;
#pragma unroll
        for (int b = 1; b <= P; ++b) pre[b] = pre[b - 1] * tt[b - 1];
        suf[P] = 1.0f;
#pragma unroll
        for (int b = P - 1; b >= 0; --b) suf[b] = suf[b + 1] * tt[b + 1];
#pragma unroll
        for (int b = 0; b <= P; ++b) wk[b] = rrd[u][b] * (pre[b] * suf[b]);
        const int j = jv[u] + off;
        float e = 0.0f;
        if constexpr (kDirect) {
            float up = 0.0f, dn = 0.0f;
#pragma unroll
            for (int b = LO + 1; b <= P; ++b) {
                up += sw[j + b - LO - 1];
                e += wk[b] * up;
            }
#pragma unroll
            for (int b = LO - 1; b >= 0; --b) {
                dn += sw[j - LO + b];
                e -= wk[b] * dn;
            }
        } else {
            const A pc = sp[j];
#pragma unroll
            for (int b = 0; b <= P; ++b)
                if (b != LO) e += wk[b] * (float)AC::diff(sp[j - LO + b], pc);
        }
        const int m = min(t + u * kLanes, kFastNodes - 1);
        sell[m] = e;
        sjc[m] = (short)j;
    }
    wave_sync();

    // ---- 4. shifted masses (lanes past the last cell repeat it) --------------------
    float ms[NCS];
#pragma unroll
    for (int u = 0; u < NCS; ++u) {
        const int ci = min(t + u * kLanes, NC - 1);
        const int ja = sjc[ci], jb = sjc[ci + 1];
        float whole;
        if constexpr (kDirect) {
            const float m0 = sw[ja], m1 = sw[ja + 1];
            whole = jb > ja ? m0 : 0.0f;
            whole += jb > ja + 1 ? m1 : 0.0f;
            for (int mm = ja + 2; mm < jb; ++mm) whole += sw[mm];
        } else {
            whole = (float)AC::diff(sp[jb], sp[ja]);
        }
        ms[u] = whole + (sell[ci + 1] - sell[ci]);
    }
    // geometry of cells i0+4l-2 .. i0+4l+5 (lanes past the tile: its last
    // cells): (dx, 1/centre gap) as four 16-byte pairs, 1/dx as 8 + 16 + 8
    // bytes (the row holds a multiple of four cells: no group straddles its end)
    float2 rr[8];
    float dxi[8];
    if constexpr (H != 0) {
        const int cb = i0 + min(c4, nd - 4) - 2;
        auto wr = [&](int c) { return c < 0 ? c + n : (c >= n ? c - n : c); };
#pragma unroll
        for (int pr = 0; pr < 4; ++pr) {
            const float4 r2 = ld_at<float4>(tb.rrf, 8u * (uint32_t)wr(cb + 2 * pr));
            rr[2 * pr] = make_float2(r2.x, r2.y);
            rr[2 * pr + 1] = make_float2(r2.z, r2.w);
        }
        const float2 d0 = ld_at<float2>(tb.dxinvf, 4u * (uint32_t)wr(cb));
        const float4 d1 = ld_at<float4>(tb.dxinvf, 4u * (uint32_t)wr(cb + 2));
        const float2 d2 = ld_at<float2>(tb.dxinvf, 4u * (uint32_t)wr(cb + 6));
        dxi[0] = d0.x; dxi[1] = d0.y;
        dxi[2] = d1.x; dxi[3] = d1.y; dxi[4] = d1.z; dxi[5] = d1.w;
        dxi[6] = d2.x; dxi[7] = d2.y;
    }
    wave_sync();                                     // the window is dead
    float *sm = (float *)su;                         // shifted masses, index ci
#pragma unroll
    for (int u = 0; u < NCS; ++u) sm[min(t + u * kLanes, NC - 1)] = ms[u];
    wave_sync();

    // ---- 5. residual (or, without one, the shifted values) ------------------------
    if (c4 < nd) {
        if constexpr (H == 0) {
            const float4 m4 = *(const float4 *)(sm + c4);
            float o[4] = {m4.x * di4.x, m4.y * di4.y, m4.z * di4.z, m4.w * di4.w};
            store_cells<true>(qo, i0, nd, c4, o);
        } else {
            const float4 m0 = *(const float4 *)(sm + c4), m1 = *(const float4 *)(sm + c4 + 4);
            const float mv[8] = {m0.x, m0.y, m0.z, m0.w, m1.x, m1.y, m1.z, m1.w};
            float sv[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) sv[c] = mv[c] * dxi[c];
            if (a.q_mid)
                *(float4 *)((float *)a.q_mid + qoff + i0 + c4) = make_float4(sv[2], sv[3], sv[4], sv[5]);
            float o[4];
            residual4(sv, dvv, (float)a.dt, [&](int c) { return rr[c]; },
                      [&](int kk) { return dxi[kk + 2]; }, o);
            store_cells<true>(qo, i0, nd, c4, o);
        }
    }
}

// ---------------------------------------------------------------------------
// The compacted records, in tile order: uniform tiles first, then the others
// (for the node plan), each with its tile id in pad[0]; the others' position
// among them (their node data) in pad[1] of both copies.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(1024) void k_tile_count(const FastTile *rec, int nt, int32_t *counts)
{
    __shared__ int swc[16];
    const int j = (int)blockIdx.x * 1024 + (int)threadIdx.x;
    const bool u = j < nt && rec[j].kind == kFastUniform;
    const int c = __popcll(__ballot(u));
    if ((threadIdx.x & 63) == 0) swc[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < 16; ++w) s += swc[w];
        counts[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(1024) void k_tile_lists(FastTile *rec, int nt,
                                                     const int32_t *counts, int nb,
                                                     FastTile *crec, int32_t *totals)
{
    __shared__ int sred[2][16];
    __shared__ int swo[2][17];
    const int tid = (int)threadIdx.x, lane = tid & 63, wv = tid >> 6;
    // uniform tiles before this block and in total
    int before = 0, all = 0;
    for (int b = tid; b < nb; b += 1024) {
        const int c = counts[b];
        all += c;
        if (b < (int)blockIdx.x) before += c;
    }
    for (int o = 32; o > 0; o >>= 1) {
        before += __shfl_xor(before, o, 64);
        all += __shfl_xor(all, o, 64);
    }
    if (lane == 0) {
        sred[0][wv] = before;
        sred[1][wv] = all;
    }
    const int j = (int)blockIdx.x * 1024 + tid;
    const bool in = j < nt;
    const bool u = in && rec[j].kind == kFastUniform;
    const uint64_t mu = __ballot(u), mg = __ballot(in && !u);
    const uint64_t below = (1ull << lane) - 1ull;
    if (lane == 0) {
        swo[0][wv + 1] = __popcll(mu);
        swo[1][wv + 1] = __popcll(mg);
    }
    __syncthreads();
    if (tid == 0) {
        int b0 = 0, a0 = 0;
        for (int w = 0; w < 16; ++w) {
            b0 += sred[0][w];
            a0 += sred[1][w];
        }
        sred[0][0] = b0;
        sred[1][0] = a0;
        swo[0][0] = swo[1][0] = 0;
        for (int w = 1; w <= 16; ++w) {
            swo[0][w] += swo[0][w - 1];
            swo[1][w] += swo[1][w - 1];
        }
        if (blockIdx.x == 0) {
            totals[0] = a0;
            totals[1] = nt - a0;
        }
    }
    __syncthreads();
    const int ub = sred[0][0], utot = sred[1][0];
    const int gb = (int)blockIdx.x * 1024 - ub;      // other tiles before this block
    if (in) {
        int pos;
        if (u) pos = ub + swo[0][wv] + __popcll(mu & below);
        else pos = utot + gb + swo[1][wv] + __popcll(mg & below);
        FastTile r = rec[j];
        if (!u) {
            r.pad[1] = pos - utot;                   // the tile's node data
            rec[j].pad[1] = r.pad[1];
        }
        crec[pos] = r;
    }
}

// The step, in two kernels, one tile a wave: the uniform tiles (the
// compacted list's first part; 26 registers, eight waves a SIMD), then the
// other tiles (the rest of the list).  Both grids span the whole tile count
// (the host does not know the split); the waves past their part of the list
// return at once.  Measured alternatives on the refined disk: one kernel over
// both kinds (in tile order, or the other tiles spread evenly through the
// grid) ran the uniform tiles at the other path's register and LDS footprint
// and took 135-163 us a step against 123; persistent waves striding over the
// other tiles, 128-157; the two kernels on two streams with an event pair
// around every eager step, 342.  Inside a captured step loop the two kernels
// are parallel branches of the graph (fork / join events, ForkJoin): the
// latency-bound searching tiles then run beside the HBM-bound uniform ones.
template <int P, int H, bool VEC>
__global__ __launch_bounds__(kBlock, 8) void k_step_uni(StepArgs a)
{
    __shared__ __attribute__((aligned(16))) float swin[kWaves][kUniWin];
    const int wid = wave_id();
    const int i = (int)blockIdx.x * kWaves + wid;
    if (i >= a.fast.totals[0]) return;
    const FastTile r = load_rec(a.fast.rec + a.rows.n_tiles, i);
    uniform_tile<P, H, VEC>(a, r, swin[wid], (int)threadIdx.x % kLanes);
}

// A uniform-run tile of the limited step (Section 3.1's PLM / PPM, App. A),
// FP32: every node of the tile sits in the next window cell at the tile's
// theta, so shifted cell ci is the average of window cell LO + ci plus the
// difference of the limited cubics of window cells LO + ci + 1 and LO + ci
// at theta (in value units: the run's cells are all of one size).  Each lane
// forms, from its window values in registers, the slopes, the PPM interface
// values and the constrained parabolas its eight shifted cells need (the
// mesh's weights of window cell 1, whose neighbours lie in the run, serve the
// whole tile), then the residual as in uniform_tile.
template <int R, int H, bool VEC>
__device__ __forceinline__ void uniform_tile_lim(const StepArgs &a, const FastTile &r, float *sw,
                                                 int t)
{
    constexpr int LO = LimHalo<R>::lo;
    constexpr int P = 2 * LO + 1;
    constexpr int NV = 4 + 2 * H;                    // shifted cells a lane
    constexpr int NQ = NV + 2 * LO + 1;             // window values c4 .. c4 + NQ - 1
    constexpr int NW = (NQ + 3) / 4 * 4;             // whole float4s
    constexpr int NUW = (kFT + 2 * H + P + kLanes - 1) / kLanes;  // window slots a lane
    static_assert(NUW * kLanes <= kUniWin && 4 * (kLanes - 1) + NW <= kUniWin, "window");
    const MeshTab &tb = a.rows.tab;
    const int n = (int)a.rows.n_cols;
    const float dt = (float)a.dt;
    const int c4 = 4 * t;
    const TilePos p = tile_pos(r.pad[0], n, H);
    const int64_t qoff = (int64_t)p.row * n;
    const float th = __int_as_float(r.pad[1]);

    float wv[NUW];
    {
        const float *q = (const float *)a.q_in + qoff;
#pragma unroll
        for (int k = 0; k < NUW; ++k) {
            int mm = r.base + min(t + k * kLanes, r.w - 1);
            mm = mm >= n ? mm - n : mm;
            wv[k] = q[mm];
        }
    }
    float pw[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    {
        const int c1 = r.base + 1 >= n ? r.base + 1 - n : r.base + 1;
        if constexpr (R == kReconPPM) {
#pragma unroll
            for (int k = 0; k < 5; ++k) pw[k] = tb.ppmf[k * n + c1];
        }
    }
    float dvv[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if constexpr (H != 0) load_faces<VEC>((const float *)a.dv + qoff, n, p.i0, p.nd, c4, dvv);
#pragma unroll
    for (int k = 0; k < NUW; ++k) sw[t + k * kLanes] = wv[k];
    wave_sync();
    float win[NW];
#pragma unroll
    for (int v = 0; v < NW / 4; ++v) {
        const float4 w4 = *(const float4 *)(sw + c4 + 4 * v);
        win[4 * v] = w4.x;
        win[4 * v + 1] = w4.y;
        win[4 * v + 2] = w4.z;
        win[4 * v + 3] = w4.w;
    }
    // ell[v]: the limited cubic at theta of window cell c4 + LO + v (value units)
    float ell[NV + 1];
    if constexpr (R == kReconPPM) {
        // slope of window cell c4 + 1 + s, then the interface between window
        // cells c4 + 1 + s and c4 + 2 + s
        float dl[NV + 3], iv[NV + 2];
#pragma unroll
        for (int k = 0; k < NV + 3; ++k) dl[k] = ppm_delta<float>(win[k], win[k + 1], win[k + 2], pw[0], pw[1]);
#pragma unroll
        for (int k = 0; k < NV + 2; ++k)
            iv[k] = win[k + 1] + pw[2] * (win[k + 2] - win[k + 1]) + pw[3] * dl[k + 1] + pw[4] * dl[k];
#pragma unroll
        for (int v = 0; v <= NV; ++v) {
            float pa, pb, pc;
            ppm_cubic<float>(win[v + 2], iv[v], iv[v + 1], 1.0f, pa, pb, pc);
            pb = win[v + 2] - pa - pc;
            ell[v] = th * (pa + th * (pb + th * pc));
        }
    } else {
        const float g = r.hinv, hh = r.dx;
#pragma unroll
        for (int v = 0; v <= NV; ++v) {
            const float dp = (win[v + 2] - win[v + 1]) * g, dm = (win[v + 1] - win[v]) * g;
            const float sig = (dp * dm <= 0.0f) ? 0.0f : harmonic2(dp, dm);
            const float kap = 0.5f * sig * hh;
            ell[v] = th * (win[v + 1] - kap + th * kap);
        }
    }
    float s[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] = win[v + LO] + (ell[v + 1] - ell[v]);
    float *qo = (float *)a.q_out + qoff;
    if constexpr (H == 0) {
        store_cells<VEC>(qo, p.i0, p.nd, c4, s);
    } else {
        if (a.q_mid && c4 < p.nd) {
            float *qm = (float *)a.q_mid + qoff;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (c4 + k < p.nd) qm[p.i0 + c4 + k] = s[k + 2];
        }
        const float2 g = make_float2(r.dx, r.hinv);
        const float dxi = r.dxinv;
        float o[4];
        residual4(s, dvv, dt, [&](int) { return g; }, [&](int) { return dxi; }, o);
        store_cells<VEC>(qo, p.i0, p.nd, c4, o);
    }
}

template <int R, int H, bool VEC>
__global__ __launch_bounds__(kBlock) void k_step_uni_lim(StepArgs a)
{
    __shared__ __attribute__((aligned(16))) float swin[kWaves][kUniWin];
    const int wid = wave_id();
    const int i = (int)blockIdx.x * kWaves + wid;
    if (i >= a.fast.totals[0]) return;
    const FastTile r = load_rec(a.fast.rec + a.rows.n_tiles, i);
    uniform_tile_lim<R, H, VEC>(a, r, swin[wid], (int)threadIdx.x % kLanes);
}

// The other tiles: a grid of a quarter of the tile count in waves (the host
// does not know how many there are; a quarter covers the refined disk with
// one tile a wave), each wave stepping through the list by the grid's size.
constexpr int kGenShare = 4;

template <int P, int H, bool VEC, int S>
__global__ __launch_bounds__(kBlock) void k_step_gen(StepArgs a)
{
    __shared__ __attribute__((aligned(16))) unsigned char su[kWaves][wave_lds_bytes<S>()];
    __shared__ __attribute__((aligned(16))) float sell_[kWaves][WaveLds::nodes];
    __shared__ __attribute__((aligned(16))) short sjc_[kWaves][WaveLds::nodes];
    const int wid = wave_id();
    const int nt = (int)a.rows.n_tiles;
    const int n = (int)a.rows.n_cols;
    const int t = (int)threadIdx.x % kLanes;
    const int stride = (int)gridDim.x * kWaves;
    for (int i = a.fast.totals[0] + (int)blockIdx.x * kWaves + wid; i < nt; i += stride) {
        const FastTile r = load_rec(a.fast.rec + nt, i);
        if (VEC && r.kind == kFastWindow && r.base + r.w + 3 < 2 * n)
            window_tile<P, H, S>(a, r, su[wid], sell_[wid], sjc_[wid], t);
        else
            general_tile<P, H, VEC>(a, r, su[wid], sell_[wid], sjc_[wid], t);
        wave_sync();                                 // the next tile reuses the LDS
    }
}

template <int P, int H, bool VEC, int S>
hipError_t step_fast_kernels(const StepArgs &a, hipStream_t st)
{
    const dim3 g((unsigned)((a.rows.n_tiles + kWaves - 1) / kWaves)), b(kBlock);
    const dim3 gg((unsigned)((a.rows.n_tiles + kWaves * kGenShare - 1) / (kWaves * kGenShare)));
    if (const ForkJoin *fj = capture_fork) {
        // the two kinds of tile write disjoint cells and read only q_in: the
        // searching tiles' kernel on the side stream, between a fork after
        // everything before the step and a join before everything after it
        hipError_t e = hipEventRecord(fj->fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(fj->side, fj->fork, 0);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_step_gen<P, H, VEC, S>), gg, b, 0, fj->side, a);
        e = hipEventRecord(fj->join, fj->side);
        hipLaunchKernelGGL((k_step_uni<P, H, VEC>), g, b, 0, st, a);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, fj->join, 0);
        if (e != hipSuccess) return e;
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_step_uni<P, H, VEC>), g, b, 0, st, a);
    hipLaunchKernelGGL((k_step_gen<P, H, VEC, S>), gg, b, 0, st, a);
    return hipGetLastError();
}

template <int P, int S>
hipError_t step_fast_ps(const StepArgs &a, bool vec, hipStream_t st)
{
    if (a.dv) return vec ? step_fast_kernels<P, 2, true, S>(a, st) : step_fast_kernels<P, 2, false, S>(a, st);
    return vec ? step_fast_kernels<P, 0, true, S>(a, st) : step_fast_kernels<P, 0, false, S>(a, st);
}

template <int P>
hipError_t step_fast_p(const StepArgs &a, int scan, hipStream_t st)
{
    const bool vec = (a.rows.n_cols % 4) == 0 && ((uintptr_t)a.q_out % 16) == 0 &&
                     ((uintptr_t)a.q_in % 16) == 0 &&
                     (!a.q_mid || ((uintptr_t)a.q_mid % 16) == 0) &&
                     (!a.dv || ((uintptr_t)a.dv % 16) == 0);
    switch (scan) {
    case kScanF64: return step_fast_ps<P, kScanF64>(a, vec, st);
    case kScanTwoSum: return step_fast_ps<P, kScanTwoSum>(a, vec, st);
    case kScanF32: return step_fast_ps<P, kScanF32>(a, vec, st);
    default: return step_fast_ps<P, kSumDirect>(a, vec, st);
    }
}

// The limited step's other tiles: general_tile with the limited partials, the
// window tabulated in LDS where it fits, else every node located by the bucket
// index and its partial integral the limited profile of its cell.
template <int R, int H, bool VEC>
__global__ __launch_bounds__(kBlock) void k_step_gen_lim(StepArgs a)
{
    constexpr int P = 2 * LimHalo<R>::lo + 1;
    constexpr size_t U = kGenLimLds > WaveLds::u ? kGenLimLds : WaveLds::u;
    __shared__ __attribute__((aligned(16))) unsigned char su[kWaves][U];
    __shared__ __attribute__((aligned(16))) float sell_[kWaves][WaveLds::nodes];
    __shared__ __attribute__((aligned(16))) short sjc_[kWaves][WaveLds::nodes];
    const int wid = wave_id();
    const int nt = (int)a.rows.n_tiles;
    const int t = (int)threadIdx.x % kLanes;
    const int stride = (int)gridDim.x * kWaves;
    for (int i = a.fast.totals[0] + (int)blockIdx.x * kWaves + wid; i < nt; i += stride) {
        const FastTile r = load_rec(a.fast.rec + nt, i);
        general_tile<P, H, VEC, R>(a, r, su[wid], sell_[wid], sjc_[wid], t);
        wave_sync();                                 // the next tile reuses the LDS
    }
}

template <int R, int H, bool VEC>
hipError_t step_fast_lim_kernels(const StepArgs &a, hipStream_t st)
{
    const dim3 g((unsigned)((a.rows.n_tiles + kWaves - 1) / kWaves)), b(kBlock);
    const dim3 gg((unsigned)((a.rows.n_tiles + kWaves * kGenShare - 1) / (kWaves * kGenShare)));
    if (const ForkJoin *fj = capture_fork) {
        // parallel graph branches, as in step_fast_kernels
        hipError_t e = hipEventRecord(fj->fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(fj->side, fj->fork, 0);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_step_gen_lim<R, H, VEC>), gg, b, 0, fj->side, a);
        e = hipEventRecord(fj->join, fj->side);
        hipLaunchKernelGGL((k_step_uni_lim<R, H, VEC>), g, b, 0, st, a);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, fj->join, 0);
        if (e != hipSuccess) return e;
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_step_uni_lim<R, H, VEC>), g, b, 0, st, a);
    hipLaunchKernelGGL((k_step_gen_lim<R, H, VEC>), gg, b, 0, st, a);
    return hipGetLastError();
}

template <int R>
hipError_t step_fast_lim_r(const StepArgs &a, hipStream_t st)
{
    const bool vec = (a.rows.n_cols % 4) == 0 && ((uintptr_t)a.q_out % 16) == 0 &&
                     ((uintptr_t)a.q_in % 16) == 0 &&
                     (!a.q_mid || ((uintptr_t)a.q_mid % 16) == 0) &&
                     (!a.dv || ((uintptr_t)a.dv % 16) == 0);
    if (a.dv) return vec ? step_fast_lim_kernels<R, 2, true>(a, st) : step_fast_lim_kernels<R, 2, false>(a, st);
    return vec ? step_fast_lim_kernels<R, 0, true>(a, st) : step_fast_lim_kernels<R, 0, false>(a, st);
}

// ---------------------------------------------------------------------------
// Per-row meshes (every row its own nodes, ragged or not), FP32 state, the
// shift alone.  The tiles are the ragged tile table's, kRagTile cells of one
// row, one a wave.  Per call, k_plan_rag locates every shifted node of a tile
// (a binary search of the row, Eq. condition_p), takes its Lagrange weights
// from the row's nodes (Section 3, Step 2: the cumulative's interpolant
// through the p+1 nodes around the source cell) and its source cell's index
// in the tile's window, and writes the row cells' FP32 sizes.  Per step,
// k_step_rag then needs no search and no division by the mesh: the window's
// masses into LDS (or, for the prefix modes, their cumulative), each node's
// partial integral from its planned weights, each cell's whole source cells
// and the two partials, over the cell size (Eqs. mass_shift_algo, step3).
// ---------------------------------------------------------------------------

__device__ inline RagTile load_rag(const RagTile *rec, int64_t i)
{
    RagTile r;
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) int32_t *CI;
    const CI c = (CI)(rec + i);
    int32_t *o = (int32_t *)&r;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(RagTile) / 4); ++k) o[k] = c[k];
#else
    r = rec[i];
#endif
    return r;
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_plan_rag(StepArgs a, RagPlan pl)
{
    constexpr int LO = (P - 1) / 2;
    constexpr int NS = (kFastNodes + kLanes - 1) / kLanes;
    const Rows &R = a.rows;
    const int t = (int)threadIdx.x % kLanes;
    const int64_t tile = (int64_t)blockIdx.x * kWaves + wave_id();
    if (tile >= R.n_tiles) return;
    RagTile rt;
    rt.kind = -1;
    rt.row = rt.i0 = rt.nd = rt.n = rt.w = rt.base = rt.pad0 = 0;
    rt.qoff = rt.eoff = rt.wlo = 0;
    rt.pad[0] = rt.pad[1] = 0;
    Tile ti;
    if (!get_tile(R, tile, ti)) {                    // past the batch's last tile
        if (t == 0) pl.rec[tile] = rt;
        return;
    }
    const int n = ti.n, i0 = ti.i0;
    const int nd = min(R.tile, n - i0);
    const int NE = nd + 1;
    const double *x = ti.x;
    const double len = x[n] - x[0];
    const double invlen = 1.0 / len;
    const double s = a.v0[ti.row] * a.dt;
    for (int c = t; c < nd; c += kLanes)
        pl.dx[ti.qoff + i0 + c] = (float)(x[i0 + c + 1] - x[i0 + c]);
    // extended source index g = c + k n of row node e (node n: node 0 one
    // period on) and the wrapped shifted position
    auto locate = [&](int e, double &xh) -> int64_t {
        int kx = 0;
        if (e >= n) {
            e -= n;
            kx = 1;
        }
        int64_t k;
        shifted_node_inv(x, n, s, e, invlen, len, xh, k);
        return (int64_t)find_cell(x, n, xh) + (k + kx) * (int64_t)n;
    };
    double xh0, xh1;
    const int64_t g0 = locate(i0, xh0);
    const int64_t g1 = locate(i0 + nd, xh1);
    const int64_t wlo = g0 - LO;
    const int64_t wide = g1 - g0 + P;
    bool ok = wide >= P && wide <= kFastWin;
    const int64_t slot = tile * kFastNodes;
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const int m = t + u * kLanes;
        if (m < kFastNodes) {
            double xh;
            const int64_t g = locate(i0 + min(m, NE - 1), xh);
            const int c = (int)(g - (g >= 0 ? g / n : -((-g + n - 1) / n)) * (int64_t)n);
            double X[P + 1];
#pragma unroll
            for (int b = 0; b <= P; ++b) X[b] = node_x(x, n, len, c - LO + b) - x[c];
            float w[P + 1];
            lagrange_rel<float, P>(xh - x[c], X, w);
            float v[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
            int k = 0;
#pragma unroll
            for (int b = 0; b <= P; ++b)
                if (b != LO) v[k++] = w[b];
            pl.wa[slot + m] = make_float4(v[0], v[1], v[2], v[3]);
            pl.wb[slot + m] = v[4];
            const int64_t j = g - wlo;
            ok = ok && j >= LO && j + P - LO <= wide;
            pl.jc[slot + m] = (int16_t)min(max(j, (int64_t)0), (int64_t)kFastWin);
        }
    }
    const bool all = __all(ok ? 1 : 0) != 0;
    if (t == 0) {
        rt.kind = all ? kFastWindow : kFastDirect;
        rt.row = (int32_t)ti.row;
        rt.i0 = i0;
        rt.nd = nd;
        rt.n = n;
        rt.w = all ? (int32_t)wide : 0;
        rt.base = (int32_t)(wlo - (wlo >= 0 ? wlo / n : -((-wlo + n - 1) / n)) * (int64_t)n);
        rt.qoff = ti.qoff;
        rt.eoff = (int64_t)(x - R.edges);
        rt.wlo = wlo;
        pl.rec[tile] = rt;
    }
}

// The prefix modes on per-row tiles: one window cell a lane per slot (cell j
// = l + 64 u), the slot's masses scanned across the wave, the slots before
// carried on; sp[j] = cumulative before cell j, sp[W] the total.
template <int S>
__device__ __forceinline__ void wave_prefix1(typename Acc<S>::A *sp, typename Acc<S>::M m, int j,
                                             int W, typename Acc<S>::A &carry)
{
    using AC = Acc<S>;
    using A = typename AC::A;
    const int lane = (int)threadIdx.x % kLanes;
    const bool live = j < W;
    const A inc = wave_inclusive<AC>(live ? AC::add(AC::zero(), m) : AC::zero());
    A ex = AC::template dpp<kDppWaveShr1, 0xf, 0xf>(inc);
    if (lane == 0) ex = AC::zero();
    if (live) {
        sp[j] = AC::comb(carry, ex);
        if (j == W - 1) sp[W] = AC::comb(carry, inc);
    }
    carry = AC::comb(carry, lane63(inc));
}

template <int P, int S>
__device__ __forceinline__ void rag_tile(const StepArgs &a, const RagTile &r, int64_t tile,
                                         unsigned char *su, float *sell, short *sjc, int t)
{
    using AC = Acc<S == kSumDirect ? kScanF32 : S>;
    using A = typename AC::A;
    using M = typename AC::M;
    constexpr bool kDirect = S == kSumDirect;
    constexpr int LO = (P - 1) / 2;
    constexpr int NS = (kRagTile + 1 + kLanes - 1) / kLanes;     // node slots
    constexpr int NCS = (kRagTile + kLanes - 1) / kLanes;        // cell slots
    constexpr int NB = 5;                                         // window slots a batch
    const int n = r.n, i0 = r.i0, nd = r.nd, W = r.w, base = r.base;
    const float *q = (const float *)a.q_in + r.qoff;
    float *qo = (float *)a.q_out + r.qoff;
    const float *dxr = a.rag.dx + r.qoff;
    const int64_t slot = tile * kFastNodes;
    float *sw = (float *)su;                         // direct sums: window masses
    A *sp = (A *)su;                                 // prefix modes: the cumulative

    // ---- plan of the nodes, sizes of the destination cells -------------------
    float4 wa[NS];
    float wb[NS];
    int jv[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const int m = min(t + u * kLanes, kFastNodes - 1);
        wa[u] = a.rag.wa[slot + m];
        wb[u] = a.rag.wb[slot + m];
        jv[u] = a.rag.jc[slot + m];
    }
    float dxd[NCS];
#pragma unroll
    for (int u = 0; u < NCS; ++u) dxd[u] = dxr[i0 + min(t + u * kLanes, nd - 1)];

    // ---- window masses, five slots of loads at a time (a whole window of
    // up to 320 cells in one batch); the FP64 prefix widens the FP32 masses
    const bool once = base + W <= 2 * n;             // the window wraps the row at most once
    A carry = AC::zero();
    for (int s0 = 0; s0 * kLanes < W; s0 += NB) {
        float vq[NB], vd[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = min(t + (s0 + u) * kLanes, W - 1);
            int c = base + j;
            c = once ? (c >= n ? c - n : c) : c % n;
            vq[u] = q[c];
            vd[u] = dxr[c];
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            if ((s0 + u) * kLanes >= W) break;
            const int j = t + (s0 + u) * kLanes;
            if constexpr (kDirect) {
                if (j < W) sw[j] = vq[u] * vd[u];
            } else {
                const M m = (M)(vq[u] * vd[u]);
                wave_prefix1<S == kSumDirect ? kScanF32 : S>(sp, m, j, W, carry);
            }
        }
    }
    wave_sync();

    // ---- partial integrals C~(x) - C(c) of the nodes ---------------------------
#pragma unroll
    for (int u = 0; u < NS; ++u) {
        const float v[5] = {wa[u].x, wa[u].y, wa[u].z, wa[u].w, wb[u]};
        float wk[P + 1];
        int k = 0;
#pragma unroll
        for (int b = 0; b <= P; ++b) wk[b] = b == LO ? 0.0f : v[k++];
        const int j = jv[u];
        float e = 0.0f;
        if constexpr (kDirect) {
            float up = 0.0f, dn = 0.0f;
#pragma unroll
            for (int b = LO + 1; b <= P; ++b) {
                up += sw[j + b - LO - 1];
                e += wk[b] * up;
            }
#pragma unroll
            for (int b = LO - 1; b >= 0; --b) {
                dn += sw[j - LO + b];
                e -= wk[b] * dn;
            }
        } else {
            const A pc = sp[j];
#pragma unroll
            for (int b = 0; b <= P; ++b)
                if (b != LO) e += wk[b] * (float)AC::diff(sp[j - LO + b], pc);
        }
        const int m = min(t + u * kLanes, kFastNodes - 1);
        sell[m] = e;
        sjc[m] = (short)j;
    }
    wave_sync();

    // ---- destination cells: whole source cells + two partials, / dx ----------
#pragma unroll
    for (int u = 0; u < NCS; ++u) {
        const int ci = t + u * kLanes;
        if (ci < nd) {
            const int ja = sjc[ci], jb = sjc[ci + 1];
            float whole;
            if constexpr (kDirect) {
                const float m0 = sw[ja], m1 = sw[ja + 1];
                whole = jb > ja ? m0 : 0.0f;
                whole += jb > ja + 1 ? m1 : 0.0f;
                for (int mm = ja + 2; mm < jb; ++mm) whole += sw[mm];
            } else {
                whole = (float)AC::diff(sp[jb], sp[ja]);
            }
            qo[i0 + ci] = (whole + (sell[ci + 1] - sell[ci])) / dxd[u];
        }
    }
}

// A per-row tile whose window exceeds the LDS: nodes located again and the
// masses summed from global memory, FP64.
template <int P>
__device__ __forceinline__ void rag_direct(const StepArgs &a, const RagTile &r,
                                           unsigned char *su, float *sell, int t)
{
    const int n = r.n, i0 = r.i0, nd = r.nd;
    const float *q = (const float *)a.q_in + r.qoff;
    float *qo = (float *)a.q_out + r.qoff;
    const double *x = a.rows.edges + r.eoff;
    const double len = x[n] - x[0];
    const double invlen = 1.0 / len;
    const double s = a.v0[r.row] * a.dt;
    int64_t *sg = (int64_t *)su;
    for (int m = t; m <= nd; m += kLanes) {
        int e = i0 + m, kx = 0;
        if (e >= n) {
            e -= n;
            kx = 1;
        }
        double xh;
        int64_t k;
        shifted_node_inv(x, n, s, e, invlen, len, xh, k);
        const int64_t g = (int64_t)find_cell(x, n, xh) + (k + kx) * (int64_t)n;
        sg[m] = g;
        sell[m] = (float)direct_partial<float, P>(x, q, n, len, s, invlen, i0 + m, g);
    }
    wave_sync();
    for (int ci = t; ci < nd; ci += kLanes) {
        const int c = i0 + ci;
        const double mp = direct_whole<float>(x, q, n, sg[ci], sg[ci + 1]) +
                          ((double)sell[ci + 1] - (double)sell[ci]);
        qo[c] = (float)(mp / (x[c + 1] - x[c]));
    }
}

template <int P, int S>
__global__ __launch_bounds__(kBlock) void k_step_rag(StepArgs a)
{
    __shared__ __attribute__((aligned(16))) unsigned char su[kWaves][wave_lds_bytes<S>()];
    __shared__ __attribute__((aligned(16))) float sell_[kWaves][WaveLds::nodes];
    __shared__ __attribute__((aligned(16))) short sjc_[kWaves][WaveLds::nodes];
    const int wid = wave_id();
    const int64_t tile = (int64_t)blockIdx.x * kWaves + wid;
    if (tile >= a.rows.n_tiles) return;
    const RagTile r = load_rag(a.rag.rec, tile);
    const int t = (int)threadIdx.x % kLanes;
    if (r.kind == kFastWindow) rag_tile<P, S>(a, r, tile, su[wid], sell_[wid], sjc_[wid], t);
    else if (r.kind == kFastDirect) rag_direct<P>(a, r, su[wid], sell_[wid], t);
}

template <int P>
hipError_t step_rag_p(const StepArgs &a, int scan, hipStream_t st)
{
    const dim3 g((unsigned)((a.rows.n_tiles + kWaves - 1) / kWaves)), b(kBlock);
    switch (scan) {
    case kScanF64: hipLaunchKernelGGL((k_step_rag<P, kScanF64>), g, b, 0, st, a); break;
    case kScanTwoSum: hipLaunchKernelGGL((k_step_rag<P, kScanTwoSum>), g, b, 0, st, a); break;
    case kScanF32: hipLaunchKernelGGL((k_step_rag<P, kScanF32>), g, b, 0, st, a); break;
    default: hipLaunchKernelGGL((k_step_rag<P, kSumDirect>), g, b, 0, st, a); break;
    }
    return hipGetLastError();
}

} // namespace

hipError_t launch_plan_fast(const StepArgs &a, int order, const FastPlan &plan,
                            hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    if (a.rows.tile != kFastTile || a.rows.n_tiles > INT32_MAX / 2) return hipErrorInvalidValue;
    const int nt = (int)a.rows.n_tiles;
    const unsigned grid = (unsigned)((nt + 63) / 64);
    switch (order) {
    case 1: hipLaunchKernelGGL(k_plan_fast<1>, dim3(grid), dim3(64), 0, stream, a, plan.rec); break;
    case 3: hipLaunchKernelGGL(k_plan_fast<3>, dim3(grid), dim3(64), 0, stream, a, plan.rec); break;
    default: hipLaunchKernelGGL(k_plan_fast<5>, dim3(grid), dim3(64), 0, stream, a, plan.rec); break;
    }
    const int nb = (nt + 1023) / 1024;
    hipLaunchKernelGGL(k_tile_count, dim3(nb), dim3(1024), 0, stream, plan.rec, nt, plan.counts);
    // the compacted records follow the per-tile ones (fast_plan_bytes)
    hipLaunchKernelGGL(k_tile_lists, dim3(nb), dim3(1024), 0, stream, plan.rec, nt, plan.counts,
                       nb, plan.rec + nt, plan.totals);
    StepArgs b = a;
    b.fast = plan;
    const dim3 gn((unsigned)((nt + kWaves - 1) / kWaves));
    switch (order) {
    case 1: hipLaunchKernelGGL(k_node_plan<1>, gn, dim3(kBlock), 0, stream, b); break;
    case 3: hipLaunchKernelGGL(k_node_plan<3>, gn, dim3(kBlock), 0, stream, b); break;
    default: hipLaunchKernelGGL(k_node_plan<5>, gn, dim3(kBlock), 0, stream, b); break;
    }
    return hipGetLastError();
}

hipError_t launch_step_fast(const StepArgs &a, int order, int scan, hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    if (a.rows.tile != kFastTile) return hipErrorInvalidValue;
    switch (order) {
    case 1: return step_fast_p<1>(a, scan, stream);
    case 3: return step_fast_p<3>(a, scan, stream);
    default: return step_fast_p<5>(a, scan, stream);
    }
}

hipError_t launch_step_fast_lim(const StepArgs &a, int recon, hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    if (a.rows.tile != kFastTile) return hipErrorInvalidValue;
    return recon == kReconPLM ? step_fast_lim_r<kReconPLM>(a, stream)
                              : step_fast_lim_r<kReconPPM>(a, stream);
}

hipError_t launch_plan_rag(const StepArgs &a, int order, const RagPlan &plan,
                           hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    if (a.rows.tile != kRagTile || a.dv) return hipErrorInvalidValue;
    const dim3 g((unsigned)((a.rows.n_tiles + kWaves - 1) / kWaves)), b(kBlock);
    switch (order) {
    case 1: hipLaunchKernelGGL(k_plan_rag<1>, g, b, 0, stream, a, plan); break;
    case 3: hipLaunchKernelGGL(k_plan_rag<3>, g, b, 0, stream, a, plan); break;
    default: hipLaunchKernelGGL(k_plan_rag<5>, g, b, 0, stream, a, plan); break;
    }
    return hipGetLastError();
}

hipError_t launch_step_rag(const StepArgs &a, int order, int scan, hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    if (a.rows.tile != kRagTile || a.dv) return hipErrorInvalidValue;
    switch (order) {
    case 1: return step_rag_p<1>(a, scan, stream);
    case 3: return step_rag_p<3>(a, scan, stream);
    default: return step_rag_p<5>(a, scan, stream);
    }
}

} // namespace ram
