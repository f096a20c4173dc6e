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
//   * the shift of a row is reduced by whole periods once per tile, so a
//     shifted node is wrapped into the period with one subtraction and one
//     compare instead of a floor;
//   * the source cell of a shifted node takes one bucket record (lower-bound
//     cell and the next two nodes) and the stencil one cell record (x_c, 1/dx_c,
//     normalised node offsets, reciprocal Lagrange denominators);
//   * the residual reads per-cell (dx, 1/centre gap) records staged in LDS;
//   * with kSumDirect the cumulative differences are summed directly from the
//     window masses (a partial integral needs at most p of them, a whole-cell
//     sum the masses between two nodes), so no prefix sum is formed and no
//     cancellation arises;
//   * tiles away from the row seam skip all periodic index wrapping.
//
// The same kernel serves the limited reconstructions of Section 3.1 (R = PLM
// or PPM, direct sums only): after the window masses are stored, every window
// cell's limited profile is reduced in LDS to its partial-integral cubic
// ell(theta) (PLM: the slope term kappa = sigma dx^2 / 2; PPM: the limited
// slopes, the interface values, then the constrained parabola's coefficients),
// and each node evaluates its cell's cubic instead of Lagrange weights.  P is
// then the Lagrange order whose stencil halo matches (3 for PLM, 5 for PPM),
// which is what the window plan is made for.
#include "ram_device.h"

#include <type_traits>

namespace ram {
namespace {

using namespace dev;

constexpr int kWinSh = 1536;                    // LDS window capacity, cells
constexpr int kWinRegs = kWinSh / kBlock;       // window cells per thread
constexpr int kPad = 8;                         // residual arrays: halo slack

// The FP32 residual stages its (dx, 1/gap) records in LDS; FP64 reads them
// from the (cache-resident) table, which keeps its LDS at four blocks a CU.
template <typename CT> struct StageRR { static constexpr bool on = sizeof(CT) == 4; };

template <typename M, typename A, typename CT, bool kDirect, int NX, int NODES>
struct ShLds {
    using CT2 = typename TabT<CT>::T2;
    // NX: window arrays of a limited reconstruction beside the masses
    static constexpr size_t win =
        sizeof(M) * kWinSh * (1 + NX) + (kDirect ? 0 : sizeof(A) * (kWinSh + 1));
    static constexpr size_t res =
        (2 * sizeof(CT) + (StageRR<CT>::on ? sizeof(CT2) : 0)) * (NODES + kPad);
    static constexpr size_t nodes = sizeof(int64_t) * NODES;
    static constexpr size_t u0 = win > res ? win : res;
    static constexpr size_t uni = u0 > nodes ? u0 : nodes;
};

// Window plan: extended source index of each tile's first node minus lo
// (wlo_out), the window length or -1 when it exceeds the LDS capacity
// (w_out[tile]), and the window start inside the row, wlo mod n
// (w_out[n_tiles + tile]).
template <int P>
__global__ __launch_bounds__(256) void k_plan(StepArgs a, int64_t *wlo_out,
                                              int32_t *w_out)
{
    constexpr int LO = (P - 1) / 2;
    const int64_t tile = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
    const RowShift rs = row_shift(a.v0[row] * a.dt, len, R.tab.scal[1]);
    double xt0;
    int c0;
    const int64_t g0 = node_locate(x, n, R.tab, rs, i0 - H, xt0, c0);
    const int64_t g1 = node_index(x, n, R.tab, rs, len, i0 + nd + H);
    const int64_t wide = g1 - g0 + P;
    const int64_t wlo = g0 - LO;
    wlo_out[tile] = wlo;
    w_out[tile] = (wide >= P && wide <= kWinSh) ? (int32_t)wide : -1;
    // the window start inside the row, wlo mod n
    const int64_t kk = wlo >= 0 ? wlo / n : -((-wlo + n - 1) / n);
    w_out[R.n_tiles + tile] = (int32_t)(wlo - kk * n);
    // a uniform tile: the cells on both sides of its nodes and its source
    // window lie in one of the mesh's uniform runs (all cells at the largest
    // size, or all at the smallest), and the window holds exactly one
    // source cell per node (plus the stencil), so node i0 - H + k sits in
    // window cell LO + k at the first node's theta
    float thu = -1.0f;
    auto in_run = [&](const int32_t *pre) {
        return nonu_count(pre, n, i0 - H - 1, i0 + nd + H + 1) == 0 &&
               nonu_count(pre, n, wlo, wlo + wide) == 0;
    };
    if (R.tab.nonu && wide == nd + 2 * H + P && (in_run(R.tab.nonu) || in_run(R.tab.nonu_min)))
        thu = (float)((xt0 - x[c0]) * R.tab.dxinv[c0]);
    w_out[2 * R.n_tiles + tile] = __float_as_int(thu);
}

// Periodic index for j in [-n, 2n).
__device__ inline int wrap1(int j, int n)
{
    return j < 0 ? j + n : (j >= n ? j - n : j);
}

// Source cell of a wrapped shifted node from the mesh-density index: the
// closed-form floor(F(xt)), then checked against the nodes (a step either way
// while outside; any error in F only costs steps).
__device__ inline int density_cell(const double *x, int n, const MeshDensity &d, double xt)
{
    int c = (int)floor(d.scale * (bump_prim(xt, d) - d.p0));
    c = min(max(c, 0), n - 1);
    double lo = x[c], hi = x[c + 1];
    while (xt < lo && c > 0) {
        --c;
        hi = lo;
        lo = x[c];
    }
    while (xt >= hi && c + 1 < n) {
        ++c;
        lo = hi;
        hi = x[c + 1];
    }
    return c;
}

// A uniform tile of the FP32 Lagrange step: the plan found the tile's nodes
// and its source window in one uniform run of the mesh, so node k sits in
// window cell LO + k at one theta and each shifted cell value is the same
// (P+1)-point combination of the window's cell values (uniform_stencil); the
// residual's cell sizes and centre gaps are the run's.  No node search, no
// masses, no partial integrals, no per-cell geometry.  LDS: the shifted
// state and the fluxes as in the general path, the window cell values in
// the bytes of the staged cell records, so that no barrier separates them.
template <typename TQ, int P, int H, int NI>
__device__ __forceinline__ void step_uniform_tile(const StepArgs &a, unsigned char *su,
                                                  float thu, int row, int i0, int nd, int W,
                                                  int base, bool inner)
{
    static_assert(sizeof(TQ) == 4, "uniform tiles: FP32");
    using CT = TQ;
    using CT2 = typename TabT<CT>::T2;
    constexpr int NODES = kBlock * NI;
    static_assert(P <= kPad && 3 * sizeof(CT) * (NODES + kPad) <=
                  ShLds<CT, double, CT, true, 0, NODES>::uni, "uniform tile LDS");
    const int t = threadIdx.x;
    const Rows &R = a.rows;
    const MeshTab &tb = R.tab;
    const int n = (int)R.n_cols;
    const int NC = nd + 2 * H;
    const int64_t qoff = (int64_t)row * n;
    const TQ *q = (const TQ *)a.q_in + qoff;
    TQ *qo = (TQ *)a.q_out + qoff;
    TQ *qmid = a.q_mid ? (TQ *)a.q_mid + qoff : nullptr;
    CT *sq = (CT *)su;
    CT *sf = sq + (NODES + kPad);
    CT *sw = sf + (NODES + kPad);
    const bool wsmall = W + base <= 2 * n;
    TQ wq[kWinRegs];
#pragma unroll
    for (int r = 0; r < kWinRegs; ++r) {
        const int j = t + r * kBlock;
        if (j < W) {
            int mm = base + j;
            if (wsmall) mm = mm >= n ? mm - n : mm;
            else mm = wrap_small(mm, n);
            wq[r] = q[mm];
        }
    }
    TQ dvr[NI];
    if (H) {
        const TQ *dv = (const TQ *)a.dv + qoff;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int u = t + k * kBlock;
            if (u < nd + 1) {
                const int f = i0 + u;
                dvr[k] = dv[inner ? f : wrap1(f, n)];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < kWinRegs; ++r) {
        const int j = t + r * kBlock;
        if (j < W) sw[j] = (CT)wq[r];
    }
    CT cc[P + 1];
    uniform_stencil<CT, P>((CT)thu, cc);
    __syncthreads();
    // destination cell ci (cell i0 - H + ci) from window cells ci .. ci + P,
    // one cell at a time (sq does not overlap the window): six reads in
    // flight rather than the tile's twenty-four keep the registers of the
    // general path's occupancy
#pragma unroll 1
    for (int ci = t; ci < NC; ci += kBlock) {
        CT v = (CT)0;
#pragma unroll
        for (int d = 0; d <= P; ++d) v += cc[d] * sw[ci + d];
        const int c0 = i0 - H + ci;
        const int cell = inner ? c0 : wrap1(c0, n);
        if (H == 0) qo[cell] = (TQ)v;
        else {
            sq[ci] = v;
            if (qmid && ci >= H && ci < H + nd) qmid[cell] = (TQ)v;
        }
    }
    if (H == 0) return;
    __syncthreads();
    const CT2 rr0 = TabT<CT>::rr(tb)[i0];          // the run's (dx, 1 / centre gap)
    const CT dxi0 = TabT<CT>::dxinv(tb)[i0];
    // fluxes on faces i0 .. i0+nd (sq index j is cell i0-2+j), as in the
    // general path with the run's geometry
    const CT dt = (CT)a.dt;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int u = t + k * kBlock;
        if (u < nd + 1) {
            const CT v = (CT)dvr[k];
            const bool up = v >= (CT)0;
            const int c = up ? u + 1 : u + 2;
            const CT qm = sq[c - 1], q0 = sq[c], qp = sq[c + 1];
            const CT dp = (qp - q0) * rr0.y;
            const CT dm = (q0 - qm) * rr0.y;
            const CT sig = (dp * dm <= (CT)0) ? (CT)0 : harmonic2(dp, dm);
            const CT half = up ? (CT)0.5 * (rr0.x - v * dt) : (CT)-0.5 * (rr0.x + v * dt);
            sf[u] = v * (q0 + sig * half);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int u = t + k * kBlock;
        if (u < nd) qo[i0 + u] = (TQ)(sq[u + 2] - dt * (sf[u + 1] - sf[u]) * dxi0);
    }
}

// The FP32 Lagrange direct-sum schedule asks for seven waves a SIMD, the
// count its LDS allows: the compiler then fits it in 72 VGPRs (a spill or
// so) where it would otherwise take 74 and six waves.
template <typename TQ, int P, int S, int H, int RECON, int NI, int IDX>
constexpr int step_min_waves()
{
    return (S == kSumDirect && RECON == 0 && sizeof(TQ) == 4 && NI == kItems && IDX == 0) ? 7
                                                                                           : 1;
}

// IDX 1: the source cells come from the mesh-density index (a.dens) instead of
// the bucket index.
template <typename TQ, int P, int S, int H, int RECON = 0, int NI = kItems, int IDX = 0>
__global__ __launch_bounds__(kBlock, (step_min_waves<TQ, P, S, H, RECON, NI, IDX>()))
void k_step_sh(StepArgs a)
{
    constexpr bool kDirect = S == kSumDirect;
    constexpr bool kLim = RECON != 0;
    static_assert(!kLim || (kDirect && P == (RECON == kReconPLM ? 3 : 5)),
                  "limited reconstructions: direct sums, stencil halo of order 3 / 5");
    using AC = Acc<kDirect ? kScanF64 : S>;
    using M = typename std::conditional<kDirect, TQ, typename AC::M>::type;
    using A = typename AC::A;
    using CT = TQ;                       // arithmetic after the prefix sums
    using CT2 = typename TabT<CT>::T2;
    constexpr int NODES = kBlock * NI;   // shifted nodes per tile
    using L = ShLds<M, A, CT, kDirect, kLim ? 3 : 0, NODES>;
    constexpr int LO = (P - 1) / 2;
    constexpr int WCAP = kWinSh;

    __shared__ short sjc[NODES];         // window index of each node's cell (<= kWinSh)
    __shared__ CT sell[NODES];           // partial integral C~(xh) - C(c)
    __shared__ A swt[kBlock / 64];
    __shared__ __attribute__((aligned(16))) unsigned char su[L::uni];
    __shared__ int s_flag;
    M *sm = (M *)su;                                 // window masses
    A *sp = (A *)(su + sizeof(M) * WCAP);            // exclusive prefix
    int64_t *sg = (int64_t *)su;                     // direct path: node indices
    CT *sq = (CT *)su;                               // shifted state
    CT *sf = sq + (NODES + kPad);                    // face fluxes
    CT2 *srr = (CT2 *)(sf + (NODES + kPad));         // (dx, 1/gap) per cell
    // limited reconstructions, beside the window masses:
    //   PLM  sx1 averages, sx2 1/centre gap (j, j+1), sx3 kappa
    //   PPM  sx1 averages (then C), sx2 limited slopes (then A), sx3 interfaces
    CT *sx1 = (CT *)(su + sizeof(M) * WCAP);
    CT *sx2 = sx1 + WCAP;
    CT *sx3 = sx2 + WCAP;

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
    const double x0 = x[0], xN = x[n];
    const double len = xN - x0;
    const double bsc = tb.scal[0], invlen = tb.scal[1], bx0 = tb.scal[2];
    const double s = a.v0[row] * a.dt;
    const int64_t wlo = a.plan_wlo[blockIdx.x];
    const int W = a.plan_w[blockIdx.x];
    const int t = threadIdx.x;
    const RowShift rs = row_shift(s, len, invlen);
    // window index of a node = c + (dk + kx) n + jbase
    const int jbase = (int)(rs.kf0 * (int64_t)n - wlo);

    // A uniform tile (FP32, direct sums): the plan found its nodes and source
    // window in the mesh's uniform run, so node k of the tile sits in window
    // cell LO + k at one theta -- no search, no cell record; the Lagrange
    // shift becomes one stencil on the cell values (step_uniform_tile), the
    // limited shift evaluates each cell's cubic at that theta (per-node
    // values would agree to FP32 rounding).
    bool uni = false;
    float thu = -1.0f;
    if constexpr (kDirect && sizeof(TQ) == 4) {
        thu = __int_as_float(a.plan_w[2 * R.n_tiles + blockIdx.x]);
        uni = thu >= 0.0f;
        if constexpr (!kLim) {
            if (uni) {
                step_uniform_tile<TQ, P, H, NI>(a, su, thu, row, i0, nd, W,
                                                a.plan_w[R.n_tiles + blockIdx.x], inner);
                return;
            }
        }
    }
    // ---- loads that do not depend on the search, issued first ------------
    double xe[NI];
    int kxn[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int ei = t + k * kBlock;
        const int e = i0 - H + ei;
        kxn[k] = inner ? 0 : (e < 0 ? -n : (e >= n ? n : 0));
        xe[k] = (ei < NE && !uni) ? x[inner ? e : wrap1(e, n)] : x0;
    }
    // window start inside the row: wlo mod n
    const int base = a.plan_w[R.n_tiles + blockIdx.x];   // wlo mod n
    const bool wsmall = W + base <= 2 * n;
    M wq[kWinRegs], wd[kWinRegs];
    int wm[kWinRegs];                    // limited: the window cells' row index
    CT wg[kWinRegs];                     // PLM: 1 / centre gap (j, j+1)
#pragma unroll
    for (int r = 0; r < kWinRegs; ++r) {
        const int j = t + r * kBlock;
        if (j < W) {
            int mm = base + j;
            if (wsmall) mm = mm >= n ? mm - n : mm;
            else mm = wrap_small(mm, n);
            wq[r] = (M)q[mm];
            wd[r] = TabT<M>::dx(tb)[mm];
            if constexpr (kLim) wm[r] = mm;
            if constexpr (RECON == kReconPLM) wg[r] = TabT<CT>::hinv(tb)[mm];
        }
    }
#pragma unroll
    for (int r = 0; r < kWinRegs; ++r) {
        const int j = t + r * kBlock;
        if (j < W) {
            sm[j] = wq[r] * wd[r];
            if constexpr (kLim) sx1[j] = wq[r];
            if constexpr (RECON == kReconPLM) sx2[j] = wg[r];
        }
    }
    // ---- (A) shifted nodes: source index and stencil weights -------------
    // Direct sums: the window masses are visible after one barrier, so each
    // node's partial integral is formed as soon as its weights are, and the
    // weights die there; the registers that frees pay for issuing the four
    // nodes' bucket lookups together.  Prefix modes keep the weights until
    // the scan is done and look the nodes up one at a time.
    int jc[NI];
    CT w[NI][P + 1];
    bool ok = true;
    if (t == 0) s_flag = W > 0 ? 1 : 0;
    if constexpr (kDirect) {
        __syncthreads();
        if constexpr (RECON == kReconPLM) {
            // kappa = sigma dx^2 / 2 of window cells 1 .. W-2
#pragma unroll
            for (int r = 0; r < kWinRegs; ++r) {
                const int j = t + r * kBlock;
                if (j >= 1 && j < W - 1) {
                    const CT dp = (sx1[j + 1] - wq[r]) * sx2[j];
                    const CT dm = (wq[r] - sx1[j - 1]) * sx2[j - 1];
                    const CT sig = (dp * dm <= (CT)0) ? (CT)0 : harmonic2(dp, dm);
                    sx3[j] = (CT)0.5 * sig * wd[r] * wd[r];
                }
            }
            __syncthreads();
        } else if constexpr (RECON == kReconPPM) {
            const CT *pw;
            if constexpr (sizeof(CT) == 8) pw = (const CT *)tb.ppmd;
            else pw = (const CT *)tb.ppmf;
            // a uniform tile: the cells that take weights (window cells 1 ..
            // W-3) and their neighbours lie in the run, so one set serves
            // them all -- window cell 1's, whose neighbours (window cells
            // 0 .. 3) are in the window; window cell 0's left neighbour need
            // not be
            CT pu[5];
            if (uni) {
                const int c1 = base + 1 >= n ? base + 1 - n : base + 1;
#pragma unroll
                for (int k = 0; k < 5; ++k) pu[k] = pw[k * n + c1];
            }
            // limited slopes of window cells 1 .. W-2
#pragma unroll
            for (int r = 0; r < kWinRegs; ++r) {
                const int j = t + r * kBlock;
                if (j >= 1 && j < W - 1) {
                    CT d1, d2;
                    if (uni) {
                        d1 = pu[0];
                        d2 = pu[1];
                    } else {
                        d1 = pw[wm[r]];
                        d2 = pw[n + wm[r]];
                    }
                    sx2[j] = ppm_delta<CT>(sx1[j - 1], wq[r], sx1[j + 1], d1, d2);
                }
            }
            __syncthreads();
            // interface values between cells j and j+1, j = 1 .. W-3
#pragma unroll
            for (int r = 0; r < kWinRegs; ++r) {
                const int j = t + r * kBlock;
                if (j >= 1 && j < W - 2) {
                    const int m = wm[r];
                    CT e1, e2, e3;
                    if (uni) {
                        e1 = pu[2];
                        e2 = pu[3];
                        e3 = pu[4];
                    } else {
                        e1 = pw[2 * n + m];
                        e2 = pw[3 * n + m];
                        e3 = pw[4 * n + m];
                    }
                    sx3[j] = wq[r] + e1 * (sx1[j + 1] - wq[r]) + e2 * sx2[j + 1] + e3 * sx2[j];
                }
            }
            __syncthreads();
            // constrained parabolas of cells 2 .. W-3: A and C (B = M - A - C)
#pragma unroll
            for (int r = 0; r < kWinRegs; ++r) {
                const int j = t + r * kBlock;
                if (j >= 2 && j < W - 2) {
                    CT pa, pb, pc;
                    ppm_cubic<CT>(wq[r], sx3[j - 1], sx3[j], wd[r], pa, pb, pc);
                    sx2[j] = pa;           // the slopes are dead
                    sx1[j] = pc;           // so are the averages
                }
            }
            __syncthreads();
        }
        if (uni && kLim) {
            // the limited cubic of each node's cell at the shared theta
            const CT tt = (CT)thu;
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                const int ei = t + k * kBlock;
                jc[k] = 0;
                if (ei < NE) {
                    const int j = LO + ei;
                    jc[k] = j;
                    ok = ok && j + P - LO <= W;
                    CT ell;
                    if constexpr (RECON == kReconPLM) {
                        const CT kap = sx3[j];
                        ell = tt * ((CT)sm[j] - kap + tt * kap);
                    } else {
                        const CT pa = sx2[j], pc = sx1[j];
                        const CT pb = (CT)sm[j] - pa - pc;
                        ell = tt * (pa + tt * (pb + tt * pc));
                    }
                    sell[ei] = ell;
                    sjc[ei] = (short)j;
                }
            }
        } else {
        NodePos np[NI];
        int cb[NI];
        double2 nx[NI];
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            np[k] = node_pos(xe[k], rs, x0, xN, bsc, bx0, tb.nb);
            if constexpr (IDX == 0) {
                cb[k] = tb.bucket[np[k].b];
                nx[k] = tb.bnext[np[k].b];
            }
        }
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int ei = t + k * kBlock;
            jc[k] = 0;
            if (ei < NE) {
                int c;
                if constexpr (IDX == 1) {
                    c = density_cell(x, n, a.dens, np[k].xt);
                } else {
                    c = cell_from_bucket(cb[k], nx[k], np[k].xt);
                    if (np[k].xt >= nx[k].y) c = cell_walk(x, n, c, np[k].xt);
                }
                CT wk[P + 1];
                CT tt = (CT)0;
                if constexpr (kLim) {
                    const CellRec<CT> &rc = RecT<CT>::get(tb)[c];
                    tt = (CT)((np[k].xt - rc.xc) * rc.dxinv);
                } else {
                    rec_weights<CT, P>(RecT<CT>::get(tb)[c], np[k].xt, wk);
                }
                const int j = c + np[k].dk * n + kxn[k] + jbase;
                jc[k] = j;
                const bool in = j >= LO && j + P - LO <= W;
                ok = ok && in;
                CT ell = (CT)0;
                if (kLim && in) {
                    // the cell's cubic: PLM theta (M - kappa + theta kappa),
                    // PPM theta (A + theta (B + theta C))
                    if constexpr (RECON == kReconPLM) {
                        const CT kap = sx3[j];
                        ell = tt * ((CT)sm[j] - kap + tt * kap);
                    } else {
                        const CT pa = sx2[j], pc = sx1[j];
                        const CT pb = (CT)sm[j] - pa - pc;
                        ell = tt * (pa + tt * (pb + tt * pc));
                    }
                } else if (in) {
                    // C(j-lo+b) - C(j): the masses between, summed outward
                    CT up = (CT)0, dn = (CT)0;
#pragma unroll
                    for (int b = LO + 1; b <= P; ++b) {
                        up += (CT)sm[j + b - LO - 1];
                        ell += wk[b] * up;
                    }
#pragma unroll
                    for (int b = LO - 1; b >= 0; --b) {
                        dn += (CT)sm[j - LO + b];
                        ell -= wk[b] * dn;
                    }
                }
                sell[ei] = ell;
                sjc[ei] = (short)j;
            }
        }
        }
    } else {
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            // one node at a time: the guard keeps the four lookups from being
            // interleaved, which would cost more registers than the waves it
            // leaves room for are worth
            jc[k] = 0;
            if (t + k * kBlock < NE) {
                const NodePos np = node_pos(xe[k], rs, x0, xN, bsc, bx0, tb.nb);
                const double2 nx = tb.bnext[np.b];
                int c = cell_from_bucket(tb.bucket[np.b], nx, np.xt);
                if (np.xt >= nx.y) c = cell_walk(x, n, c, np.xt);
                rec_weights<CT, P>(RecT<CT>::get(tb)[c], np.xt, w[k]);
                jc[k] = c + np.dk * n + kxn[k] + jbase;
                ok = ok && jc[k] >= LO && jc[k] + P - LO <= W;
            }
        }
    }
    __syncthreads();
    if (!ok) s_flag = 0;
    // ---- (B) the block scan of the prefix modes ------------------------------
    __syncthreads();
    const bool windowed = s_flag != 0;
    if (windowed) {
        if constexpr (!kDirect) {
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
        }
        // ---- (C) partial integrals of the interpolated cumulative ----------
        if constexpr (!kDirect) {
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                const int ei = t + k * kBlock;
                if (ei < NE) {
                    const int j = jc[k];
                    const A pc = sp[j];
                    CT ell = (CT)0;
#pragma unroll
                    for (int b = 0; b <= P; ++b)
                        if (b != LO) ell += w[k][b] * (CT)AC::diff(sp[j - LO + b], pc);
                    sell[ei] = ell;
                    sjc[ei] = (short)j;
                }
            }
        }
    } else {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int ei = t + k * kBlock;
            if (ei < NE) {
                const int64_t g = (int64_t)jc[k] + wlo;
                sg[ei] = g;
                if constexpr (kLim) {
                    // the node's cell and wrapped position as the search found
                    // them, the profile from global memory
                    int e = i0 - H + ei;
                    e = e < 0 ? e + n : (e >= n ? e - n : e);
                    const NodePos np = node_pos(x[e], rs, x0, xN, bsc, bx0, tb.nb);
                    const double2 nx = tb.bnext[np.b];
                    int c = cell_from_bucket(tb.bucket[np.b], nx, np.xt);
                    if (np.xt >= nx.y) c = cell_walk(x, n, c, np.xt);
                    sell[ei] = (CT)lim_partial_global<TQ, RECON>(x, q, n, c, np.xt);
                } else {
                    sell[ei] = (CT)direct_partial<TQ, P>(x, q, n, len, s, invlen,
                                                         i0 - H + ei, g);
                }
            }
        }
    }
    // residual inputs, fetched while the partial integrals settle: per-cell mesh records of cells i0-2 .. i0+nd+1, face
    // velocities of faces i0 .. i0+nd, 1/dx of the tile's cells
    constexpr bool kStage = StageRR<CT>::on;
    CT2 rrv[NI];
    TQ dvr[NI];
    CT dxi[NI];
    if (H) {
        const TQ *dv = (const TQ *)a.dv + qoff;
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int u = t + k * kBlock;
            if (kStage && u < nd + 4) {
                const int c = i0 - 2 + u;
                rrv[k] = TabT<CT>::rr(tb)[inner ? c : wrap1(c, n)];
            }
            if (u < nd + 1) {
                const int f = i0 + u;
                dvr[k] = dv[inner ? f : wrap1(f, n)];
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
                CT whole;
                if constexpr (kDirect) {
                    // the first two whole cells as independent reads (a node
                    // step of at most two cells is the common case; ja + 1 <=
                    // W stays inside the LDS buffer), the rest in order
                    const CT m0 = (CT)sm[ja], m1 = (CT)sm[ja + 1];
                    whole = jb > ja ? m0 : (CT)0;
                    whole += jb > ja + 1 ? m1 : (CT)0;
                    for (int m = ja + 2; m < jb; ++m) whole += (CT)sm[m];
                } else {
                    whole = (jb - ja == 1) ? (CT)sm[ja] : (CT)AC::diff(sp[jb], sp[ja]);
                }
                mp = whole + (sell[ci + 1] - sell[ci]);
            } else {
                mp = (CT)(direct_whole<TQ>(x, q, n, sg[ci], sg[ci + 1]) +
                          ((double)sell[ci + 1] - (double)sell[ci]));
            }
            // 1/dx: from the cell's staged record (the residual's, loaded
            // before the barrier) where there is one, else from the table
            if constexpr (H != 0 && kStage) qs[k] = mp * __builtin_amdgcn_rcpf(rrv[k].x);
            else qs[k] = mp * TabT<CT>::dxinv(tb)[cell];
            if (H == 0) qo[cell] = (TQ)qs[k];
            else if (qmid && ci >= H && ci < H + nd) qmid[cell] = (TQ)qs[k];
        }
    }
    if (H == 0) return;
    __syncthreads();   // the window bytes become the residual's arrays
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int u = t + k * kBlock;
        if (u < NC) sq[u] = qs[k];
        if (kStage && u < nd + 4) srr[u] = rrv[k];
    }
    __syncthreads();

    // ---- (E) fluxes on faces i0 .. i0+nd, with the upwind cell's slope -----
    // face i0+u lies between cells i0+u-1 (index u+1) and i0+u (index u+2);
    // index j of sq / srr is cell i0-2+j
    const CT dt = (CT)a.dt;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int u = t + k * kBlock;
        if (u < nd + 1) {
            const CT v = (CT)dvr[k];
            const bool up = v >= (CT)0;
            const int c = up ? u + 1 : u + 2;             // upwind cell
            const CT qm = sq[c - 1], q0 = sq[c], qp = sq[c + 1];
            CT2 rc, rm;
            if constexpr (kStage) {
                rc = srr[c];
                rm = srr[c - 1];
            } else {
                const int cg = i0 - 2 + c;
                rc = TabT<CT>::rr(tb)[inner ? cg : wrap1(cg, n)];
                rm = TabT<CT>::rr(tb)[inner ? cg - 1 : wrap1(cg - 1, n)];
            }
            const CT dp = (qp - q0) * rc.y;               // gap (c, c+1)
            const CT dm = (q0 - qm) * rm.y;               // gap (c-1, c)
            const CT sig = (dp * dm <= (CT)0) ? (CT)0 : harmonic2(dp, dm);
            const CT half = up ? (CT)0.5 * (rc.x - v * dt) : (CT)-0.5 * (rc.x + v * dt);
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
hipError_t step_sh_h(const StepArgs &a, int scan, int items, hipStream_t st)
{
    const dim3 g((unsigned)a.rows.n_tiles), b(kBlock);
    switch (scan) {
    case kScanF64: hipLaunchKernelGGL((k_step_sh<TQ, P, kScanF64, H>), g, b, 0, st, a); break;
    case kScanTwoSum: hipLaunchKernelGGL((k_step_sh<TQ, P, kScanTwoSum, H>), g, b, 0, st, a); break;
    case kScanF32: hipLaunchKernelGGL((k_step_sh<TQ, P, kScanF32, H>), g, b, 0, st, a); break;
    default:
        // direct sums: the mesh-density index (default schedule), or the
        // schedule's shifted nodes per thread
        if (a.dens.kind != 0 && items == kItems) {
            hipLaunchKernelGGL((k_step_sh<TQ, P, kSumDirect, H, 0, kItems, 1>), g, b, 0, st, a);
            break;
        }
        switch (items) {
        case 2: hipLaunchKernelGGL((k_step_sh<TQ, P, kSumDirect, H, 0, 2>), g, b, 0, st, a); break;
        case 3: hipLaunchKernelGGL((k_step_sh<TQ, P, kSumDirect, H, 0, 3>), g, b, 0, st, a); break;
        case 5: hipLaunchKernelGGL((k_step_sh<TQ, P, kSumDirect, H, 0, 5>), g, b, 0, st, a); break;
        default: hipLaunchKernelGGL((k_step_sh<TQ, P, kSumDirect, H>), g, b, 0, st, a); break;
        }
        break;
    }
    return hipGetLastError();
}

template <typename TQ, int P>
hipError_t step_sh_scan(const StepArgs &a, int scan, int items, hipStream_t st)
{
    if (a.dv) return step_sh_h<TQ, P, 2>(a, scan, items, st);
    return step_sh_h<TQ, P, 0>(a, scan, items, st);
}

template <typename TQ>
hipError_t step_sh_order(const StepArgs &a, int scan, int order, int items, hipStream_t st)
{
    switch (order) {
    case 1: return step_sh_scan<TQ, 1>(a, scan, items, st);
    case 3: return step_sh_scan<TQ, 3>(a, scan, items, st);
    default: return step_sh_scan<TQ, 5>(a, scan, items, st);
    }
}

template <typename TQ, int R>
hipError_t step_sh_lim(const StepArgs &a, hipStream_t st)
{
    constexpr int P = R == kReconPLM ? 3 : 5;
    const dim3 g((unsigned)a.rows.n_tiles), b(kBlock);
    if (a.dv) hipLaunchKernelGGL((k_step_sh<TQ, P, kSumDirect, 2, R>), g, b, 0, st, a);
    else hipLaunchKernelGGL((k_step_sh<TQ, P, kSumDirect, 0, R>), g, b, 0, st, a);
    return hipGetLastError();
}

} // namespace

__global__ __launch_bounds__(256) void k_density_cells(MeshDensity d, int n, const double *x,
                                                      int64_t m, int32_t *cells)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= m) return;
    const int c = (int)floor(d.scale * (bump_prim(x[i], d) - d.p0));
    cells[i] = min(max(c, 0), n - 1);
}

hipError_t launch_density_cells(const MeshDensity &d, int n, const double *x, int64_t m,
                                int32_t *cells, hipStream_t stream)
{
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_density_cells, dim3((unsigned)((m + 255) / 256)), dim3(256), 0,
                       stream, d, n, x, m, cells);
    return hipGetLastError();
}

hipError_t launch_step_shared_limited(const StepArgs &a, bool f64, int recon,
                                      hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    if (a.fast.rec) return f64 ? hipErrorInvalidValue : launch_step_fast_lim(a, recon, stream);
    if (f64) return recon == kReconPLM ? step_sh_lim<double, kReconPLM>(a, stream)
                                       : step_sh_lim<double, kReconPPM>(a, stream);
    return recon == kReconPLM ? step_sh_lim<float, kReconPLM>(a, stream)
                              : step_sh_lim<float, kReconPPM>(a, stream);
}

hipError_t launch_plan(const StepArgs &a, int order, int64_t *wlo, int32_t *w,
                       hipStream_t stream)
{
    // one wave per workgroup: a few hundred waves of dependent searches, spread
    // over every CU rather than packed four to a workgroup
    const unsigned grid = (unsigned)((a.rows.n_tiles + 63) / 64);
    switch (order) {
    case 1: hipLaunchKernelGGL(k_plan<1>, dim3(grid), dim3(64), 0, stream, a, wlo, w); break;
    case 3: hipLaunchKernelGGL(k_plan<3>, dim3(grid), dim3(64), 0, stream, a, wlo, w); break;
    default: hipLaunchKernelGGL(k_plan<5>, dim3(grid), dim3(64), 0, stream, a, wlo, w); break;
    }
    return hipGetLastError();
}

hipError_t launch_step_shared(const StepArgs &a, bool f64, int scan, int order,
                              int items, hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    if (a.fast.rec)
        return f64 ? launch_step_fast64(a, order, scan, stream)
                   : launch_step_fast(a, order, scan, stream);
    if (a.rows.tile != step_tile_for(scan == kSumDirect ? items : kItems, a.dv != nullptr))
        return hipErrorInvalidValue;       // the tiles were planned for another schedule
    if (f64) return step_sh_order<double>(a, scan == kSumDirect ? kSumDirect : kScanF64,
                                          order, items, stream);
    return step_sh_order<float>(a, scan, order, items, stream);
}

} // namespace ram
