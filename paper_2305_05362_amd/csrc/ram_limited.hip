// ram_limited.hip -- bulk shift with the limited (monotone) reconstructions of
// Section 3.1 on gfx950 (PLM with the van Leer slope, or PPM with the
// interface values and constraints of App. A), for rows that each have their
// own mesh.  A mesh shared by every row takes the shared-mesh step kernel's
// limited mode instead (window plan, tables, fused residual).
//
// Same remap as the Lagrange shift (Section 3, Steps 1-3; Eq.
// mass_shift_algo): destination mass = the whole source cells between the two
// shifted nodes + the partial integrals of the reconstruction at both nodes.
// Only the partial integral changes: each source cell's limited profile is
// turned once into the cubic ell(theta) = theta (A + theta (B + theta C)),
// the integral of q_c from its left node to x_c + theta dx_c.
//
// One workgroup (four wave64) per tile of kStepNodes-1 destination cells of one
// row, kItems shifted nodes per thread:
//   (1) two threads locate the tile's first and last shifted nodes; the source
//       window is the cells between plus the reconstruction stencil (one cell
//       a side for PLM, two for PPM);
//   (2) every node finds its source cell by a binary search over the window's
//       nodes staged in LDS, and keeps theta in FP64;
//   (3) the window's averages, sizes and masses go to LDS (coalesced loads);
//   (4) every window cell's cubic is formed in LDS: PLM in one pass (slope
//       from the neighbouring averages), PPM in three (limited slopes, then
//       interface values, then the constrained parabolas);
//   (5) each node's ell from its cell's cubic; destination masses from the
//       window masses in between, times 1/dx (Eq. step3).
// The masses are summed directly in the state's type (no prefix sums).  Tiles
// whose window does not fit in LDS take a direct path that reads the stencil
// and the masses from global memory in FP64.
#include "ram_device.h"

namespace ram {
namespace {

using namespace dev;

constexpr int kWinLim = 1536;     // LDS window capacity, cells

template <typename CT>
struct LimLds {
    static constexpr size_t win = 5 * sizeof(CT) * kWinLim;
    static constexpr size_t stage = (sizeof(double) + sizeof(short)) * (kWinLim + 1);
    static constexpr size_t direct = (sizeof(int64_t) + sizeof(double)) * kStepNodes;
    static constexpr size_t u0 = win > stage ? win : stage;
    static constexpr size_t uni = u0 > direct ? u0 : direct;
};

// m mod n for m >= 0 (one subtraction in the common case)
__device__ inline int mod_pos(int m, int n)
{
    if (m < n) return m;
    m -= n;
    return m < n ? m : m % n;
}

// floor(a / n) for any a
__device__ inline int64_t floor_div(int64_t a, int n)
{
    return a >= 0 ? a / n : -((-a + n - 1) / n);
}

// Source cell and wrapped position of node e in [0, n] of a row: c, xh and
// the extended index g = c + k n (node n is node 0 one period on).
struct NodeLoc {
    int c;
    double xh;
    int64_t g;
};

__device__ inline NodeLoc locate_node(const double *x, int n, double len,
                                      double s, double invlen, int e)
{
    int kx = 0;
    if (e >= n) { e -= n; kx = 1; }
    NodeLoc r;
    double xh;
    int64_t k;
    shifted_node_inv(x, n, s, e, invlen, len, xh, k);
    r.c = find_cell(x, n, xh);
    r.xh = xh;
    r.g = (int64_t)r.c + (k + kx) * (int64_t)n;
    return r;
}

template <typename TQ, int R>
__global__ __launch_bounds__(kBlock) void k_shift_lim(StepArgs a)
{
    using CT = TQ;
    using L = LimLds<CT>;
    constexpr int LO = LimHalo<R>::lo;
    constexpr int NI = kItems;

    __shared__ short sjc[kStepNodes];     // window index of each node's cell
    __shared__ CT sell[kStepNodes];       // each node's partial integral
    __shared__ __attribute__((aligned(16))) unsigned char su[L::uni];
    __shared__ long long s_lo, s_hi;
    __shared__ int s_flag;
    CT *sm = (CT *)su;                    // window masses
    CT *sq = sm + kWinLim;                // averages     (PPM: then C)
    CT *sh = sq + kWinLim;                // sizes        (then B)
    CT *s1 = sh + kWinLim;                // PPM slopes   (then A)
    CT *s2 = s1 + kWinLim;                // PLM: 1/centre gap, PPM: interfaces
    double *sxs = (double *)su;           // per-row meshes: window nodes
    short *skq = (short *)(su + sizeof(double) * (kWinLim + 1));   // their periods
    int64_t *sg = (int64_t *)su;          // direct path: node indices
    double *sgl = (double *)(su + sizeof(int64_t) * kStepNodes);   // ... and ell

    const Rows &Rw = a.rows;
    Tile ti;
    if (!get_tile(Rw, blockIdx.x, ti)) return;
    const int n = ti.n;
    const int i0 = ti.i0;
    const int nd = min(Rw.tile, n - i0);
    const int NE = nd + 1;
    const double *x = ti.x;
    const TQ *q = (const TQ *)a.q_in + ti.qoff;
    TQ *qo = (TQ *)a.q_out + ti.qoff;
    const double s = a.v0[ti.row] * a.dt;
    const double len = x[n] - x[0];
    const double invlen = 1.0 / len;
    const int t = threadIdx.x;

    // ---- (1) the source window from the tile's end nodes --------------------
    if (t < 2) {
        const NodeLoc nl = locate_node(x, n, len, s, invlen, t == 0 ? i0 : i0 + nd);
        if (t == 0) s_lo = nl.g - LO;
        else s_hi = nl.g + LO + 1;
    }
    if (t == 0) s_flag = 1;
    __syncthreads();
    const int64_t wlo = s_lo;
    const int64_t wide = s_hi - s_lo;
    const bool fits = wide >= 2 * LO + 1 && wide <= kWinLim;
    const int W = fits ? (int)wide : 0;
    const int64_t pk0 = floor_div(wlo, n);          // period of the first window cell
    const int base = (int)(wlo - pk0 * n);         // wlo mod n

    // ---- (2) every node's source cell and theta ----------------------------
    int jc[NI];
    double th[NI];
    bool ok = fits;
    if (fits) {
        for (int j = t; j <= W; j += kBlock) {
            int m = base + j, kq = 0;
            if (m >= n) {
                kq = m / n;
                m -= kq * n;
            }
            sxs[j] = x[m];
            skq[j] = (short)kq;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int ei = t + k * kBlock;
            jc[k] = LO;
            th[k] = 0.0;
            if (ei < NE) {
                int e = i0 + ei, kx = 0;
                if (e >= n) { e -= n; kx = 1; }
                double xh;
                int64_t kk;
                shifted_node_inv(x, n, s, e, invlen, len, xh, kk);
                // the last window node at or below the shifted node,
                // comparing (period, coordinate) pairs exactly
                const int dk = (int)(kk + kx - pk0);
                auto le = [&](int j) {
                    const int kj = skq[j];
                    return kj < dk || (kj == dk && sxs[j] <= xh);
                };
                int lo = 0, hi = W + 1;
                if (le(0)) {
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (le(mid)) lo = mid;
                        else hi = mid;
                    }
                } else {
                    lo = -1;
                }
                if (lo >= LO && lo <= W - LO - 1) {
                    const int c = mod_pos(base + lo, n);
                    jc[k] = lo;
                    th[k] = (xh - sxs[lo]) / (x[c + 1] - x[c]);
                } else {
                    ok = false;
                }
            }
        }
    }
    __syncthreads();              // staged nodes are read; s_flag is settled
    if (!ok) s_flag = 0;
    __syncthreads();
    const bool windowed = s_flag != 0;

    if (windowed) {
        // ---- (3) window averages, sizes and masses -------------------------
        for (int j = t; j < W; j += kBlock) {
            const int m = mod_pos(base + j, n);
            const CT qv = (CT)q[m];
            const CT hv = (CT)(x[m + 1] - x[m]);
            sq[j] = qv;
            sh[j] = hv;
            sm[j] = qv * hv;
            if constexpr (R == kReconPLM) {
                // 1 / centre gap (j, j+1)
                const int m1 = mod_pos(m + 1, n);
                s2[j] = (CT)(2.0 / ((x[m + 1] - x[m]) + (x[m1 + 1] - x[m1])));
            }
        }
        __syncthreads();
        // ---- (4) every window cell's cubic -----------------------------------
        if constexpr (R == kReconPLM) {
            for (int j = t + 1; j < W - 1; j += kBlock) {
                CT A, B;
                const CT hv = sh[j];
                plm_cubic<CT>(sq[j - 1], sq[j], sq[j + 1], s2[j - 1], s2[j], sm[j], hv, A, B);
                s1[j] = A;
                sh[j] = B;           // cell j alone reads its own size
            }
        } else {
            // limited slopes of cells 1 .. W-2
            for (int j = t + 1; j < W - 1; j += kBlock) {
                const PpmW w = ppm_weights((double)sh[j - 1], (double)sh[j],
                                           (double)sh[j + 1], 1.0);
                s1[j] = ppm_delta<CT>(sq[j - 1], sq[j], sq[j + 1], (CT)w.d1, (CT)w.d2);
            }
            __syncthreads();
            // interface values between cells j and j+1, j = 1 .. W-3
            for (int j = t + 1; j < W - 2; j += kBlock) {
                const PpmW w = ppm_weights((double)sh[j - 1], (double)sh[j],
                                           (double)sh[j + 1], (double)sh[j + 2]);
                s2[j] = sq[j] + (CT)w.e1 * (sq[j + 1] - sq[j]) + (CT)w.e2 * s1[j + 1] +
                        (CT)w.e3 * s1[j];
            }
            __syncthreads();
            // constrained parabolas of cells 2 .. W-3
            for (int j = t + 2; j < W - 2; j += kBlock) {
                CT A, B, C;
                ppm_cubic<CT>(sq[j], s2[j - 1], s2[j], sh[j], A, B, C);
                s1[j] = A;           // the slopes are dead
                sh[j] = B;           // cell j alone reads its own size ...
                sq[j] = C;           // ... and its own average
            }
        }
        __syncthreads();
        // ---- (5a) partial integrals of the nodes -------------------------------
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int ei = t + k * kBlock;
            if (ei < NE) {
                const int j = jc[k];
                const CT tt = (CT)th[k];
                const CT C = (R == kReconPLM) ? (CT)0 : sq[j];
                sell[ei] = tt * (s1[j] + tt * (sh[j] + tt * C));
                sjc[ei] = (short)j;
            }
        }
        __syncthreads();
        // ---- (5b) destination masses, Step 3 ---------------------------------
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int ci = t + k * kBlock;
            if (ci < nd) {
                const int ja = sjc[ci], jb = sjc[ci + 1];
                CT whole = (CT)0;
                for (int m = ja; m < jb; ++m) whole += sm[m];
                const CT mp = whole + (sell[ci + 1] - sell[ci]);
                const int cell = i0 + ci;
                qo[cell] = (TQ)((double)mp / (x[cell + 1] - x[cell]));
            }
        }
        return;
    }

    // ---- direct path: stencils and masses from global memory, FP64 ----------
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int ei = t + k * kBlock;
        if (ei < NE) {
            const NodeLoc nl = locate_node(x, n, len, s, invlen, i0 + ei);
            sg[ei] = nl.g;
            sgl[ei] = lim_partial_global<TQ, R>(x, q, n, nl.c, nl.xh);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int ci = t + k * kBlock;
        if (ci < nd) {
            const int cell = i0 + ci;
            const double wh = direct_whole<TQ>(x, q, n, sg[ci], sg[ci + 1]);
            const double mp = wh + (sgl[ci + 1] - sgl[ci]);
            qo[cell] = (TQ)(mp / (x[cell + 1] - x[cell]));
        }
    }
}

template <typename TQ>
hipError_t shift_lim_t(const StepArgs &a, int recon, hipStream_t st)
{
    const dim3 g((unsigned)a.rows.n_tiles), b(kBlock);
    if (recon == kReconPLM) hipLaunchKernelGGL((k_shift_lim<TQ, kReconPLM>), g, b, 0, st, a);
    else hipLaunchKernelGGL((k_shift_lim<TQ, kReconPPM>), g, b, 0, st, a);
    return hipGetLastError();
}

} // namespace

hipError_t launch_shift_limited(const StepArgs &a, bool f64, int recon,
                                hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    if (f64) return shift_lim_t<double>(a, recon, stream);
    return shift_lim_t<float>(a, recon, stream);
}

} // namespace ram
