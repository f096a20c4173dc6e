// ram_kernels.hip -- HIP kernels of the RAM advection step for gfx950.
//
// Layout: rows are independent periodic lines (paper Section 2).  Every kernel
// works on tiles of kTile consecutive destination cells of one row, one
// workgroup (kBlock threads = 4 wave64) per tile, row-major coalesced access.
//
//   k_shift      bulk shift (Section 3, Steps 1-3).  Per tile:
//                (1) each thread places one shifted node x~ = x - v0 dt on the
//                    periodic mesh: wrap count k and source cell c
//                    (Eq. condition_p);
//                (2) the tile's source window [g_first - lo, g_last - lo + p)
//                    is staged in LDS as cell masses M = Q dx (Eq. Qmass_i) and
//                    turned into an exclusive prefix (the cumulative integral)
//                    by a block scan in FP64, compensated FP32 or FP32;
//                (3) each node's partial integral of the reconstruction is the
//                    degree-p Lagrange interpolant of the window cumulative;
//                (4) destination mass = whole source cells in between + the
//                    two partial integrals (Eq. mass_shift_algo), divided by
//                    dx (Eq. step3).
//                Windows wider than the LDS capacity take a direct path that
//                sums masses from global memory.
//   k_residual   residual upwind step (Eq. splitting_second) with the van
//                Leer slope of Section 3.1; halo of two cells per side.
#include "ram_device.h"

namespace ram {
namespace {

using namespace dev;

// Mass of (wrapped) cell m of a row, FP64.
template <typename TQ>
__device__ inline double cell_mass(const double *x, const TQ *q, int n, int64_t m)
{
    const int w = wrapi(m, n);
    return (double)q[w] * (x[w + 1] - x[w]);
}

// Partial integral C~(xh) - C(c) computed from global memory (direct path).
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

// ---------------------------------------------------------------------------
// bulk shift
// ---------------------------------------------------------------------------

template <typename TQ, int P, int S>
__global__ __launch_bounds__(kBlock) void k_shift(ShiftArgs a)
{
    using AC = Acc<S>;
    using M = typename AC::M;
    using A = typename AC::A;
    constexpr int LO = (P - 1) / 2;

    __shared__ int64_t sg[kTile + 1];   // extended source index g = c + k N
    __shared__ double sxh[kTile + 1];   // wrapped shifted node
    __shared__ double sell[kTile + 1];  // partial integral C~(xh) - C(c)
    __shared__ int sj[kTile + 1];       // window index of node c
    __shared__ M sm[kWindowCap];        // window cell masses
    __shared__ A sp[kWindowCap + 1];    // exclusive prefix of sm
    __shared__ A swt[kBlock / 64];

    Tile ti;
    if (!get_tile(a.rows, blockIdx.x, ti)) return;
    const int n = ti.n;
    if (n < P + 1) return;
    const double *x = ti.x;
    const TQ *q = (const TQ *)a.q_in + ti.qoff;
    TQ *qo = (TQ *)a.q_out + ti.qoff;
    const double s = a.v0[ti.row] * a.dt;
    const double len = x[n] - x[0];
    const int nd = min(kTile, n - ti.i0);
    const int ne = nd + 1;

    // (1) shifted nodes and their source cells; node N is node 0 of the next
    // period.
    for (int t = threadIdx.x; t < ne; t += kBlock) {
        const int e = ti.i0 + t;
        double xh;
        int64_t k;
        if (e == n) {
            shifted_node(x, n, s, 0, xh, k);
            k += 1;
        } else {
            shifted_node(x, n, s, e, xh, k);
        }
        const int c = find_cell(x, n, xh);
        sg[t] = (int64_t)c + k * (int64_t)n;
        sxh[t] = xh;
    }
    __syncthreads();

    // the source index of the shifted nodes is non-decreasing along the tile;
    // anything else (never expected) takes the direct path, which has no
    // LDS indexing to protect
    __shared__ int s_order_ok;
    if (threadIdx.x == 0) s_order_ok = 1;
    __syncthreads();
    for (int t = threadIdx.x + 1; t < ne; t += kBlock)
        if (sg[t] < sg[t - 1]) s_order_ok = 0;
    __syncthreads();

    const int64_t g0 = sg[0];
    const int64_t wide = sg[ne - 1] - g0 + P;
    if (s_order_ok && wide <= kWindowCap) {
        const int W = (int)wide;
        const int64_t wlo = g0 - LO;
        const int base = wrapi(wlo, n);
        // (2) window masses, then the block scan into the cumulative
        for (int j = threadIdx.x; j < W; j += kBlock) {
            const int mm = (base + j) % n;
            sm[j] = AC::template mass<TQ>(q[mm], x[mm + 1] - x[mm]);
        }
        __syncthreads();
        const int per = (W + kBlock - 1) / kBlock;
        const int j0 = min(W, (int)threadIdx.x * per);
        const int j1 = min(W, j0 + per);
        A run = AC::zero();
        for (int j = j0; j < j1; ++j) run = AC::add(run, sm[j]);
        A total;
        A acc = block_exscan<AC>(run, swt, total);
        for (int j = j0; j < j1; ++j) {
            sp[j] = acc;
            acc = AC::add(acc, sm[j]);
        }
        if (threadIdx.x == 0) sp[W] = total;
        __syncthreads();
        // (3) partial integrals from the interpolated cumulative
        for (int t = threadIdx.x; t < ne; t += kBlock) {
            const int64_t g = sg[t];
            const double xh = sxh[t];
            const int c = wrapi(g, n);
            const int jc = (int)(g - wlo);
            double X[P + 1], w[P + 1];
#pragma unroll
            for (int b = 0; b <= P; ++b) X[b] = node_x(x, n, len, c - LO + b);
            lagrange_weights<P>(xh, X, w);
            double ell = 0.0;
            const A pc = sp[jc];
#pragma unroll
            for (int b = 0; b <= P; ++b)
                if (b != LO) ell += w[b] * AC::diff(sp[jc - LO + b], pc);
            sell[t] = ell;
            sj[t] = jc;
        }
        __syncthreads();
        // (4) destination mass and Step 3
        for (int t = threadIdx.x; t < nd; t += kBlock) {
            const int ja = sj[t], jb = sj[t + 1];
            const double whole = (jb - ja == 1) ? (double)sm[ja]
                                                : AC::diff(sp[jb], sp[ja]);
            const double mp = whole + (sell[t + 1] - sell[t]);
            const int i = ti.i0 + t;
            qo[i] = (TQ)(mp / (x[i + 1] - x[i]));
        }
    } else {
        // direct path for windows wider than the LDS capacity
        for (int t = threadIdx.x; t < ne; t += kBlock)
            sell[t] = partial_direct<TQ, P>(x, q, n, len, sg[t], sxh[t]);
        __syncthreads();
        for (int t = threadIdx.x; t < nd; t += kBlock) {
            double whole = 0.0;
            for (int64_t m = sg[t]; m < sg[t + 1]; ++m) whole += cell_mass(x, q, n, m);
            const double mp = whole + (sell[t + 1] - sell[t]);
            const int i = ti.i0 + t;
            qo[i] = (TQ)(mp / (x[i + 1] - x[i]));
        }
    }
}

// ---------------------------------------------------------------------------
// residual upwind step
// ---------------------------------------------------------------------------

template <typename TQ>
__global__ __launch_bounds__(kBlock) void k_residual(ResidualArgs a)
{
    __shared__ double sq[kTile + 4];    // cells i0-2 .. i0+nd+1
    __shared__ double ssig[kTile + 2];  // slopes of cells i0-1 .. i0+nd
    __shared__ double sf[kTile + 1];    // fluxes on faces i0 .. i0+nd

    Tile ti;
    if (!get_tile(a.rows, blockIdx.x, ti)) return;
    const int n = ti.n;
    const double *x = ti.x;
    const TQ *q = (const TQ *)a.q_in + ti.qoff;
    const TQ *dv = (const TQ *)a.dv + ti.qoff;
    TQ *qo = (TQ *)a.q_out + ti.qoff;
    const double dt = a.dt;
    const double len = x[n] - x[0];
    const int i0 = ti.i0;
    const int nd = min(kTile, n - i0);

    for (int t = threadIdx.x; t < nd + 4; t += kBlock)
        sq[t] = (double)q[wrapi((int64_t)i0 - 2 + t, n)];
    __syncthreads();
    for (int t = threadIdx.x; t < nd + 2; t += kBlock) {
        const int64_t i = (int64_t)i0 - 1 + t;
        const double dp = (sq[t + 2] - sq[t + 1]) / centre_gap(x, n, len, i);
        const double dm = (sq[t + 1] - sq[t]) / centre_gap(x, n, len, i - 1);
        ssig[t] = (dp * dm <= 0.0) ? 0.0 : 2.0 * dp * dm / (dp + dm);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nd + 1; t += kBlock) {
        const int64_t f = (int64_t)i0 + t;
        const double v = (double)dv[wrapi(f, n)];
        double qs;
        if (v >= 0.0) {
            const int u = wrapi(f - 1, n);
            qs = sq[t + 1] + 0.5 * ssig[t] * ((x[u + 1] - x[u]) - v * dt);
        } else {
            const int u = wrapi(f, n);
            qs = sq[t + 2] - 0.5 * ssig[t + 1] * ((x[u + 1] - x[u]) + v * dt);
        }
        sf[t] = v * qs;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nd; t += kBlock) {
        const int i = i0 + t;
        qo[i] = (TQ)(sq[t + 2] - dt * (sf[t + 1] - sf[t]) / (x[i + 1] - x[i]));
    }
}

// ---------------------------------------------------------------------------
// ragged-row tile table: tile_ptr[r] = sum_{r'<r} ceil(N_r'/kTile) and
// tile_row[t] = row of tile t.  One workgroup of 1024 threads.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(1024) void k_tiles_prep(const int64_t *row_ptr,
                                                     int64_t n_rows,
                                                     int64_t *tile_ptr,
                                                     int32_t *tile_row)
{
    __shared__ int64_t stot[1024];
    const int64_t per = (n_rows + 1023) / 1024;
    const int64_t r0 = min(n_rows, (int64_t)threadIdx.x * per);
    const int64_t r1 = min(n_rows, r0 + per);
    int64_t run = 0;
    for (int64_t r = r0; r < r1; ++r)
        run += (row_ptr[r + 1] - row_ptr[r] + kTile - 1) / kTile;
    stot[threadIdx.x] = run;
    __syncthreads();
    // inclusive Hillis-Steele scan of the 1024 chunk totals
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t o = threadIdx.x >= (unsigned)d ? stot[threadIdx.x - d] : 0;
        __syncthreads();
        stot[threadIdx.x] += o;
        __syncthreads();
    }
    int64_t acc = stot[threadIdx.x] - run;
    for (int64_t r = r0; r < r1; ++r) {
        tile_ptr[r] = acc;
        const int64_t nt = (row_ptr[r + 1] - row_ptr[r] + kTile - 1) / kTile;
        for (int64_t t = 0; t < nt; ++t) tile_row[acc + t] = (int32_t)r;
        acc += nt;
    }
    if (threadIdx.x == 1023) tile_ptr[n_rows] = stot[1023];
}

template <typename TQ, int P>
hipError_t shift_dispatch_scan(const ShiftArgs &a, int scan, hipStream_t st)
{
    const dim3 grid((unsigned)a.rows.n_tiles), block(kBlock);
    switch (scan) {
    case kScanF64:
        hipLaunchKernelGGL((k_shift<TQ, P, kScanF64>), grid, block, 0, st, a);
        break;
    case kScanTwoSum:
        hipLaunchKernelGGL((k_shift<TQ, P, kScanTwoSum>), grid, block, 0, st, a);
        break;
    default:
        hipLaunchKernelGGL((k_shift<TQ, P, kScanF32>), grid, block, 0, st, a);
        break;
    }
    return hipGetLastError();
}

template <typename TQ>
hipError_t shift_dispatch(const ShiftArgs &a, int scan, int order, hipStream_t st)
{
    switch (order) {
    case 1: return shift_dispatch_scan<TQ, 1>(a, scan, st);
    case 3: return shift_dispatch_scan<TQ, 3>(a, scan, st);
    default: return shift_dispatch_scan<TQ, 5>(a, scan, st);
    }
}

} // namespace

hipError_t launch_tiles_prep(const int64_t *row_ptr, int64_t n_rows,
                             int64_t *tile_ptr, int32_t *tile_row,
                             hipStream_t stream)
{
    hipLaunchKernelGGL(k_tiles_prep, dim3(1), dim3(1024), 0, stream, row_ptr,
                       n_rows, tile_ptr, tile_row);
    return hipGetLastError();
}

hipError_t launch_shift(const ShiftArgs &a, bool f64, int scan, int order,
                        hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    // FP64 state always scans in FP64
    if (f64) return shift_dispatch<double>(a, kScanF64, order, stream);
    return shift_dispatch<float>(a, scan, order, stream);
}

hipError_t launch_residual(const ResidualArgs &a, bool f64, hipStream_t stream)
{
    if (a.rows.n_tiles <= 0) return hipSuccess;
    const dim3 grid((unsigned)a.rows.n_tiles), block(kBlock);
    if (f64)
        hipLaunchKernelGGL(k_residual<double>, grid, block, 0, stream, a);
    else
        hipLaunchKernelGGL(k_residual<float>, grid, block, 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, int64_t bytes,
                       hipStream_t stream)
{
    return hipMemcpyAsync(dst, src, (size_t)bytes, hipMemcpyDeviceToDevice,
                          stream);
}

} // namespace ram
