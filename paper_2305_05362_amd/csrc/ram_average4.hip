// ram_average4.hip -- centre values <-> cell averages with the fourth-order
// correction (gfx950).
//
// Section 3.1 notes that reading the state Q_i as the cell average <Q>_i is a
// second-order assumption and names the fourth-order correction
// <Q>_i = Q_i + (Q_{i+1} - 2 Q_i + Q_{i-1}) / 24 on a uniform mesh.  With Q_i
// the value at the cell's centre the average is Q_i + dx_i^2 Q''_i / 24 to
// fourth order; on any mesh Q'' is the three-point second derivative through
// the centres of cells i-1, i, i+1 (periodic rows), which is the printed
// formula on a uniform mesh:
//     <Q>_i = Q_i + w+_i (Q_{i+1} - Q_i) - w-_i (Q_i - Q_{i-1}),
//     w+-_i = dx_i^2 / (12 g+- (g- + g+)),   g+- the centre gaps either side.
// The inverse (averages -> centre values) subtracts the same correction
// formed from the averages.
//
// On a mesh shared by every row the two weights of each cell are tabulated
// once per call (FP64 from the nodes, one division, then cast) and read from
// cache, so the passes stream 8 (FP32) or 16 (FP64) bytes a cell and are
// bound by HBM; per-row and ragged meshes form them from the row's nodes in
// the kernel.
#include "ram_device.h"

#include <type_traits>

namespace ram {
namespace {

using namespace dev;

// The two weights of cell i (FP64, from the row's nodes; rows are periodic,
// so the neighbours of the end cells lie one period away).
__device__ inline void avg4_weights(const double *x, int n, double len, int i, double &wp,
                                    double &wm)
{
    const double c0 = 0.5 * (x[i] + x[i + 1]);
    const double cm = i == 0 ? 0.5 * (x[n - 1] + x[n]) - len : 0.5 * (x[i - 1] + x[i]);
    const double cp = i == n - 1 ? 0.5 * (x[0] + x[1]) + len : 0.5 * (x[i + 1] + x[i + 2]);
    const double gm = c0 - cm, gp = cp - c0;
    const double dx = x[i + 1] - x[i];
    const double c = dx * dx / (12.0 * gm * gp * (gm + gp));
    wp = c * gm;
    wm = c * gp;
}

// Weights of a mesh shared by every row, once per call: (w+, w-) per cell.
template <typename TQ>
__global__ __launch_bounds__(kBlock) void k_average4_weights(const double *x, int n, TQ *w)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double wp, wm;
    avg4_weights(x, n, x[n] - x[0], i, wp, wm);
    w[2 * i] = (TQ)wp;
    w[2 * i + 1] = (TQ)wm;
}

// One kernel for the three passes.  MODE 0: centre values -> averages,
// out_i = C(y)_i; MODE 1: averages -> centre values, out_i = C^-1(y)_i;
// MODE 2 (between two steps on centre values): out_i = C(C^-1(y))_i, the
// centre values in between never stored.  A workgroup takes a tile of up to
// 1024 cells of one row and stages its inputs (with a halo of one cell a
// side, two for MODE 2) and the weights in LDS: every lane issues all of its
// loads before the first store, and each input is read from global memory
// once.  MODE 2 keeps the intermediate centre values of the tile and one
// halo cell a side in LDS and applies C to them; each stage uses the same
// arithmetic as the separate passes.
// w: the shared mesh's weights (then every row reads the same cached table),
// or null (per-row and ragged meshes: formed from the row's nodes).
template <typename TQ, int MODE>
__global__ __launch_bounds__(kBlock) void k_average4(Rows R, const TQ *y, TQ *out, const TQ *w)
{
    using T2 = typename std::conditional<sizeof(TQ) == 4, float2, double2>::type;
    constexpr int HY = MODE == 2 ? 2 : 1;   // input halo a side
    constexpr int HW = MODE == 2 ? 1 : 0;   // weight halo a side
    constexpr int kSlots = kAvgItems + 1;   // covers the tile and its halo
    __shared__ TQ sy[kAvgTile + 2 * HY];    // y of cells i0-HY .. i0+nt-1+HY
    __shared__ T2 sw[kAvgTile + 2 * HW];    // weights of cells i0-HW .. i0+nt-1+HW
    __shared__ TQ sz[MODE == 2 ? kAvgTile + 2 : 1];   // C^-1(y), cells i0-1 .. i0+nt
    Tile ti;
    if (!get_tile(R, blockIdx.x, ti)) return;
    const int n = ti.n;
    const int i0 = ti.i0;
    const int nt = min(kAvgTile, n - i0);
    const double *x = ti.x;
    const double len = x[n] - x[0];
    const TQ *yr = y + ti.qoff;
    TQ *orow = out + ti.qoff;
    // periodic index for the halo (offsets of at most two cells; n >= 1)
    auto wrap = [&](int c) {
        c = c < 0 ? c + n : (c >= n ? c - n : c);
        return c < 0 ? c + n : (c >= n ? c - n : c);
    };
    TQ yv[kSlots];
    T2 wv[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
        const int j = k * kBlock + (int)threadIdx.x;
        yv[k] = yr[wrap(min(i0 - HY + j, i0 + nt - 1 + HY))];
        if (w) wv[k] = ((const T2 *)w)[wrap(min(i0 - HW + j, i0 + nt - 1 + HW))];
    }
#pragma unroll
    for (int k = 0; k < kSlots; ++k) {
        const int j = k * kBlock + (int)threadIdx.x;
        if (j < nt + 2 * HY) sy[j] = yv[k];
        if (j < nt + 2 * HW) {
            if (!w) {
                double dp, dm;
                avg4_weights(x, n, len, wrap(i0 - HW + j), dp, dm);
                wv[k].x = (TQ)dp;
                wv[k].y = (TQ)dm;
            }
            sw[j] = wv[k];
        }
    }
    __syncthreads();
    if constexpr (MODE == 2) {
        for (int j = threadIdx.x; j < nt + 2; j += kBlock) {
            const T2 ww = sw[j];
            const TQ ym = sy[j], y0 = sy[j + 1], yp = sy[j + 2];
            const TQ corr = ww.x * (yp - y0) - ww.y * (y0 - ym);
            sz[j] = y0 - corr;
        }
        __syncthreads();
    }
    const TQ *src = MODE == 2 ? sz : sy;
    for (int j = threadIdx.x; j < nt; j += kBlock) {
        const T2 ww = sw[j + HW];
        const TQ am = src[j], a0 = src[j + 1], ap = src[j + 2];
        const TQ corr = ww.x * (ap - a0) - ww.y * (a0 - am);
        orow[i0 + j] = MODE == 1 ? a0 - corr : a0 + corr;
    }
}

} // namespace

namespace {
template <typename TQ>
hipError_t avg4_launch(const Rows &R, int mode, const void *in, void *out, const void *w,
                       hipStream_t stream)
{
    if (R.n_tiles <= 0) return hipSuccess;
    if (R.tile != kAvgTile) return hipErrorInvalidValue;
    const dim3 g((unsigned)R.n_tiles), b(kBlock);
    const TQ *a = (const TQ *)in, *ww = (const TQ *)w;
    TQ *o = (TQ *)out;
    if (mode == 0) hipLaunchKernelGGL((k_average4<TQ, 0>), g, b, 0, stream, R, a, o, ww);
    else if (mode == 1) hipLaunchKernelGGL((k_average4<TQ, 1>), g, b, 0, stream, R, a, o, ww);
    else hipLaunchKernelGGL((k_average4<TQ, 2>), g, b, 0, stream, R, a, o, ww);
    return hipGetLastError();
}
} // namespace

hipError_t launch_average4_between(const Rows &R, bool f64, const void *in, void *out,
                                   const void *w, hipStream_t stream)
{
    return f64 ? avg4_launch<double>(R, 2, in, out, w, stream)
               : avg4_launch<float>(R, 2, in, out, w, stream);
}

hipError_t launch_average4_weights(const double *x, int64_t n, bool f64, void *w,
                                   hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const dim3 g((unsigned)((n + kBlock - 1) / kBlock)), b(kBlock);
    if (f64)
        hipLaunchKernelGGL(k_average4_weights<double>, g, b, 0, stream, x, (int)n, (double *)w);
    else
        hipLaunchKernelGGL(k_average4_weights<float>, g, b, 0, stream, x, (int)n, (float *)w);
    return hipGetLastError();
}

hipError_t launch_average4(const Rows &R, bool f64, bool inverse, const void *in, void *out,
                           const void *w, hipStream_t stream)
{
    const int mode = inverse ? 1 : 0;
    return f64 ? avg4_launch<double>(R, mode, in, out, w, stream)
               : avg4_launch<float>(R, mode, in, out, w, stream);
}

} // namespace ram
