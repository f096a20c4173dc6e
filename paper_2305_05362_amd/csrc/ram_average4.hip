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
// One workgroup per tile of 1024 cells of a row, four cells per lane strided
// by the workgroup width, so every load and store is coalesced; the
// neighbours' values come from the same lines (L1/L2).  On a mesh shared by
// every row the two weights of each cell are tabulated once per call (FP64
// from the nodes, one division, then cast) and read from cache, so the kernel
// streams 8 (FP32) or 16 (FP64) bytes a cell and is bound by HBM; per-row and
// ragged meshes form them from the row's nodes in the kernel.
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

// w: the shared mesh's weights (then every row reads the same cached table),
// or null (per-row and ragged meshes: formed from the row's nodes).
template <typename TQ, bool INV>
__global__ __launch_bounds__(kBlock) void k_average4(Rows R, const TQ *q, TQ *out, const TQ *w)
{
    using T2 = typename std::conditional<sizeof(TQ) == 4, float2, double2>::type;
    Tile ti;
    if (!get_tile(R, blockIdx.x, ti)) return;
    const int n = ti.n;
    const double *x = ti.x;
    const double len = x[n] - x[0];
    const TQ *qr = q + ti.qoff;
    TQ *orow = out + ti.qoff;
#pragma unroll
    for (int k = 0; k < kAvgItems; ++k) {
        const int i = ti.i0 + k * kBlock + (int)threadIdx.x;
        if (i >= n) break;
        TQ wp, wm;
        if (w) {
            const T2 ww = ((const T2 *)w)[i];
            wp = ww.x;
            wm = ww.y;
        } else {
            double dp, dm;
            avg4_weights(x, n, len, i, dp, dm);
            wp = (TQ)dp;
            wm = (TQ)dm;
        }
        const TQ qm = qr[i == 0 ? n - 1 : i - 1], q0 = qr[i], qp = qr[i == n - 1 ? 0 : i + 1];
        const TQ corr = wp * (qp - q0) - wm * (q0 - qm);
        orow[i] = INV ? q0 - corr : q0 + corr;
    }
}

} // namespace

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
    if (R.n_tiles <= 0) return hipSuccess;
    if (R.tile != kAvgTile) return hipErrorInvalidValue;
    const dim3 g((unsigned)R.n_tiles), b(kBlock);
    if (f64) {
        const double *wd = (const double *)w;
        if (inverse)
            hipLaunchKernelGGL((k_average4<double, true>), g, b, 0, stream, R,
                               (const double *)in, (double *)out, wd);
        else
            hipLaunchKernelGGL((k_average4<double, false>), g, b, 0, stream, R,
                               (const double *)in, (double *)out, wd);
    } else {
        const float *wf = (const float *)w;
        if (inverse)
            hipLaunchKernelGGL((k_average4<float, true>), g, b, 0, stream, R,
                               (const float *)in, (float *)out, wf);
        else
            hipLaunchKernelGGL((k_average4<float, false>), g, b, 0, stream, R,
                               (const float *)in, (float *)out, wf);
    }
    return hipGetLastError();
}

} // namespace ram
