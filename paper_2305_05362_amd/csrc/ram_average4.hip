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
// neighbours' values come from the same lines (L1/L2).  The weights are
// formed per cell in FP64 from the row's nodes (one division), so the kernel
// serves shared, per-row and ragged meshes alike; it streams 8 (FP32) or 16
// (FP64) bytes a cell and is bound by HBM.
#include "ram_device.h"

namespace ram {
namespace {

using namespace dev;

template <typename TQ, bool INV>
__global__ __launch_bounds__(kBlock) void k_average4(Rows R, const TQ *q, TQ *out)
{
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
        if (i >= ti.i0 + R.tile || i >= n) break;
        const double gm = centre_gap(x, n, len, (int64_t)i - 1);
        const double gp = centre_gap(x, n, len, i);
        const double dx = x[i + 1] - x[i];
        const double c = dx * dx / (12.0 * gm * gp * (gm + gp));
        const TQ wp = (TQ)(c * gm), wm = (TQ)(c * gp);
        const TQ qm = qr[i == 0 ? n - 1 : i - 1], q0 = qr[i], qp = qr[i == n - 1 ? 0 : i + 1];
        const TQ corr = wp * (qp - q0) - wm * (q0 - qm);
        orow[i] = INV ? q0 - corr : q0 + corr;
    }
}

} // namespace

hipError_t launch_average4(const Rows &R, bool f64, bool inverse, const void *in, void *out,
                           hipStream_t stream)
{
    if (R.n_tiles <= 0) return hipSuccess;
    if (R.tile != kAvgTile) return hipErrorInvalidValue;
    const dim3 g((unsigned)R.n_tiles), b(kBlock);
    if (f64) {
        if (inverse)
            hipLaunchKernelGGL((k_average4<double, true>), g, b, 0, stream, R,
                               (const double *)in, (double *)out);
        else
            hipLaunchKernelGGL((k_average4<double, false>), g, b, 0, stream, R,
                               (const double *)in, (double *)out);
    } else {
        if (inverse)
            hipLaunchKernelGGL((k_average4<float, true>), g, b, 0, stream, R,
                               (const float *)in, (float *)out);
        else
            hipLaunchKernelGGL((k_average4<float, false>), g, b, 0, stream, R,
                               (const float *)in, (float *)out);
    }
    return hipGetLastError();
}

} // namespace ram
