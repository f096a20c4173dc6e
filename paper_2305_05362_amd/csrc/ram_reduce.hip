// ram_reduce.hip -- per-row checks of a state (gfx950): the row's mass
// sum_i Q_i dx_i (the quantity Eq. qmass_total conserves), the L1 distance to
// a reference state weighted by dx, and max |Q|.
//
// One workgroup per row: the threads stride over the row's cells (coalesced),
// accumulate in FP64, and combine within each wave by cross-lane shuffles and
// across the four waves through LDS.  The combination order is fixed, so a
// result is reproducible run to run.
#include "ram_device.h"

namespace ram {
namespace {

using namespace dev;

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <typename TQ>
__global__ __launch_bounds__(kBlock) void k_row_norms(Rows R, const TQ *q, const TQ *qref,
                                                      double *out)
{
    __shared__ double sw[3][kBlock / 64];
    const int64_t row = blockIdx.x;
    if (row >= R.n_rows) return;
    int64_t off, n;
    const double *x;
    if (R.n_cols > 0) {
        off = row * R.n_cols;
        n = R.n_cols;
        x = R.shared ? R.edges : R.edges + row * (R.n_cols + 1);
    } else {
        off = R.row_ptr[row];
        n = R.row_ptr[row + 1] - off;
        x = R.edges + off + row;
    }
    const int t = threadIdx.x;
    double mass = 0.0, dist = 0.0, amax = 0.0;
    for (int64_t i = t; i < n; i += kBlock) {
        const double dx = x[i + 1] - x[i];
        const double v = (double)q[off + i];
        mass += v * dx;
        if (qref) dist += fabs(v - (double)qref[off + i]) * dx;
        amax = fmax(amax, fabs(v));
    }
    mass = wave_sum(mass);
    dist = wave_sum(dist);
    amax = wave_max(amax);
    if ((t & 63) == 0) {
        sw[0][t >> 6] = mass;
        sw[1][t >> 6] = dist;
        sw[2][t >> 6] = amax;
    }
    __syncthreads();
    if (t == 0) {
        double m = 0.0, d = 0.0, a = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) {
            m += sw[0][w];
            d += sw[1][w];
            a = fmax(a, sw[2][w]);
        }
        out[3 * row + 0] = m;
        out[3 * row + 1] = d;
        out[3 * row + 2] = a;
    }
}

} // namespace

hipError_t launch_row_norms(const Rows &R, bool f64, const void *q, const void *qref,
                            double *out, hipStream_t stream)
{
    if (R.n_rows <= 0) return hipSuccess;
    const dim3 g((unsigned)R.n_rows), b(kBlock);
    if (f64)
        hipLaunchKernelGGL(k_row_norms<double>, g, b, 0, stream, R, (const double *)q,
                           (const double *)qref, out);
    else
        hipLaunchKernelGGL(k_row_norms<float>, g, b, 0, stream, R, (const float *)q,
                           (const float *)qref, out);
    return hipGetLastError();
}

} // namespace ram
