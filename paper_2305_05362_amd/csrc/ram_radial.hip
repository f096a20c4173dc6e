// ram_radial.hip -- radial transport of a polar grid on gfx950: the standard
// upwind half of a 2D dimensionally split step (RAM along the bulk flow in
// azimuth, standard transport across it in radius).
//
// Rows are radii bounded by the radial edges re[0..R]; every azimuthal column
// is advected along r with the residual's upwind scheme (PLM, van Leer slope
// from centre gaps, swept-interval face value) in polar geometry: per unit
// angle, face j (between rows j-1 and j) has length re[j] and row j the area
// A_j = (re[j+1]^2 - re[j]^2) / 2,
//     q'_j = q_j - dt (re[j+1] F_{j+1} - re[j] F_j) / A_j,   F = u q*.
// No flux crosses the inner and outer edges; the edge rows take a zero slope.
//
// One thread per cell, a workgroup per 256 consecutive cells of one row, so
// every load of a neighbouring row (two up, two down) and of the radial face
// velocities is a coalesced row segment; the row geometry is uniform across
// the workgroup.
#include "ram_device.h"

namespace ram {
namespace {

using namespace dev;

template <typename TQ>
__global__ __launch_bounds__(256) void k_radial(RadialArgs a)
{
    using CT = TQ;
    const int R = (int)a.n_rows;
    const int64_t N = a.n_cols;
    const int j = (int)blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const double *re = a.r_edges;
    const TQ *q = (const TQ *)a.q_in;
    const TQ *u = (const TQ *)a.u;
    TQ *qo = (TQ *)a.q_out;
    auto Q = [&](int row) { return (CT)q[(int64_t)row * N + i]; };
    auto centre = [&](int row) { return 0.5 * (re[row] + re[row + 1]); };
    // van Leer slope of row w (zero in the edge rows)
    auto slope = [&](int w) -> CT {
        if (w <= 0 || w >= R - 1) return (CT)0;
        const CT gp = (CT)(1.0 / (centre(w + 1) - centre(w)));
        const CT gm = (CT)(1.0 / (centre(w) - centre(w - 1)));
        const CT dp = (Q(w + 1) - Q(w)) * gp, dm = (Q(w) - Q(w - 1)) * gm;
        return (dp * dm <= (CT)0) ? (CT)0 : harmonic2(dp, dm);
    };
    // r-weighted flux through face f (between rows f-1 and f)
    auto flux = [&](int f) -> CT {
        if (f == 0 || f == R) return (CT)0;
        const CT v = (CT)u[(int64_t)f * N + i];
        const CT dt = (CT)a.dt;
        CT qs;
        if (v >= (CT)0) {
            const int w = f - 1;
            qs = Q(w) + (CT)0.5 * slope(w) * ((CT)(re[w + 1] - re[w]) - v * dt);
        } else {
            const int w = f;
            qs = Q(w) - (CT)0.5 * slope(w) * ((CT)(re[w + 1] - re[w]) + v * dt);
        }
        return (CT)re[f] * v * qs;
    };
    const CT inv_area = (CT)(2.0 / (re[j + 1] * re[j + 1] - re[j] * re[j]));
    qo[(int64_t)j * N + i] = (TQ)(Q(j) - (CT)a.dt * (flux(j + 1) - flux(j)) * inv_area);
}

} // namespace

hipError_t launch_radial(const RadialArgs &a, bool f64, hipStream_t stream)
{
    if (a.n_rows <= 0 || a.n_cols <= 0) return hipSuccess;
    const dim3 g((unsigned)((a.n_cols + 255) / 256), (unsigned)a.n_rows), b(256);
    if (f64) hipLaunchKernelGGL(k_radial<double>, g, b, 0, stream, a);
    else hipLaunchKernelGGL(k_radial<float>, g, b, 0, stream, a);
    return hipGetLastError();
}

} // namespace ram
