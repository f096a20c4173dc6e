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
// Layout and schedule.  A lane owns one column and marches down a strip of S
// rows; the 256 lanes of a workgroup take 256 consecutive columns, so every
// load of a row (q, and u on the faces) is one coalesced 1 KiB (FP32) row
// segment and each value is read from HBM once (the 4 halo rows a strip
// shares with its neighbours come from L2: with 2^k column tiles per row the
// strips of one column tile land on the same XCD).  The strip is unrolled:
// its S + 4 state rows and S + 1 face rows are all in flight at once, and the
// slopes and fluxes live in registers.  The row geometry (widths, inverse
// centre gaps, face radii, inverse areas) is uniform across the workgroup:
// it is computed once per strip in FP64 into LDS instead of per lane.
#include "ram_device.h"

namespace ram {
namespace {

using namespace dev;

constexpr int kRadBlock = 256;

template <typename TQ, int S>
__global__ __launch_bounds__(kRadBlock) void k_radial(RadialArgs a)
{
    using CT = TQ;
    // geometry of rows j0-2 .. j0+S+1 (index w - j0 + 2)
    __shared__ CT s_width[S + 4];     // re[w+1] - re[w]
    __shared__ CT s_gap[S + 4];       // 1 / (c[w+1] - c[w]), c the arithmetic centre
    __shared__ CT s_rf[S + 4];        // re[w] (the radius of face w)
    __shared__ CT s_ia[S + 4];        // 2 / (re[w+1]^2 - re[w]^2)
    const int R = (int)a.n_rows;
    const int64_t N = a.n_cols;
    const int j0 = (int)blockIdx.y * S;
    const double *re = a.r_edges;
    for (int t = threadIdx.x; t < S + 4; t += kRadBlock) {
        const int w = j0 - 2 + t;
        CT wd = 0, gp = 0, rf = 0, ia = 0;
        if (w >= 0 && w < R) {
            wd = (CT)(re[w + 1] - re[w]);
            ia = (CT)(2.0 / (re[w + 1] * re[w + 1] - re[w] * re[w]));
            if (w + 1 < R) {
                const double c0 = 0.5 * (re[w] + re[w + 1]), c1 = 0.5 * (re[w + 1] + re[w + 2]);
                gp = (CT)(1.0 / (c1 - c0));
            }
        }
        if (w >= 0 && w <= R) rf = (CT)re[w];
        s_width[t] = wd;
        s_gap[t] = gp;
        s_rf[t] = rf;
        s_ia[t] = ia;
    }
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kRadBlock + threadIdx.x;
    if (i >= N) return;
    const TQ *q = (const TQ *)a.q_in;
    const TQ *u = (const TQ *)a.u;
    TQ *qo = (TQ *)a.q_out;
    const CT dt = (CT)a.dt;
    // state rows j0-2 .. j0+S+1, clamped into the grid (a clamped row is
    // never used: the edge rows have zero slope and the edge faces no flux)
    CT Q[S + 4];
#pragma unroll
    for (int k = 0; k < S + 4; ++k) {
        const int w = min(max(j0 - 2 + k, 0), R - 1);
        Q[k] = (CT)q[(int64_t)w * N + i];
    }
    // face velocities on faces j0 .. j0+S, clamped into 0..R
    CT U[S + 1];
#pragma unroll
    for (int k = 0; k <= S; ++k) {
        const int f = min(j0 + k, R);
        U[k] = (CT)u[(int64_t)f * N + i];
    }
    // van Leer slopes of rows j0-1 .. j0+S (index k: row j0-1+k)
    CT sl[S + 2];
#pragma unroll
    for (int k = 0; k < S + 2; ++k) {
        const int w = j0 - 1 + k;
        const int t = k + 1;                       // geometry / Q index of row w
        CT s = 0;
        if (w > 0 && w < R - 1) {
            const CT dp = (Q[t + 1] - Q[t]) * s_gap[t];
            const CT dm = (Q[t] - Q[t - 1]) * s_gap[t - 1];
            s = (dp * dm <= (CT)0) ? (CT)0 : harmonic2(dp, dm);
        }
        sl[k] = s;
    }
    // r-weighted fluxes through faces j0 .. j0+S
    CT F[S + 1];
#pragma unroll
    for (int k = 0; k <= S; ++k) {
        const int f = j0 + k;
        CT fl = 0;
        if (f > 0 && f < R) {
            const CT v = U[k];
            CT qs;
            if (v >= (CT)0) {                      // upwind row f-1
                qs = Q[k + 1] + (CT)0.5 * sl[k] * (s_width[k + 1] - v * dt);
            } else {                               // upwind row f
                qs = Q[k + 2] - (CT)0.5 * sl[k + 1] * (s_width[k + 2] + v * dt);
            }
            fl = s_rf[k + 2] * v * qs;
        }
        F[k] = fl;
    }
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const int j = j0 + k;
        if (j < R)
            qo[(int64_t)j * N + i] = (TQ)(Q[k + 2] - dt * (F[k + 1] - F[k]) * s_ia[k + 2]);
    }
}

} // namespace

hipError_t launch_radial(const RadialArgs &a, bool f64, hipStream_t stream)
{
    if (a.n_rows <= 0 || a.n_cols <= 0) return hipSuccess;
    const unsigned gx = (unsigned)((a.n_cols + kRadBlock - 1) / kRadBlock);
    const dim3 b(kRadBlock);
    if (f64) {
        constexpr int S = 8;
        const dim3 g(gx, (unsigned)((a.n_rows + S - 1) / S));
        hipLaunchKernelGGL((k_radial<double, S>), g, b, 0, stream, a);
    } else {
        constexpr int S = 16;
        const dim3 g(gx, (unsigned)((a.n_rows + S - 1) / S));
        hipLaunchKernelGGL((k_radial<float, S>), g, b, 0, stream, a);
    }
    return hipGetLastError();
}

} // namespace ram
