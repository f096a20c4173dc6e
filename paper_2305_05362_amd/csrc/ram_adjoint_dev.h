// ram_adjoint_dev.h -- device helpers of the shared-mesh adjoint kernels:
// a shifted node's search with its Lagrange weights, the x-derivatives of
// the weights, and the reconstruction at a node summed from global memory.
#pragma once

#include "ram_device.h"

namespace ram {
namespace dev {

// Shifted node -> extended source index g, its cell c, the wrapped position
// xh and the Lagrange weights of its stencil (the search of the step kernel).
template <typename WT, int P>
__device__ inline int64_t node_eval_adj(const double *x, int n, const MeshTab &tb,
                                        const RowShift &rs, double len, double xe,
                                        int kx, WT *w, int &cc, double &xh_out)
{
    const NodePos np = node_pos(xe, rs, x[0], x[n], tb.scal[0], tb.scal[2], tb.nb);
    const double2 nx = tb.bnext[np.b];
    int c = cell_from_bucket(tb.bucket[np.b], nx, np.xt);
    if (np.xt >= nx.y) c = cell_walk(x, n, c, np.xt);
    rec_weights<WT, P>(RecT<WT>::get(tb)[c], np.xt, w);
    cc = c;
    xh_out = np.xt;
    return (int64_t)c + (rs.kf0 + np.dk + kx) * (int64_t)n;
}

// x-derivatives of the stencil weights at xh in cell c (the product rule
// carried through the prefix/suffix products), from the cell record of the
// state's type: FP64 for an FP64 state; for an FP32 state the FP32 record
// and arithmetic, so v0bar, which sums differences of the reconstruction
// between neighbouring nodes, carries about 1e-4 relative rounding there.
template <typename WT, int P>
__device__ inline void node_dweights(const MeshTab &tb, int c, double xh, double *dw)
{
    const CellRec<WT> &r = RecT<WT>::get(tb)[c];
    const WT th = (WT)((xh - r.xc) * r.dxinv);
    WT t[P + 1], pre[P + 1], suf[P + 1], dpre[P + 1], dsuf[P + 1];
#pragma unroll
    for (int a = 0; a <= P; ++a) t[a] = th - r.th[a];
    pre[0] = (WT)1;
    dpre[0] = (WT)0;
#pragma unroll
    for (int a = 1; a <= P; ++a) {
        pre[a] = pre[a - 1] * t[a - 1];
        dpre[a] = dpre[a - 1] * t[a - 1] + pre[a - 1];
    }
    suf[P] = (WT)1;
    dsuf[P] = (WT)0;
#pragma unroll
    for (int a = P - 1; a >= 0; --a) {
        suf[a] = suf[a + 1] * t[a + 1];
        dsuf[a] = dsuf[a + 1] * t[a + 1] + suf[a + 1];
    }
#pragma unroll
    for (int a = 0; a <= P; ++a)
        dw[a] = (double)(r.rd[a] * (dpre[a] * suf[a] + pre[a] * dsuf[a])) * r.dxinv;
}

// The reconstruction q~ at a shifted node from global memory (direct path).
template <typename TQ, int P>
__device__ __attribute__((noinline)) double direct_qtilde(
    const double *x, const TQ *q, int n, const double *dw, int c)
{
    constexpr int LO = (P - 1) / 2;
    double dq = 0.0;
    for (int b = 0; b <= P; ++b) {
        const int j = c - LO + b;
        double d = 0.0;
        if (j > c) {
            for (int m = c; m < j; ++m) d += cell_mass(x, q, n, m);
        } else if (j < c) {
            for (int m = j; m < c; ++m) d += cell_mass(x, q, n, m);
            d = -d;
        }
        dq += dw[b] * d;
    }
    return dq;
}

} // namespace dev
} // namespace ram
