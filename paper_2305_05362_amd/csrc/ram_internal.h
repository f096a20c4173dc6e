// ram_internal.h -- private declarations shared by the host API and the HIP
// kernels of the RAM library (not installed, not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ram {

// Destination cells per workgroup tile, threads per workgroup, and the
// capacity (in source cells) of the LDS window that holds a tile's sources.
constexpr int kTile = 256;
constexpr int kBlock = 256;
constexpr int kWindowCap = 2048;
// Cells per tile of the residual step alone: four per thread, with the
// two-cell halo a side staged in one item per thread.
constexpr int kResTile = 1020;
// int32 entries per tile of the window plan
constexpr int kPlanW = 3;
// Cells per tile of the one-node-per-thread adjoint kernels (the limited
// shift's, the per-row shift's and the residual's): a tile's nodes (tile + 1)
// and its window or halo (tile + up to 5) take one pass of kBlock threads,
// so no thread runs a second node's chain while the others wait.
constexpr int kAdjTile = kBlock - 5;
// Centre value <-> cell average conversion: four cells per thread.
constexpr int kAvgItems = 4;
constexpr int kAvgTile = kBlock * kAvgItems;

// How cumulative differences are formed: from a window prefix sum in FP64,
// compensated FP32 or plain FP32, or (kSumDirect) summed directly from the
// masses between the two nodes, with no prefix at all.
enum ScanMode { kScanF64 = 0, kScanTwoSum = 1, kScanF32 = 2, kSumDirect = 3 };

// Limited reconstructions of the bulk shift (Section 3.1): PLM with the van
// Leer slope, PPM with the interface values and constraints of App. A.
enum Recon { kReconPLM = 1, kReconPPM = 2 };

// Mesh-only tables for a mesh shared by every row (built once per call by
// launch_mesh_prep): cell sizes and their reciprocals, reciprocal centre gaps
// for the slopes, reciprocal Lagrange denominators of every source cell's
// stencil, and a uniform bucket index over [x0, xN) that turns the cell
// search into one lookup plus a short walk.
struct MeshTab {
    const double *dx = nullptr;
    const double *dxinv = nullptr;
    const double *hinv = nullptr;     // 1 / (centre_{j+1} - centre_j), periodic
    const double *stc = nullptr;      // [n][2(order+1)]: stencil data, below
    const float *dxf = nullptr;
    const float *dxinvf = nullptr;
    const float *hinvf = nullptr;
    const float *stcf = nullptr;
    const int32_t *bucket = nullptr;  // largest j with x_j <= x0 + b L / nb
    const double2 *bnext = nullptr;   // per bucket: the next two nodes (or +inf)
    int32_t nb = 0;
    const double *scal = nullptr;     // device scalars: nb / L, 1 / L, x0 nb / L
    const float2 *rrf = nullptr;      // per cell: (dx, 1/centre gap), FP32
    // FP32 stencil data of each source cell in planes (float4 [n], float4 [n],
    // float [n] back to back): the offsets th_b other than the cell's own edges
    // (0 and 1), then the reciprocal denominators rd_b other than the own
    // node's, in that order (nine values at order 5); planes, so that the
    // records of neighbouring cells are neighbours in memory
    const float *stp = nullptr;
    const double2 *rrd = nullptr;     // per cell: (dx, 1/centre gap), FP64
    // FP64 per cell, six planes of n pairs: (x_c, 1/dx_c), then stp's values
    // in FP64 two at a time (the last pair padded with 0)
    const double2 *stpd = nullptr;
    // the same offsets and denominators as FP32 deviations from those of
    // equally spaced nodes (planes as stp): th_b - (b - lo), rd_b / rd_eq_b - 1;
    // on a uniform run they are below about 1e-9, so their FP32 rounding is
    // far below FP64 rounding of the values they restore
    const float *stdv = nullptr;
    const void *crf = nullptr;        // CellRec<float>[n]
    const void *crd = nullptr;        // CellRec<double>[n]
    // PPM interface weights (d1, d2, e1, e2, e3 of every cell; five arrays of
    // n back to back), FP64 and FP32
    const double *ppmd = nullptr;
    const float *ppmf = nullptr;
    // prefix counts (n + 1) of the cells whose size differs from the mesh's
    // largest (nonu) or smallest (nonu_min) by more than kUniformTol of it: a
    // range with no such cell is uniformly spaced (a refined-zone mesh has a
    // coarse and a fine uniform run)
    const int32_t *nonu = nullptr;
    const int32_t *nonu_min = nullptr;
};

// Relative spacing tolerance of a uniform run (a tile's shifted nodes then
// share one stencil offset and one theta to within FP32 rounding).
constexpr double kUniformTol = 1e-10;

// Everything the bulk shift needs about source cell c in one record (one
// cache line in FP32, two in FP64): x_c, 1/dx_c, and the stencil data
// (offsets and reciprocal denominators, as in MeshTab::stc) in type T.
template <typename T> struct CellRec {
    double xc;
    double dxinv;
    T th[6];
    T rd[6];
};
static_assert(sizeof(CellRec<float>) == 64, "one cache line");
static_assert(sizeof(CellRec<double>) == 112, "FP64 record");
// Stencil data of source cell c (order p, lo = (p-1)/2), in units of dx_c:
//   stc[c][a]       = (x_{c-lo+a} - x_c) / dx_c                   a = 0..p
//   stc[c][p+1+a]   = 1 / prod_{b != a} (stc[c][a] - stc[c][b])
// so the Lagrange weight of node a at theta = (xh - x_c)/dx_c is
//   stc[c][p+1+a] * prod_{b != a} (theta - stc[c][b]).

// Where the rows are.  Uniform batches (n_cols > 0) map tile t to
// (row = t / tiles_per_row, start = (t % tiles_per_row) * kTile); ragged
// batches read the tile's row from tile_row (built by launch_tiles_prep).
struct Rows {
    int64_t n_rows = 0;
    int64_t n_cols = 0;               // > 0 uniform rows, 0 ragged
    const int64_t *row_ptr = nullptr; // ragged: n_rows+1 cell offsets
    const int64_t *tile_ptr = nullptr;// ragged: n_rows+1 first tile per row
    const int32_t *tile_row = nullptr;// ragged: row of each tile
    int64_t n_tiles = 0;              // grid size (upper bound when ragged)
    int tile = kTile;                 // cells per tile (kernel-specific)
    const double *edges = nullptr;
    int shared = 1;                   // one node array for every row
    MeshTab tab;                      // shared mesh: its tables
    int has_tab = 0;                  // tab is filled in
};

// Mesh-density index of a shared mesh (Section 3.2.1): the nodes satisfy
// F(x_j) = j with F(x) = N (P(x) - P(x_min)) / I, P the antiderivative of the
// density psi with P(0) = 0 and I its integral over the period, so the source
// cell of a shifted node is floor(F(x)) (checked against the nodes).  kind 1:
// the periodic bump of App. B, psi = 1 + c on |s| <= a, 1 + c cos^2(pi/2
// (|s| - a)/(b - a)) on a < |s| < b, 1 beyond.
struct MeshDensity {
    int64_t kind = 0;          // 0 none (bucket index), 1 periodic bump (8 bytes: no padding in StepArgs)
    double a = 0.0, b = 0.0, c = 0.0;
    double w_pi = 0.0;         // pi / (b - a)
    double ramp_amp = 0.0;     // c (b - a) / (2 pi)
    double ramp_end = 0.0;     // P(b) = (1 + c) a + (1 + c / 2) (b - a)
    double scale = 0.0;        // N / I
    double p0 = 0.0;           // P(x_min)
};

// P(t) of the periodic bump: odd, linear with slope 1 + c inside a, the
// cos^2 ramp's integral between a and b, slope 1 beyond b.
__host__ __device__ inline double bump_prim(double t, const MeshDensity &d)
{
    const double at = fabs(t);
    double v;
    if (at <= d.a) v = (1.0 + d.c) * at;
    else if (at < d.b) v = (1.0 + d.c) * d.a + (1.0 + 0.5 * d.c) * (at - d.a) +
                           d.ramp_amp * sin(d.w_pi * (at - d.a));
    else v = d.ramp_end + (at - d.b);
    return copysign(v, t);
}

// The FP32 step on a shared mesh with direct sums (k_step_fast): tiles of
// kFastTile destination cells, one a wave (four consecutive cells a lane),
// each with a source window of at most kFastWin cells in LDS.  One record per
// tile, planned once per call (k_plan_fast), read with scalar loads.
constexpr int kFastTile = 256;
constexpr int kFastWin = 768;
// Rows of the streaming kernels hold fewer cells than this (64 Mi): their
// per-lane byte offsets into a row or a mesh table (16 bytes a cell at most)
// fit 32 bits.  Longer rows take the general kernels.
constexpr int64_t kFastMaxCols = int64_t(1) << 26;
enum FastKind { kFastWindow = 0, kFastUniform = 1, kFastDirect = 2 };
struct FastTile {
    int32_t kind;            // FastKind
    int32_t w;               // window length, cells
    int32_t base;            // window start mod n
    int32_t wlo_lo, wlo_hi;  // extended source index of the window start
    float cc[6];             // uniform: weights of the (order+1)-point stencil
    float dx, hinv, dxinv;   // uniform: the run's cell size, 1/centre gap, 1/size
    int32_t pad[2];          // tile id; the k-th other tile: k (its node data),
                             // a uniform tile: the bits of its FP32 theta
};
static_assert(sizeof(FastTile) == 64, "one record a tile");
// The tiles of one call: their records (rec[0 .. n_tiles)), then the same
// records compacted (rec[n_tiles ..)): the uniform tiles in tile order
// (totals[0] of them), then the others in tile order, each with its tile id in
// pad[0]; the per-1024-tile counts the compacted order is built from; and for
// the k-th non-uniform tile, the source-window index (jc) and position in its
// cell (theta, FP32) of each of its shifted nodes, kFastNodes entries a tile
// (the shift of a row is the same at every step of a call).
constexpr int kFastNodes = kFastTile + 8;
struct FastPlan {
    FastTile *rec = nullptr;
    int32_t *counts = nullptr;
    int32_t *totals = nullptr;
    float *theta = nullptr;
    int16_t *jc = nullptr;
};
// Device bytes of the plan of n_tiles tiles (each piece 256-byte aligned).
inline size_t fast_plan_bytes(int64_t n_tiles)
{
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t nn = (size_t)n_tiles * kFastNodes;
    return al(2 * sizeof(FastTile) * (size_t)n_tiles) +
           al(sizeof(int32_t) * (size_t)((n_tiles + 1023) / 1024)) + al(2 * sizeof(int32_t)) +
           al(sizeof(float) * nn) + al(sizeof(int16_t) * nn);
}
inline FastPlan fast_plan_at(void *mem, int64_t n_tiles)
{
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t nn = (size_t)n_tiles * kFastNodes;
    char *p = (char *)mem;
    FastPlan f;
    f.rec = (FastTile *)p;
    p += al(2 * sizeof(FastTile) * (size_t)n_tiles);
    f.counts = (int32_t *)p;
    p += al(sizeof(int32_t) * (size_t)((n_tiles + 1023) / 1024));
    f.totals = (int32_t *)p;
    p += al(2 * sizeof(int32_t));
    f.theta = (float *)p;
    p += al(sizeof(float) * nn);
    f.jc = (int16_t *)p;
    return f;
}

// Bulk shift, optionally fused with the residual step (dv != null).
// Streaming shift on per-row meshes (FP32 state, no residual): tiles of
// kRagTile cells of one row, one a wave.  The shift is fixed for a call, so
// each shifted node's source cell and Lagrange weights are too: planned once
// per call into a record per tile, per node slot (kFastNodes a tile; the
// slots past the tile's last node repeat it) the weights other than the own
// node's (four in wa, the fifth in wb) and the source cell's index in the
// tile's window, and the row cells' FP32 sizes.
struct RagTile {
    int32_t kind;        // kFastWindow, or kFastDirect (window beyond the LDS)
    int32_t row, i0, nd; // row, first cell, cells
    int32_t n, w, base;  // row length, window length, window start mod n
    int32_t pad0;
    int64_t qoff, eoff;  // the row's first cell and first node
    int64_t wlo;         // the window start as an extended source index
    int32_t pad[2];
};
static_assert(sizeof(RagTile) == 64, "one record a cache line half");
// Cells of a per-row streaming tile: 255, so that its 256 shifted nodes fill
// four slots of a wave (no residual halo on this path).
constexpr int kRagTile = 255;
struct RagPlan {
    RagTile *rec = nullptr;
    float4 *wa = nullptr;
    float *wb = nullptr;
    int16_t *jc = nullptr;
    float *dx = nullptr;       // FP32 sizes of the row cells, [n_cells]
};
inline size_t rag_plan_bytes(int64_t n_tiles, int64_t n_cells)
{
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t nn = (size_t)n_tiles * kFastNodes;
    return al(sizeof(RagTile) * (size_t)n_tiles) + al(sizeof(float4) * nn) +
           al(sizeof(float) * nn) + al(sizeof(int16_t) * nn) + al(sizeof(float) * (size_t)n_cells);
}
inline RagPlan rag_plan_at(void *mem, int64_t n_tiles)
{
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t nn = (size_t)n_tiles * kFastNodes;
    char *p = (char *)mem;
    RagPlan r;
    r.rec = (RagTile *)p;
    p += al(sizeof(RagTile) * (size_t)n_tiles);
    r.wa = (float4 *)p;
    p += al(sizeof(float4) * nn);
    r.wb = (float *)p;
    p += al(sizeof(float) * nn);
    r.jc = (int16_t *)p;
    p += al(sizeof(int16_t) * nn);
    r.dx = (float *)p;
    return r;
}

struct StepArgs {
    Rows rows;
    const void *q_in = nullptr;
    void *q_out = nullptr;
    const double *v0 = nullptr;
    const void *dv = nullptr;         // null: shift only
    double dt = 0.0;
    const int64_t *plan_wlo = nullptr;  // shared mesh: per-tile window start
    const int32_t *plan_w = nullptr;    // ... length (-1: direct path), then
                                        // [n_tiles + tile]: start mod n
    void *q_mid = nullptr;              // optional: the state after the shift
    MeshDensity dens;                   // shared mesh, direct sums: closed-form index
    FastPlan fast;                      // FP32 streaming kernels: their tile plan (rec set)
    RagPlan rag;                        // per-row meshes, FP32 streaming shift (rec set)
};

// Radial transport of a polar grid (rows = radii): q [n_rows][n_cols], u on
// the radial faces [n_rows + 1][n_cols], radial edges r_edges[n_rows + 1].
struct RadialArgs {
    int64_t n_rows = 0;
    int64_t n_cols = 0;
    const double *r_edges = nullptr;
    const void *q_in = nullptr;
    void *q_out = nullptr;
    const void *u = nullptr;
    double dt = 0.0;
};

struct ResidualArgs {
    Rows rows;
    const void *q_in = nullptr;
    void *q_out = nullptr;
    const void *dv = nullptr;
    double dt = 0.0;
};

struct ShiftAdjArgs {
    Rows rows;
    const void *q_fwd = nullptr;      // forward input (for v0bar), may be null
    const void *qbar_out = nullptr;
    void *qbar_in = nullptr;
    const double *v0 = nullptr;
    double dt = 0.0;
    double *v0bar = nullptr;          // per-row accumulator or null
    double *v0part = nullptr;         // [n_tiles] each tile's v0bar term (v0bar set)
    void *edge = nullptr;             // [n_tiles][2 p] (state's type) each tile's terms for
                                      // its window's first and last p cells
    int64_t *wstart = nullptr;        // [n_tiles] each tile's window start (extended index)
};

// One step backwards on a shared mesh (fused residual adjoint, then shift
// adjoint).  dv == null: the step had no residual, qbar_out is the shift's.
struct StepAdjArgs {
    Rows rows;                          // tile = step_tile(true), tables set
    const void *q_fwd = nullptr;        // state before the shift (v0bar)
    const void *q_half = nullptr;       // state the residual read
    const void *dv = nullptr;
    const void *qbar_out = nullptr;
    void *qbar_in = nullptr;
    void *dvbar = nullptr;              // accumulator or null
    double *v0bar = nullptr;            // accumulator or null
    double *v0part = nullptr;           // [n_tiles] each tile's v0bar term (v0bar set)
    const double *v0 = nullptr;
    double dt = 0.0;
    const int64_t *plan_wlo = nullptr;  // window plan of the shift (no halo)
    const int32_t *plan_w = nullptr;    // [n_tiles] lengths, [n_tiles] starts mod n
    FastPlan fast;                      // streaming adjoint: the shift's tile plan (no halo)
    void *edge = nullptr;               // [n_tiles][2 p] each tile's terms for its window's
                                        // first and last p cells (FP32 on the streaming
                                        // kernels, the state's type on the general one)
};

struct ResidualAdjArgs {
    Rows rows;
    const void *q_fwd = nullptr;
    const void *dv = nullptr;
    const void *qbar_out = nullptr;
    void *qbar_in = nullptr;
    void *dvbar = nullptr;            // accumulator or null
    double dt = 0.0;
};

// Number of tiles a ragged batch can need at most (grid size).
inline int64_t ragged_tile_bound(int64_t n_cells, int64_t n_rows, int tile)
{
    return n_cells / tile + n_rows + 1;
}

// Shifted nodes per thread in the bulk-shift kernel, and its destination
// cells per tile: kBlock*kItems nodes bound kBlock*kItems-1 cells, less a
// two-cell halo per side when the residual step is fused in.
constexpr int kItems = 4;
constexpr int kStepNodes = kBlock * kItems;
inline int step_tile(bool fused) { return kStepNodes - 1 - (fused ? 4 : 0); }
// The shared-mesh kernel with direct sums also comes with 2, 3 and 5 nodes
// per thread (a schedule the caller or the autotuner chooses).
inline bool valid_items(int items) { return items >= 2 && items <= 5; }
inline int step_tile_for(int items, bool fused) { return kBlock * items - 1 - (fused ? 4 : 0); }

// The static device scratch of ram_shift_noalloc (ram_noalloc.hip): its size,
// the once-per-device lookup of its address (with the device current; call
// from ram_create), and that address (null until the lookup succeeded).
constexpr size_t kNoAllocBytes = size_t(16) << 20;
hipError_t noalloc_setup(int device);
void *noalloc_scratch(int device);

hipError_t launch_tiles_prep(const int64_t *row_ptr, int64_t n_rows, int tile,
                             int64_t *tile_ptr, int32_t *tile_row,
                             hipStream_t stream);
// Bytes of scratch the shared-mesh tables of an n-cell mesh need.
size_t mesh_tab_bytes(int64_t n, int order);
// Build the tables in `mem` (mesh_tab_bytes) and point `tab` at them.
hipError_t launch_mesh_prep(const double *x, int64_t n, int order, void *mem,
                            MeshTab &tab, hipStream_t stream, bool uniform = false);
hipError_t launch_step(const StepArgs &a, bool f64, int scan, int order,
                       hipStream_t stream);
// Shared-mesh specialisation: plan the tiles' source windows once per call
// (launch_plan, into n_tiles int64 + kPlanW n_tiles int32), then one launch per step.
// The int32 part holds per tile its window length (-1: direct path), the
// window start mod n, and, for a tile whose nodes and source window lie in
// one uniform run, the float bits of its first node's theta (else -1.0f).
hipError_t launch_plan(const StepArgs &a, int order, int64_t *wlo, int32_t *w,
                       hipStream_t stream);
hipError_t launch_step_shared(const StepArgs &a, bool f64, int scan, int order,
                              int items, hipStream_t stream);
// The FP32 direct-sum step on a shared mesh: plan the tiles into `plan`
// (R.tile == kFastTile, tables with the uniform-run counts; records, then the
// two tile lists), then per step the uniform-tile and the searching-tile
// kernels (a.fast set).
hipError_t launch_plan_fast(const StepArgs &a, int order, const FastPlan &plan,
                            hipStream_t stream);
hipError_t launch_step_fast(const StepArgs &a, int order, int scan, hipStream_t stream);
// A second stream and two events of a context: while a step loop is being
// captured into a graph (the calling thread's capture_fork points at them),
// the FP32 streaming step forks its searching tiles' kernel onto the side
// stream and joins it back, so that the graph holds the two kernels as
// parallel branches.  Outside a capture the kernels run one after the other.
struct ForkJoin {
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
extern thread_local const ForkJoin *capture_fork;
// The same plan's limited FP32 step (PLM / PPM: k_step_uni_lim, k_step_gen_lim).
hipError_t launch_step_fast_lim(const StepArgs &a, int recon, hipStream_t stream);
// The same plan's FP64 step (k_step64, ram_step_fast64.hip): scan kScanF64 or kSumDirect.
hipError_t launch_step_fast64(const StepArgs &a, int order, int scan, hipStream_t stream);
// Per-row meshes, FP32, shift only: the per-call plan into `plan` (R.tile ==
// kRagTile, a.dv null), then per step the streaming shift (a.rag set).
hipError_t launch_plan_rag(const StepArgs &a, int order, const RagPlan &plan,
                           hipStream_t stream);
hipError_t launch_step_rag(const StepArgs &a, int order, int scan, hipStream_t stream);
hipError_t launch_residual(const ResidualArgs &a, bool f64,
                           hipStream_t stream);
hipError_t launch_shift_adjoint(const ShiftAdjArgs &a, bool f64, int order,
                                hipStream_t stream);
hipError_t launch_residual_adjoint(const ResidualAdjArgs &a, bool f64,
                                   hipStream_t stream);
// v0bar[row] += the row's per-tile terms part[tile], summed in tile order (the
// adjoint kernels write one term per tile instead of adding atomically, so
// that v0bar does not depend on the order the tiles finish in).
hipError_t launch_v0_reduce(const Rows &R, const double *part, double *v0bar,
                            hipStream_t stream);
// The window cells neighbouring tiles share (the first p of each tile's
// window), each the sum in a fixed order of the terms the tiles holding it
// stored in `edge` (tile k's window starts at wstart[k]; [n_tiles][2 p]
// values of the state's type, head then tail).
hipError_t launch_edge_sum(const Rows &R, const int64_t *wstart, const void *edge, void *qbar,
                           bool f64, int p, hipStream_t stream);
// Bytes of those buffers for n_tiles tiles.
inline size_t adj_edge_bytes(int64_t n_tiles, int p, size_t elem)
{
    return 2 * (size_t)p * elem * (size_t)n_tiles;
}
// Zero the cells several tiles accumulate into, then the fused adjoint.
hipError_t launch_step_adjoint_shared(const StepAdjArgs &a, bool f64, int order,
                                      hipStream_t stream);
// The same step backwards for an FP32 state on rows of a multiple of four
// cells (16-byte aligned states), one tile of kFastTile cells a wave, on the
// shift's tile plan without halo (a.fast, from launch_plan_fast): the
// uniform-run tiles, the other tiles, the sums of the window cells that
// neighbouring tiles share (a.edge), the v0bar sums.
hipError_t launch_step_adjoint_fast(const StepAdjArgs &a, int order, hipStream_t stream);
// The limited (PLM / PPM) step backwards on the same tiles (plan of order
// 2 lo + 1, a.q_fwd the state the shift read; a.dv null: the shift alone).
hipError_t launch_step_limited_adjoint_fast(const StepAdjArgs &a, int recon,
                                            hipStream_t stream);
hipError_t launch_copy(const void *src, void *dst, int64_t bytes,
                       hipStream_t stream);
// Bulk shift with a limited reconstruction (recon: Recon) on any layout; a.dv
// is ignored.
hipError_t launch_shift_limited(const StepArgs &a, bool f64, int recon,
                                hipStream_t stream);
// Transpose of the limited shift's Jacobian at a.q_fwd (any layout; a zeroing
// pass, then one gather kernel), v0bar accumulated when a.v0bar is set.
hipError_t launch_shift_limited_adjoint(const ShiftAdjArgs &a, bool f64, int recon,
                                        hipStream_t stream);
// floor(F(x)) of the mesh-density index for m points (clamped to [0, n-1]),
// without the check against the nodes (a test of the closed form).
hipError_t launch_density_cells(const MeshDensity &d, int n, const double *x, int64_t m,
                                int32_t *cells, hipStream_t stream);
hipError_t launch_radial(const RadialArgs &a, bool f64, hipStream_t stream);
// Centre values -> cell averages (inverse: back) with the fourth-order
// correction, every row of R (R.tile == kAvgTile); in and out must not alias.
// w: the (w+, w-) weights of a shared mesh from launch_average4_weights, in
// the state's type, or null (formed from the nodes in the kernel).
hipError_t launch_average4_weights(const double *x, int64_t n, bool f64, void *w,
                                   hipStream_t stream);
hipError_t launch_average4(const Rows &R, bool f64, bool inverse, const void *in, void *out,
                           const void *w, hipStream_t stream);
// The inverse conversion, then the forward one, in one pass (between two
// steps on centre values).
hipError_t launch_average4_between(const Rows &R, bool f64, const void *in, void *out,
                                   const void *w, hipStream_t stream);
// Per-row mass, dx-weighted L1 distance to qref (if non-null) and max |Q|,
// three FP64 values per row (one workgroup per row).
hipError_t launch_row_norms(const Rows &R, bool f64, const void *q, const void *qref,
                            double *out, hipStream_t stream);
// Shared meshes: the limited shift in the specialised step kernel, fused with
// the residual when a.dv is set; needs the window plan of order 3 (PLM) or 5
// (PPM) and the tables.
hipError_t launch_step_shared_limited(const StepArgs &a, bool f64, int recon,
                                      hipStream_t stream);

} // namespace ram
