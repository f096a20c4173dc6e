// ram_api.cpp -- C ABI of the RAM library (declared in include/ram.h): argument
// checks, context and scratch management, dispatch to the HIP kernels.
#include "ram.h"
#include "ram_internal.h"
#include "ram_stream.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <initializer_list>
#include <vector>

// set while a step loop is captured (ram_internal.h)
namespace ram {
thread_local const ForkJoin *capture_fork = nullptr;
}

struct ram_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // marks the end of the old stream's work when the context moves to
    // another stream (ram_set_stream): the new one waits for it
    hipEvent_t handoff = nullptr;
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    // multi-step loops are captured once into a graph and replayed while the
    // arguments stay the same (capture needs a stream of its own: the
    // caller's may be the null stream)
    hipStream_t cap_stream = nullptr;
    ram::ForkJoin fork;                 // parallel branches inside a captured step
    struct Graph {
        std::vector<unsigned char> key;
        hipGraphExec_t exec = nullptr;
    };
    std::vector<Graph> graphs;          // most recently used first
    // schedule of the shared-mesh step kernel with direct sums: shifted
    // nodes per thread (ram_set_schedule)
    int items = 0;                      // 0: the default (streaming kernel)
    // mesh-density description of the shared mesh (ram_set_mesh_density)
    ram_mesh_density density{};
};

namespace {

thread_local std::string g_last_error;

ram_status fail(ram_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

ram_status hip_fail(hipError_t e, const char *what)
{
    return fail(RAM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Select the context's device for the calling thread.  Every entry point
// checks its arguments first (host logic only), then enters the context.
ram_status enter(ram_ctx *ctx)
{
    if (!ctx) return fail(RAM_E_INVALID_ARG, "null context");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return RAM_OK;
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// The HIP side of ram::switch_stream.
struct HipStreams {
    using stream_t = hipStream_t;
    using event_t = hipEvent_t;
    hipError_t err = hipSuccess;
    bool capturing(hipStream_t s)
    {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
            (void)hipGetLastError();     // leave no stale error for the caller's checks
            return true;
        }
        return cs != hipStreamCaptureStatusNone;
    }
    int record(hipEvent_t ev, hipStream_t s)
    {
        err = hipEventRecord(ev, s);
        return err != hipSuccess;
    }
    int wait(hipStream_t s, hipEvent_t ev)
    {
        err = hipStreamWaitEvent(s, ev, 0);
        return err != hipSuccess;
    }
};

// Step loops of at least this many launches are captured into a graph; the
// context keeps the most recent few.
constexpr int64_t kGraphMinSteps = 4;
constexpr size_t kGraphCache = 4;

ram_status ensure_scratch(ram_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->scratch_bytes) return RAM_OK;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
    for (auto &g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);   // stream is idle
    ctx->graphs.clear();
    size_t want = align_up(bytes + bytes / 8);
    e = hipMalloc(&ctx->scratch, want);
    if (e != hipSuccess) {
        ctx->scratch = nullptr;
        return fail(RAM_E_NOMEM, "hipMalloc(%zu) for scratch: %s", want,
                    hipGetErrorString(e));
    }
    ctx->scratch_bytes = want;
    return RAM_OK;
}

size_t elem_size(ram_dtype dt) { return dt == RAM_F64 ? 8 : 4; }

int64_t layout_cells(const ram_layout *L)
{
    return L->n_cols > 0 ? L->n_rows * L->n_cols : L->n_cells;
}

ram_status check_layout(const ram_layout *L, const double *edges)
{
    if (!L) return fail(RAM_E_INVALID_ARG, "null layout");
    if (L->n_rows < 1) return fail(RAM_E_INVALID_ARG, "n_rows must be >= 1");
    if (L->n_cols < 0) return fail(RAM_E_INVALID_ARG, "n_cols must be >= 0");
    if (!edges) return fail(RAM_E_INVALID_ARG, "null edges");
    if (L->n_cols == 0) {
        if (!L->row_ptr) return fail(RAM_E_INVALID_ARG, "ragged layout needs row_ptr");
        if (L->n_cells < 1) return fail(RAM_E_INVALID_ARG, "ragged layout needs n_cells >= 1");
        if (L->edges_shared)
            return fail(RAM_E_INVALID_ARG, "shared edges need uniform rows (n_cols > 0)");
    }
    if (L->n_cols > 0 && L->n_cols > INT32_MAX - 1)
        return fail(RAM_E_INVALID_ARG, "rows longer than 2^31-2 cells");
    return RAM_OK;
}

ram_status check_dtype(ram_dtype dt)
{
    if (dt != RAM_F64 && dt != RAM_F32)
        return fail(RAM_E_UNSUPPORTED, "dtype must be RAM_F64 or RAM_F32");
    return RAM_OK;
}

ram_status check_order(const ram_layout *L, int order)
{
    if (order != 1 && order != 3 && order != 5)
        return fail(RAM_E_UNSUPPORTED, "order must be 1, 3 or 5 (got %d)", order);
    if (L->n_cols > 0 && L->n_cols < order + 1)
        return fail(RAM_E_INVALID_ARG, "rows need at least order+1 = %d cells", order + 1);
    return RAM_OK;
}

ram_status check_scan(ram_dtype dt, ram_scan scan)
{
    if (scan != RAM_SCAN_F64 && scan != RAM_SCAN_F32_TWOSUM && scan != RAM_SCAN_F32 &&
        scan != RAM_SUM_DIRECT)
        return fail(RAM_E_UNSUPPORTED, "unknown scan precision %d", (int)scan);
    if (dt == RAM_F64 && scan != RAM_SCAN_F64 && scan != RAM_SUM_DIRECT)
        return fail(RAM_E_UNSUPPORTED, "FP64 state requires RAM_SCAN_F64 or RAM_SUM_DIRECT");
    return RAM_OK;
}

ram_status check_recon(const ram_layout *L, ram_recon recon)
{
    if (recon != RAM_RECON_PLM && recon != RAM_RECON_PPM)
        return fail(RAM_E_UNSUPPORTED, "recon must be RAM_RECON_PLM or RAM_RECON_PPM (got %d)",
                    (int)recon);
    const int need = recon == RAM_RECON_PLM ? 4 : 6;
    if (L->n_cols > 0 && L->n_cols < need)
        return fail(RAM_E_INVALID_ARG, "rows need at least %d cells", need);
    return RAM_OK;
}

ram_status check_dt(double dt)
{
    if (!std::isfinite(dt)) return fail(RAM_E_INVALID_ARG, "dt must be finite");
    return RAM_OK;
}

// Scratch plan of one call: the pieces are carved out of the context's single
// device buffer, 256-byte aligned.
struct Carve {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    }
};

size_t ragged_bytes(const ram_layout *L, int tile)
{
    if (L->n_cols > 0) return 0;
    return align_up(sizeof(int64_t) * (L->n_rows + 1)) +
           align_up(sizeof(int32_t) * ram::ragged_tile_bound(L->n_cells, L->n_rows, tile));
}

struct RowsPlan {
    size_t rag_off = 0, tab_off = 0;
    int tile = ram::kTile;
    int order = 0;          // > 0: build the shared-mesh tables for this order
    bool uniform = false;   // and the uniform-run counts (the FP32 direct step)
};

// The step kernels use a shared mesh's uniform runs on the FP32 direct-sum
// Lagrange path only.
bool wants_uniform(ram_dtype dtype, ram_scan scan)
{
    return dtype == RAM_F32 && scan == RAM_SUM_DIRECT;
}

// Reserve what make_rows will need.
RowsPlan plan_rows(Carve &cv, const ram_layout *L, int tile, int tab_order)
{
    RowsPlan p;
    p.tile = tile;
    if (L->n_cols == 0) p.rag_off = cv.take(ragged_bytes(L, tile));
    if (L->edges_shared && tab_order > 0) {
        p.order = tab_order;
        p.tab_off = cv.take(ram::mesh_tab_bytes(L->n_cols, tab_order));
    }
    return p;
}

// Fill the kernel-side row description (after ensure_scratch): ragged
// batches get their tile table, shared meshes their tables.
ram_status make_rows(ram_ctx *ctx, const ram_layout *L, const double *edges,
                     const RowsPlan &p, ram::Rows &R, char *base_mem = nullptr)
{
    char *mem = base_mem ? base_mem : (char *)ctx->scratch;
    R.n_rows = L->n_rows;
    R.n_cols = L->n_cols;
    R.edges = edges;
    R.shared = L->edges_shared ? 1 : 0;
    R.tile = p.tile;
    if (L->n_cols > 0) {
        R.n_tiles = L->n_rows * ((L->n_cols + p.tile - 1) / p.tile);
    } else {
        R.row_ptr = L->row_ptr;
        R.n_tiles = ram::ragged_tile_bound(L->n_cells, L->n_rows, p.tile);
        char *base = mem + p.rag_off;
        R.tile_ptr = (const int64_t *)base;
        R.tile_row = (const int32_t *)(base + align_up(sizeof(int64_t) * (L->n_rows + 1)));
        hipError_t e = ram::launch_tiles_prep(L->row_ptr, L->n_rows, p.tile,
                                              (int64_t *)R.tile_ptr,
                                              (int32_t *)R.tile_row, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "tile table launch");
    }
    if (p.order > 0) {
        hipError_t e = ram::launch_mesh_prep(edges, L->n_cols, p.order, mem + p.tab_off,
                                             R.tab, ctx->stream, p.uniform);
        if (e != hipSuccess) return hip_fail(e, "mesh table launch");
        R.has_tab = 1;
    }
    return RAM_OK;
}

// Shifted nodes per thread the step kernel runs with: the context's schedule
// for a shared mesh with direct sums, else the default.
int sched_items(const ram_ctx *ctx, const ram_layout *L, ram_scan scan)
{
    const bool shared = L->edges_shared && L->n_cols > 0;
    return (shared && scan == RAM_SUM_DIRECT && ctx->items != 0) ? ctx->items : ram::kItems;
}

// The Lagrange step on a shared mesh at the default schedule and the bucket
// index runs the streaming kernels on tiles of kFastTile cells a wave: FP32
// k_step_uni / k_step_gen (every cumulative mode), FP64 k_step64; every other
// combination the general shared-mesh kernel.
bool use_fast_shape(const ram_ctx *ctx, bool shared, int64_t n_cols, ram_dtype dtype,
                    ram_scan scan)
{
    return shared && n_cols > 0 && n_cols < ram::kFastMaxCols && (dtype == RAM_F32 || dtype == RAM_F64) &&
           ctx->items == 0 && ctx->density.kind == RAM_DENSITY_NONE;
}
bool use_fast(const ram_ctx *ctx, const ram_layout *L, ram_dtype dtype, ram_scan scan)
{
    return use_fast_shape(ctx, L->edges_shared != 0, L->n_cols, dtype, scan);
}
// The limited (PLM / PPM) FP32 step on a shared mesh at the default schedule
// runs on the same plan (k_step_uni_lim / k_step_gen_lim); FP64 and every
// other combination the general limited kernel.
bool use_fast_lim(const ram_ctx *ctx, const ram_layout *L, ram_dtype dtype)
{
    return dtype == RAM_F32 && use_fast_shape(ctx, L->edges_shared != 0, L->n_cols, dtype,
                                              RAM_SUM_DIRECT);
}

// The FP32 shift-only step on per-row meshes at the default schedule runs the
// streaming kernel (k_step_rag) when the call is long enough to pay for its
// per-call plan (every node's weights); shorter calls and every other
// combination the general per-row kernel.
constexpr int64_t kRagMinSteps = 4;
bool use_rag(const ram_ctx *ctx, const ram_layout *L, ram_dtype dtype, const void *dv,
             int64_t n_steps)
{
    return !L->edges_shared && dtype == RAM_F32 && !dv && ctx->items == 0 &&
           n_steps >= kRagMinSteps;
}

// The FP32 step adjoint on a shared mesh at the default schedule runs the
// streaming adjoint (k_adjf_uni / k_adjf_gen) on rows of a multiple of four
// cells, at least a tile and a halo long, with 16-byte aligned arrays; every
// other combination the general shared-mesh adjoint.
bool use_fast_adjoint(const ram_ctx *ctx, const ram_layout *L, ram_dtype dtype,
                      std::initializer_list<const void *> arrays)
{
    if (dtype != RAM_F32 || !use_fast_shape(ctx, L->edges_shared != 0, L->n_cols, dtype, RAM_SCAN_F64))
        return false;
    if (L->n_cols % 4 != 0 || L->n_cols < ram::kFastTile + 8) return false;
    for (const void *p : arrays)
        if (p && ((uintptr_t)p % 16) != 0) return false;
    return true;
}

// Tile size of the step kernel a call runs.
int step_tile_of(const ram_ctx *ctx, const ram_layout *L, ram_dtype dtype, ram_scan scan,
                 int items, bool fused)
{
    return use_fast(ctx, L, dtype, scan) ? ram::kFastTile : ram::step_tile_for(items, fused);
}

// Bytes of the per-tile plan (window plan, or the fast kernels' records and
// tile lists).
size_t plan_w_bytes(int64_t nt)
{
    return std::max(ram::kPlanW * sizeof(int32_t) * (size_t)nt, ram::fast_plan_bytes(nt));
}

// Plan the tiles of a shared-mesh step once per call: the fast kernels'
// records, tile lists and node data, or the general kernel's window plan.
hipError_t plan_shared(ram::StepArgs &a, int plan_order, bool fast, void *wlo_p, void *w_p,
                       hipStream_t st)
{
    if (fast) {
        a.fast = ram::fast_plan_at(w_p, a.rows.n_tiles);
        return ram::launch_plan_fast(a, plan_order, a.fast, st);
    }
    a.plan_wlo = (const int64_t *)wlo_p;
    a.plan_w = (const int32_t *)w_p;
    return ram::launch_plan(a, plan_order, (int64_t *)wlo_p, (int32_t *)w_p, st);
}

// The kernel-side mesh-density index for a shared mesh of n cells.
ram::MeshDensity make_density(const ram_mesh_density &d, int64_t n)
{
    ram::MeshDensity m;
    if (d.kind != RAM_DENSITY_PERIODIC_BUMP) return m;
    m.kind = 1;
    m.a = d.a;
    m.b = d.b;
    m.c = d.c;
    const double w = d.b - d.a;
    m.w_pi = M_PI / w;
    m.ramp_amp = d.c * w / (2.0 * M_PI);
    m.ramp_end = (1.0 + d.c) * d.a + (1.0 + 0.5 * d.c) * w;
    const double inorm = (d.xmax - d.xmin) + d.c * (d.a + d.b);
    m.scale = (double)n / inorm;
    m.p0 = ram::bump_prim(d.xmin, m);
    return m;
}

int64_t tiles_of(const ram_layout *L, int tile)
{
    if (L->n_cols > 0) return L->n_rows * ((L->n_cols + tile - 1) / tile);
    return ram::ragged_tile_bound(L->n_cells, L->n_rows, tile);
}

// Run loop(stream) on the context's stream: directly for short loops, else
// through a graph captured once per distinct key (every argument the loop's
// launches depend on, as raw bytes) and replayed afterwards.
template <typename F>
ram_status run_graphed(ram_ctx *ctx, std::vector<unsigned char> key, int64_t n_steps,
                       F &&loop)
{
    hipError_t e;
    if (n_steps < kGraphMinSteps) {
        e = loop(ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "step launch");
        return RAM_OK;
    }
    size_t hit = ctx->graphs.size();
    for (size_t i = 0; i < ctx->graphs.size(); ++i)
        if (ctx->graphs[i].key == key) { hit = i; break; }
    if (hit < ctx->graphs.size()) {
        std::rotate(ctx->graphs.begin(), ctx->graphs.begin() + hit,
                    ctx->graphs.begin() + hit + 1);
    } else {
        if (ctx->graphs.size() >= kGraphCache) {
            e = hipStreamSynchronize(ctx->stream);          // the evicted one is done
            if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            (void)hipGraphExecDestroy(ctx->graphs.back().exec);
            ctx->graphs.pop_back();
        }
        if (!ctx->cap_stream) {
            e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
        }
        if (!ctx->fork.side) {
            e = hipStreamCreateWithFlags(&ctx->fork.side, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->fork.fork, hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->fork.join, hipEventDisableTiming);
            if (e != hipSuccess) return hip_fail(e, "fork stream / events");
        }
        e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        ram::capture_fork = &ctx->fork;
        const hipError_t le = loop(ctx->cap_stream);
        ram::capture_fork = nullptr;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(ctx->cap_stream, &g);
        if (le != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(le != hipSuccess ? le : e, "step loop capture");
        }
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
        ram_ctx::Graph entry;
        entry.key = std::move(key);
        entry.exec = x;
        ctx->graphs.insert(ctx->graphs.begin(), std::move(entry));
    }
    e = hipGraphLaunch(ctx->graphs.front().exec, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return RAM_OK;
}

// Raw bytes of the arguments a loop depends on (the graph cache's key).
template <typename... T>
std::vector<unsigned char> key_of(const T &...parts)
{
    std::vector<unsigned char> k;
    auto put = [&](const auto &p) {
        const unsigned char *b = (const unsigned char *)&p;
        k.insert(k.end(), b, b + sizeof(p));
    };
    (put(parts), ...);
    return k;
}

// n_steps launches of the bulk-shift kernel (fused with the residual when
// a.dv is set).  n_steps == 1 writes a.q_out; n_steps > 1 updates a.q_in in
// place, ping-ponging with `tmp`.  Shared meshes take the specialised kernel
// after planning the tiles' windows once; recon != 0 (shared meshes only)
// selects its limited-reconstruction mode, whose window halo is that of order
// 3 (PLM) or 5 (PPM).
ram_status launch_steps(ram_ctx *ctx, ram::StepArgs a, ram_dtype dtype,
                        ram_scan scan, int order, int64_t n_steps, void *tmp,
                        size_t wlo_off, size_t w_off, size_t state_bytes,
                        int items, int recon = 0, char *base_mem = nullptr,
                        bool allow_fast = true, int64_t rag_off = -1)
{
    char *mem = base_mem ? base_mem : (char *)ctx->scratch;
    const bool f64 = dtype == RAM_F64;
    const bool shared = a.rows.has_tab != 0 && a.rows.n_cols > 0;
    if (recon && !shared) return fail(RAM_E_UNSUPPORTED, "internal: limited step loop needs a shared mesh");
    if (shared && scan == RAM_SUM_DIRECT && recon == 0)
        a.dens = make_density(ctx->density, a.rows.n_cols);
    hipError_t e;
    if (shared) {
        const int plan_order = recon == 0 ? order : (recon == RAM_RECON_PLM ? 3 : 5);
        const bool fast = (recon == 0 || dtype == RAM_F32) && allow_fast &&
                          use_fast_shape(ctx, a.rows.shared != 0, a.rows.n_cols, dtype, scan);
        e = plan_shared(a, plan_order, fast, mem + wlo_off, mem + w_off, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "window plan launch");
    } else if (rag_off >= 0) {
        a.rag = ram::rag_plan_at(mem + rag_off, a.rows.n_tiles);
        e = ram::launch_plan_rag(a, order, a.rag, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "per-row plan launch");
    }
    auto one = [&](const ram::StepArgs &s, hipStream_t st) {
        if (recon) return ram::launch_step_shared_limited(s, f64, recon, st);
        return shared ? ram::launch_step_shared(s, f64, (int)scan, order, items, st)
                      : ram::launch_step(s, f64, (int)scan, order, st);
    };
    if (n_steps == 1 && a.q_out) {
        e = one(a, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "step launch");
        return RAM_OK;
    }
    // the ping-pong loop, on stream st
    auto loop = [&](hipStream_t st) -> hipError_t {
        ram::StepArgs b = a;
        void *q = const_cast<void *>(a.q_in);
        void *cur = q, *oth = tmp;
        for (int64_t k = 0; k < n_steps; ++k) {
            b.q_in = cur;
            b.q_out = oth;
            hipError_t r = one(b, st);
            if (r != hipSuccess) return r;
            void *t = cur; cur = oth; oth = t;
        }
        if (cur != q) return ram::launch_copy(cur, q, (int64_t)state_bytes, st);
        return hipSuccess;
    };
    const int64_t extra[4] = {(int64_t)dtype * 16 + (int64_t)scan + 256 * (int64_t)recon +
                                  4096 * (int64_t)items,
                              order, n_steps, (int64_t)(intptr_t)tmp ^ (int64_t)state_bytes};
    return run_graphed(ctx, key_of(a, extra), n_steps, loop);
}

// The streaming adjoint's per-call set-up: mesh tables, the shift's tile plan
// without halo (records, tile lists, node data), the v0bar and edge buffers;
// the per-step pointers (states, gradients) are left to the caller.
ram_status plan_adjoint_fast(ram_ctx *ctx, const ram_layout *layout, const double *edges,
                             const double *v0, double dt, int order, const void *dv,
                             void *dvbar, double *v0bar, ram::StepAdjArgs &a)
{
    ram_status st;
    Carve cv;
    RowsPlan rp = plan_rows(cv, layout, ram::kFastTile, order);
    rp.uniform = true;
    const int64_t nt = tiles_of(layout, rp.tile);
    const size_t rec_off = cv.take(ram::fast_plan_bytes(nt));
    const size_t v0_off = cv.take(v0bar ? sizeof(double) * nt : 0);
    const size_t edge_off = cv.take(sizeof(float) * 2 * (size_t)order * nt);
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    ram::StepArgs p;
    if ((st = make_rows(ctx, layout, edges, rp, p.rows)) != RAM_OK) return st;
    p.v0 = v0;
    p.dt = dt;
    const ram::FastPlan fp = ram::fast_plan_at((char *)ctx->scratch + rec_off, nt);
    const hipError_t e = ram::launch_plan_fast(p, order, fp, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "tile plan launch");
    a = ram::StepAdjArgs();
    a.rows = p.rows;
    a.dv = dv;
    a.dvbar = dvbar;
    a.v0bar = v0bar;
    a.v0part = (double *)((char *)ctx->scratch + v0_off);
    a.v0 = v0;
    a.dt = dt;
    a.fast = fp;
    a.edge = (float *)((char *)ctx->scratch + edge_off);
    return RAM_OK;
}

// One step backwards on a shared mesh: window plan of the shift (no halo),
// then the zeroing pass and the fused adjoint.
ram_status step_adjoint_shared(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                               const void *q_fwd, const void *q_half, const void *dv,
                               const void *qbar_out, void *qbar_in, const double *edges,
                               const double *v0, double dt, int order, void *dvbar,
                               double *v0bar)
{
    ram_status st;
    Carve cv;
    if (use_fast_adjoint(ctx, layout, dtype, {q_fwd, q_half, dv, qbar_out, qbar_in, dvbar})) {
        ram::StepAdjArgs a;
        if ((st = plan_adjoint_fast(ctx, layout, edges, v0, dt, order, dv, dvbar, v0bar, a)) !=
            RAM_OK)
            return st;
        a.q_fwd = q_fwd;
        a.q_half = q_half;
        a.qbar_out = qbar_out;
        a.qbar_in = qbar_in;
        const hipError_t e = ram::launch_step_adjoint_fast(a, order, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "step adjoint launch");
        return RAM_OK;
    }
    // the residual transpose stages cells i0-2 .. i0+nd+1: the fused tile
    // size keeps them within one item per thread
    RowsPlan rp = plan_rows(cv, layout, ram::step_tile(true), order);
    rp.uniform = dtype == RAM_F32;
    const int64_t nt = tiles_of(layout, rp.tile);
    const size_t wlo_off = cv.take(sizeof(int64_t) * nt), w_off = cv.take(ram::kPlanW * sizeof(int32_t) * nt);
    const size_t v0_off = cv.take(v0bar ? sizeof(double) * nt : 0);
    const size_t edge_off = cv.take(ram::adj_edge_bytes(nt, order, elem_size(dtype)));
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    ram::StepArgs p;
    if ((st = make_rows(ctx, layout, edges, rp, p.rows)) != RAM_OK) return st;
    p.v0 = v0;
    p.dt = dt;
    int64_t *wlo = (int64_t *)((char *)ctx->scratch + wlo_off);
    int32_t *w = (int32_t *)((char *)ctx->scratch + w_off);
    hipError_t e = ram::launch_plan(p, order, wlo, w, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "window plan launch");
    ram::StepAdjArgs a;
    a.rows = p.rows;
    a.q_fwd = q_fwd;
    a.q_half = q_half;
    a.dv = dv;
    a.qbar_out = qbar_out;
    a.qbar_in = qbar_in;
    a.dvbar = dvbar;
    a.v0bar = v0bar;
    a.v0part = (double *)((char *)ctx->scratch + v0_off);
    a.v0 = v0;
    a.dt = dt;
    a.plan_wlo = wlo;
    a.plan_w = w;
    a.edge = (char *)ctx->scratch + edge_off;
    e = ram::launch_step_adjoint_shared(a, dtype == RAM_F64, order, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "step adjoint launch");
    return RAM_OK;
}

} // namespace

extern "C" {

const char *ram_version(void) { return "ram-mi355x 0.1"; }

const char *ram_last_error(void) { return g_last_error.c_str(); }

const char *ram_status_string(ram_status s)
{
    switch (s) {
    case RAM_OK: return "ok";
    case RAM_E_INVALID_ARG: return "invalid argument";
    case RAM_E_UNSUPPORTED: return "unsupported configuration";
    case RAM_E_MESH: return "invalid mesh";
    case RAM_E_CFL: return "residual Courant condition violated";
    case RAM_E_HIP: return "HIP runtime error";
    case RAM_E_NOMEM: return "out of device memory";
    }
    return "unknown status";
}

ram_status ram_create(ram_ctx **out, int device, void *stream)
{
    if (!out) return fail(RAM_E_INVALID_ARG, "null output pointer");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= count)
        return fail(RAM_E_INVALID_ARG, "device %d out of range (%d devices)", device, count);
    e = hipSetDevice(device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    ram_ctx *ctx = new (std::nothrow) ram_ctx;
    if (!ctx) return fail(RAM_E_NOMEM, "host allocation failed");
    ctx->device = device;
    ctx->stream = (hipStream_t)stream;
    e = hipEventCreateWithFlags(&ctx->handoff, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete ctx;
        return hip_fail(e, "hipEventCreateWithFlags");
    }
    // the static scratch of ram_shift_noalloc: its address on this device,
    // looked up once (a failure surfaces when that entry point is called)
    (void)ram::noalloc_setup(device);
    *out = ctx;
    g_last_error.clear();
    return RAM_OK;
}

ram_status ram_destroy(ram_ctx *ctx)
{
    if (!ctx) return RAM_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->fork.side) (void)hipStreamDestroy(ctx->fork.side);
    if (ctx->fork.fork) (void)hipEventDestroy(ctx->fork.fork);
    if (ctx->fork.join) (void)hipEventDestroy(ctx->fork.join);
    if (ctx->handoff) (void)hipEventDestroy(ctx->handoff);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    delete ctx;
    return RAM_OK;
}

ram_status ram_set_schedule(ram_ctx *ctx, const ram_schedule *sched)
{
    if (!ctx) return fail(RAM_E_INVALID_ARG, "null context");
    if (!sched) return fail(RAM_E_INVALID_ARG, "null schedule");
    const int items = sched->items_per_thread;
    if (items != 0 && !ram::valid_items(items))
        return fail(RAM_E_UNSUPPORTED, "items_per_thread must be 0 or 2..5 (got %d)",
                    (int)sched->items_per_thread);
    ctx->items = items;
    return RAM_OK;
}

ram_status ram_set_mesh_density(ram_ctx *ctx, const ram_mesh_density *d)
{
    if (!ctx) return fail(RAM_E_INVALID_ARG, "null context");
    if (!d || d->kind == RAM_DENSITY_NONE) {
        ctx->density = ram_mesh_density{};
        return RAM_OK;
    }
    if (d->kind != RAM_DENSITY_PERIODIC_BUMP)
        return fail(RAM_E_UNSUPPORTED, "unknown mesh density kind %d", (int)d->kind);
    const double v[5] = {d->xmin, d->xmax, d->a, d->b, d->c};
    for (double t : v)
        if (!std::isfinite(t)) return fail(RAM_E_INVALID_ARG, "mesh density parameters must be finite");
    if (!(d->xmin <= -d->b && -d->b < -d->a && d->a > 0.0 && d->a < d->b && d->b <= d->xmax))
        return fail(RAM_E_INVALID_ARG, "periodic bump needs xmin <= -b < -a < 0 < a < b <= xmax");
    if (!(d->c > -1.0)) return fail(RAM_E_INVALID_ARG, "periodic bump needs c > -1");
    ctx->density = *d;
    return RAM_OK;
}

ram_status ram_mesh_density_cells(ram_ctx *ctx, const ram_mesh_density *d, int64_t n,
                                  const double *x, int64_t m, int32_t *cells)
{
    ram_status st;
    g_last_error.clear();
    if (!d || d->kind != RAM_DENSITY_PERIODIC_BUMP)
        return fail(RAM_E_UNSUPPORTED, "a mesh density of kind RAM_DENSITY_PERIODIC_BUMP is needed");
    if (n < 1 || n > INT32_MAX - 1 || m < 0) return fail(RAM_E_INVALID_ARG, "bad n or m");
    if (m > 0 && (!x || !cells)) return fail(RAM_E_INVALID_ARG, "null x or cells");
    if ((st = enter(ctx)) != RAM_OK) return st;
    hipError_t e = ram::launch_density_cells(make_density(*d, n), (int)n, x, m, cells,
                                             ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "density cells launch");
    return RAM_OK;
}

ram_status ram_get_schedule(const ram_ctx *ctx, ram_schedule *sched)
{
    if (!ctx || !sched) return fail(RAM_E_INVALID_ARG, "null context or schedule");
    sched->items_per_thread = ctx->items;
    return RAM_OK;
}

ram_status ram_set_stream(ram_ctx *ctx, void *stream)
{
    if (!ctx) return fail(RAM_E_INVALID_ARG, "null context");
    if ((hipStream_t)stream == ctx->stream) return RAM_OK;
    ram_status st = enter(ctx);
    if (st != RAM_OK) return st;
    HipStreams api;
    if (ram::switch_stream(api, ctx->stream, (hipStream_t)stream, ctx->handoff) != 0)
        return hip_fail(api.err, "stream hand-off");
    return RAM_OK;
}

ram_status ram_sync(ram_ctx *ctx)
{
    ram_status st = enter(ctx);
    if (st != RAM_OK) return st;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return RAM_OK;
}

ram_status ram_shift(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                     ram_scan scan, const void *q_in, void *q_out,
                     const double *edges, const double *v0, double dt,
                     int order)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_scan(dtype, scan)) != RAM_OK) return st;
    if ((st = check_order(layout, order)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!q_in || !q_out || !v0) return fail(RAM_E_INVALID_ARG, "null q_in, q_out or v0");
    if (q_in == q_out) return fail(RAM_E_INVALID_ARG, "q_in and q_out must not alias");
    if ((st = enter(ctx)) != RAM_OK) return st;
    const int items = sched_items(ctx, layout, scan);
    Carve cv;
    RowsPlan rp = plan_rows(cv, layout, step_tile_of(ctx, layout, dtype, scan, items, false),
                            order);
    rp.uniform = wants_uniform(dtype, scan) || use_fast(ctx, layout, dtype, scan);
    const int64_t nt = tiles_of(layout, rp.tile);
    const size_t wlo_off = cv.take(sizeof(int64_t) * nt), w_off = cv.take(plan_w_bytes(nt));
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    ram::StepArgs a;
    if ((st = make_rows(ctx, layout, edges, rp, a.rows)) != RAM_OK) return st;
    a.q_in = q_in;
    a.q_out = q_out;
    a.v0 = v0;
    a.dt = dt;
    if ((st = launch_steps(ctx, a, dtype, scan, order, 1, nullptr, wlo_off, w_off, 0,
                           items)) != RAM_OK)
        return st;
    return RAM_OK;
}

ram_status ram_shift_noalloc(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                             ram_scan scan, const void *q_in, void *q_out,
                             const double *edges, const double *v0, double dt, int order)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_scan(dtype, scan)) != RAM_OK) return st;
    if ((st = check_order(layout, order)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!q_in || !q_out || !v0) return fail(RAM_E_INVALID_ARG, "null q_in, q_out or v0");
    if (q_in == q_out) return fail(RAM_E_INVALID_ARG, "q_in and q_out must not alias");
    if ((st = enter(ctx)) != RAM_OK) return st;
    char *mem = (char *)ram::noalloc_scratch(ctx->device);
    if (!mem) {
        const hipError_t e = ram::noalloc_setup(ctx->device);
        mem = (char *)ram::noalloc_scratch(ctx->device);
        if (!mem) return hip_fail(e, "static scratch of ram_shift_noalloc");
    }
    // the general kernels (the streaming kernel's per-call node data would
    // not fit a modest static buffer)
    const int items = sched_items(ctx, layout, scan);
    Carve cv;
    RowsPlan rp = plan_rows(cv, layout, ram::step_tile_for(items, false), order);
    rp.uniform = wants_uniform(dtype, scan);
    const int64_t nt = tiles_of(layout, rp.tile);
    const size_t wlo_off = cv.take(sizeof(int64_t) * nt),
                 w_off = cv.take(ram::kPlanW * sizeof(int32_t) * nt);
    if (cv.off > ram::kNoAllocBytes)
        return fail(RAM_E_NOMEM,
                    "ram_shift_noalloc needs %zu bytes of device scratch for this layout; "
                    "its static buffer holds %zu",
                    cv.off, ram::kNoAllocBytes);
    ram::StepArgs a;
    if ((st = make_rows(ctx, layout, edges, rp, a.rows, mem)) != RAM_OK) return st;
    a.q_in = q_in;
    a.q_out = q_out;
    a.v0 = v0;
    a.dt = dt;
    return launch_steps(ctx, a, dtype, scan, order, 1, nullptr, wlo_off, w_off, 0, items, 0, mem,
                        false);
}

ram_status ram_residual(ram_ctx *ctx, const ram_layout *layout,
                        ram_dtype dtype, const void *q_in, void *q_out,
                        const double *edges, const void *dv, double dt)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!q_in || !q_out || !dv) return fail(RAM_E_INVALID_ARG, "null q_in, q_out or dv");
    if (q_in == q_out) return fail(RAM_E_INVALID_ARG, "q_in and q_out must not alias");
    if ((st = enter(ctx)) != RAM_OK) return st;
    Carve cv;
    RowsPlan rp = plan_rows(cv, layout, ram::kResTile, 1);
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    ram::ResidualArgs a;
    if ((st = make_rows(ctx, layout, edges, rp, a.rows)) != RAM_OK) return st;
    a.q_in = q_in;
    a.q_out = q_out;
    a.dv = dv;
    a.dt = dt;
    hipError_t e = ram::launch_residual(a, dtype == RAM_F64, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "residual launch");
    return RAM_OK;
}

ram_status ram_step(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                    ram_scan scan, void *q, const double *edges,
                    const double *v0, const void *dv, double dt, int order,
                    int64_t n_steps)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_scan(dtype, scan)) != RAM_OK) return st;
    if ((st = check_order(layout, order)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!q || !v0) return fail(RAM_E_INVALID_ARG, "null q or v0");
    if (n_steps < 0) return fail(RAM_E_INVALID_ARG, "n_steps must be >= 0");
    if (n_steps == 0) return RAM_OK;
    if ((st = enter(ctx)) != RAM_OK) return st;
    const size_t state_bytes = elem_size(dtype) * (size_t)layout_cells(layout);
    Carve cv;
    const size_t tmp_off = cv.take(state_bytes);
    const int items = sched_items(ctx, layout, scan);
    const bool rag = use_rag(ctx, layout, dtype, dv, n_steps);
    RowsPlan rp = plan_rows(cv, layout,
                            rag ? ram::kRagTile
                                : step_tile_of(ctx, layout, dtype, scan, items, dv != nullptr),
                            order);
    rp.uniform = wants_uniform(dtype, scan) || use_fast(ctx, layout, dtype, scan);
    const int64_t nt = tiles_of(layout, rp.tile);
    const size_t wlo_off = cv.take(sizeof(int64_t) * nt), w_off = cv.take(plan_w_bytes(nt));
    const int64_t rag_off =
        rag ? (int64_t)cv.take(ram::rag_plan_bytes(nt, layout_cells(layout))) : -1;
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    ram::StepArgs a;
    std::memset(&a, 0, sizeof(a));        // the graph key compares raw bytes
    if ((st = make_rows(ctx, layout, edges, rp, a.rows)) != RAM_OK) return st;
    a.q_in = q;
    a.v0 = v0;
    a.dv = dv;
    a.dt = dt;
    void *tmp = (char *)ctx->scratch + tmp_off;
    if ((st = launch_steps(ctx, a, dtype, scan, order, n_steps, tmp, wlo_off, w_off,
                           state_bytes, items, 0, nullptr, true, rag_off)) != RAM_OK)
        return st;
    return RAM_OK;
}

ram_status ram_shift_limited(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                             ram_recon recon, const void *q_in, void *q_out,
                             const double *edges, const double *v0, double dt)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_recon(layout, recon)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!q_in || !q_out || !v0) return fail(RAM_E_INVALID_ARG, "null q_in, q_out or v0");
    if (q_in == q_out) return fail(RAM_E_INVALID_ARG, "q_in and q_out must not alias");
    if ((st = enter(ctx)) != RAM_OK) return st;
    const bool shared = layout->edges_shared && layout->n_cols > 0;
    const bool fast = shared && use_fast_lim(ctx, layout, dtype);
    Carve cv;
    RowsPlan rp = plan_rows(cv, layout, fast ? ram::kFastTile : ram::step_tile(false), 1);
    rp.uniform = fast;
    const int64_t nt = tiles_of(layout, rp.tile);
    const size_t wlo_off = shared ? cv.take(sizeof(int64_t) * nt) : 0;
    const size_t w_off = shared ? cv.take(plan_w_bytes(nt)) : 0;
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    ram::StepArgs a;
    if ((st = make_rows(ctx, layout, edges, rp, a.rows)) != RAM_OK) return st;
    a.q_in = q_in;
    a.q_out = q_out;
    a.v0 = v0;
    a.dt = dt;
    if (shared)
        return launch_steps(ctx, a, dtype, RAM_SUM_DIRECT, 0, 1, nullptr, wlo_off, w_off, 0,
                            ram::kItems, (int)recon);
    hipError_t e = ram::launch_shift_limited(a, dtype == RAM_F64, (int)recon, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "limited shift launch");
    return RAM_OK;
}

ram_status ram_step_limited(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                            ram_recon recon, void *q, const double *edges,
                            const double *v0, const void *dv, double dt, int64_t n_steps)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_recon(layout, recon)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!q || !v0) return fail(RAM_E_INVALID_ARG, "null q or v0");
    if (n_steps < 0) return fail(RAM_E_INVALID_ARG, "n_steps must be >= 0");
    if (n_steps == 0) return RAM_OK;
    if ((st = enter(ctx)) != RAM_OK) return st;
    const size_t state_bytes = elem_size(dtype) * (size_t)layout_cells(layout);
    if (layout->edges_shared && layout->n_cols > 0) {
        // one fused kernel a step (limited shift + residual), window plan once
        Carve cv;
        const size_t tmp_off = cv.take(state_bytes);
        const bool fast = use_fast_lim(ctx, layout, dtype);
        RowsPlan rp = plan_rows(cv, layout,
                                fast ? ram::kFastTile : ram::step_tile(dv != nullptr), 1);
        rp.uniform = dtype == RAM_F32;
        const int64_t nt = tiles_of(layout, rp.tile);
        const size_t wlo_off = cv.take(sizeof(int64_t) * nt);
        const size_t w_off = cv.take(plan_w_bytes(nt));
        if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
        ram::StepArgs a;
        std::memset(&a, 0, sizeof(a));    // the graph key compares raw bytes
        if ((st = make_rows(ctx, layout, edges, rp, a.rows)) != RAM_OK) return st;
        a.q_in = q;
        a.v0 = v0;
        a.dv = dv;
        a.dt = dt;
        return launch_steps(ctx, a, dtype, RAM_SUM_DIRECT, 0, n_steps,
                            (char *)ctx->scratch + tmp_off, wlo_off, w_off, state_bytes,
                            ram::kItems, (int)recon);
    }
    Carve cv;
    const size_t tmp_off = cv.take(state_bytes);
    // per-row meshes: the limited shift, then the residual kernel; the
    // shift's rows carry the mesh tables, the residual's rows share them
    RowsPlan rp = plan_rows(cv, layout, ram::step_tile(false), 1);
    RowsPlan rr = plan_rows(cv, layout, ram::kResTile, 0);
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    ram::StepArgs a;
    std::memset(&a, 0, sizeof(a));        // the graph key compares raw bytes
    if ((st = make_rows(ctx, layout, edges, rp, a.rows)) != RAM_OK) return st;
    ram::ResidualArgs r;
    std::memset(&r, 0, sizeof(r));
    if ((st = make_rows(ctx, layout, edges, rr, r.rows)) != RAM_OK) return st;
    r.rows.tab = a.rows.tab;
    r.rows.has_tab = a.rows.has_tab;
    a.v0 = v0;
    a.dt = dt;
    r.dv = dv;
    r.dt = dt;
    void *tmp = (char *)ctx->scratch + tmp_off;
    const bool f64 = dtype == RAM_F64;
    // with the residual: shift q -> tmp, residual tmp -> q; without: the
    // shifts ping-pong between q and tmp
    auto loop = [&](hipStream_t st) -> hipError_t {
        ram::StepArgs b = a;
        ram::ResidualArgs c = r;
        void *cur = q, *oth = tmp;
        for (int64_t k = 0; k < n_steps; ++k) {
            b.q_in = cur;
            b.q_out = oth;
            hipError_t e = ram::launch_shift_limited(b, f64, (int)recon, st);
            if (e != hipSuccess) return e;
            if (dv) {
                c.q_in = oth;
                c.q_out = cur;
                e = ram::launch_residual(c, f64, st);
                if (e != hipSuccess) return e;
            } else {
                void *t = cur; cur = oth; oth = t;
            }
        }
        if (cur != q) return ram::launch_copy(cur, q, (int64_t)state_bytes, st);
        return hipSuccess;
    };
    const int64_t extra[4] = {(int64_t)dtype * 16 + 256 * (int64_t)recon, -1, n_steps,
                              (int64_t)(intptr_t)q ^ (int64_t)state_bytes};
    return run_graphed(ctx, key_of(a, r, extra, tmp), n_steps, loop);
}

ram_status ram_step_limited_record(ram_ctx *ctx, const ram_layout *layout,
                                   ram_dtype dtype, ram_recon recon, void *q_traj,
                                   void *q_half, const double *edges, const double *v0,
                                   const void *dv, double dt, int64_t n_steps)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_recon(layout, recon)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!q_traj || !v0) return fail(RAM_E_INVALID_ARG, "null q_traj or v0");
    if (dv && !q_half) return fail(RAM_E_INVALID_ARG, "a step with dv needs q_half");
    if (n_steps < 0) return fail(RAM_E_INVALID_ARG, "n_steps must be >= 0");
    if (n_steps == 0) return RAM_OK;
    if ((st = enter(ctx)) != RAM_OK) return st;
    const size_t state_bytes = elem_size(dtype) * (size_t)layout_cells(layout);
    const bool f64 = dtype == RAM_F64;
    const bool shared = layout->edges_shared && layout->n_cols > 0;
    Carve cv;
    // shared mesh: the fused kernel with the post-shift state written out;
    // per-row meshes: the shift kernel into q_half, then the residual kernel
    const bool fast = shared && use_fast_lim(ctx, layout, dtype);
    RowsPlan rp = plan_rows(cv, layout,
                            fast ? ram::kFastTile
                                 : (shared ? ram::step_tile(dv != nullptr) : ram::step_tile(false)),
                            1);
    rp.uniform = shared && dtype == RAM_F32;
    const int64_t nt = tiles_of(layout, rp.tile);
    const size_t wlo_off = shared ? cv.take(sizeof(int64_t) * nt) : 0;
    const size_t w_off = shared ? cv.take(plan_w_bytes(nt)) : 0;
    RowsPlan rr = plan_rows(cv, layout, ram::kResTile, 0);
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    ram::StepArgs a;
    if ((st = make_rows(ctx, layout, edges, rp, a.rows)) != RAM_OK) return st;
    ram::ResidualArgs r;
    if (!shared) {
        if ((st = make_rows(ctx, layout, edges, rr, r.rows)) != RAM_OK) return st;
        r.rows.tab = a.rows.tab;
        r.rows.has_tab = a.rows.has_tab;
        r.dv = dv;
        r.dt = dt;
    }
    a.v0 = v0;
    a.dt = dt;
    hipError_t e;
    if (shared) {
        a.dv = dv;
        e = plan_shared(a, recon == RAM_RECON_PLM ? 3 : 5, fast, (char *)ctx->scratch + wlo_off,
                        (char *)ctx->scratch + w_off, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "window plan launch");
    }
    for (int64_t k = 0; k < n_steps; ++k) {
        void *qi = (char *)q_traj + k * state_bytes;
        void *qo = (char *)q_traj + (k + 1) * state_bytes;
        void *qh = dv ? (char *)q_half + k * state_bytes : nullptr;
        a.q_in = qi;
        if (shared) {
            a.q_out = qo;
            a.q_mid = qh;
            e = ram::launch_step_shared_limited(a, f64, (int)recon, ctx->stream);
        } else {
            a.q_out = dv ? qh : qo;
            e = ram::launch_shift_limited(a, f64, (int)recon, ctx->stream);
            if (e == hipSuccess && dv) {
                r.q_in = qh;
                r.q_out = qo;
                e = ram::launch_residual(r, f64, ctx->stream);
            }
        }
        if (e != hipSuccess) return hip_fail(e, "limited step launch");
    }
    return RAM_OK;
}

} // extern "C"

namespace {

// The limited shift's transpose on the general kernel (any layout): into
// qbar_in, or with qbar_in null into a scratch state copied back over
// qbar_out's buffer `back` afterwards (a residual transpose's output).
ram_status limited_adjoint_general(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                                   ram_recon recon, const void *q_fwd, const void *qbar_out,
                                   void *qbar_in, void *back, const double *edges,
                                   const double *v0, double dt, double *v0bar_accum)
{
    ram_status st;
    Carve cv;
    // a shared mesh brings its tables (centre gaps, PPM weights)
    RowsPlan rp = plan_rows(cv, layout, ram::kAdjTile, 1);
    const size_t v0_off =
        cv.take(v0bar_accum ? sizeof(double) * tiles_of(layout, ram::kAdjTile) : 0);
    const size_t state_bytes = elem_size(dtype) * (size_t)layout_cells(layout);
    const size_t tmp_off = qbar_in ? 0 : cv.take(state_bytes);
    const int64_t nt = tiles_of(layout, ram::kAdjTile);
    const int p = recon == RAM_RECON_PLM ? 3 : 5;
    const size_t edge_off = cv.take(ram::adj_edge_bytes(nt, p, elem_size(dtype)));
    const size_t ws_off = cv.take(sizeof(int64_t) * nt);
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    ram::ShiftAdjArgs a;
    if ((st = make_rows(ctx, layout, edges, rp, a.rows)) != RAM_OK) return st;
    a.q_fwd = q_fwd;
    a.qbar_out = qbar_out;
    a.qbar_in = qbar_in ? qbar_in : (char *)ctx->scratch + tmp_off;
    a.v0 = v0;
    a.dt = dt;
    a.v0bar = v0bar_accum;
    a.v0part = (double *)((char *)ctx->scratch + v0_off);
    a.edge = (char *)ctx->scratch + edge_off;
    a.wstart = (int64_t *)((char *)ctx->scratch + ws_off);
    hipError_t e = ram::launch_shift_limited_adjoint(a, dtype == RAM_F64, (int)recon,
                                                     ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "limited shift adjoint launch");
    if (!qbar_in) {
        e = ram::launch_copy(a.qbar_in, back, (int64_t)state_bytes, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "copy launch");
    }
    return RAM_OK;
}

// The streaming limited adjoint (FP32 state, shared mesh, default schedule,
// rows of a multiple of four cells): one tile plan of the reconstruction's
// stencil width, then the fused kernel.
ram_status limited_adjoint_fast(ram_ctx *ctx, const ram_layout *layout, ram_recon recon,
                                const void *q_fwd, const void *q_half, const void *dv,
                                const void *qbar_out, void *qbar_in, const double *edges,
                                const double *v0, double dt, void *dvbar, double *v0bar)
{
    ram_status st;
    const int order = recon == RAM_RECON_PLM ? 3 : 5;
    ram::StepAdjArgs a;
    if ((st = plan_adjoint_fast(ctx, layout, edges, v0, dt, order, dv, dvbar, v0bar, a)) !=
        RAM_OK)
        return st;
    a.q_fwd = q_fwd;
    a.q_half = q_half;
    a.qbar_out = qbar_out;
    a.qbar_in = qbar_in;
    const hipError_t e = ram::launch_step_limited_adjoint_fast(a, (int)recon, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "limited step adjoint launch");
    return RAM_OK;
}

} // namespace

extern "C" {

ram_status ram_shift_limited_adjoint(ram_ctx *ctx, const ram_layout *layout,
                                     ram_dtype dtype, ram_recon recon, const void *q_fwd,
                                     const void *qbar_out, void *qbar_in,
                                     const double *edges, const double *v0, double dt,
                                     double *v0bar_accum)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_recon(layout, recon)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!q_fwd || !qbar_out || !qbar_in || !v0)
        return fail(RAM_E_INVALID_ARG, "null q_fwd, qbar_out, qbar_in or v0");
    if (qbar_in == qbar_out || qbar_in == q_fwd)
        return fail(RAM_E_INVALID_ARG, "qbar_in must not alias qbar_out or q_fwd");
    if ((st = enter(ctx)) != RAM_OK) return st;
    if (layout->edges_shared && use_fast_adjoint(ctx, layout, dtype, {q_fwd, qbar_out, qbar_in}))
        return limited_adjoint_fast(ctx, layout, recon, q_fwd, nullptr, nullptr, qbar_out,
                                    qbar_in, edges, v0, dt, nullptr, v0bar_accum);
    return limited_adjoint_general(ctx, layout, dtype, recon, q_fwd, qbar_out, qbar_in, nullptr,
                                   edges, v0, dt, v0bar_accum);
}

ram_status ram_step_limited_adjoint(ram_ctx *ctx, const ram_layout *layout,
                                    ram_dtype dtype, ram_recon recon, const void *q_fwd,
                                    const void *q_half, const void *dv,
                                    const void *qbar_out, void *qbar_in,
                                    const double *edges, const double *v0, double dt,
                                    void *dvbar_accum, double *v0bar_accum)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_recon(layout, recon)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!q_fwd || !qbar_out || !qbar_in || !v0)
        return fail(RAM_E_INVALID_ARG, "null q_fwd, qbar_out, qbar_in or v0");
    if (dv && !q_half) return fail(RAM_E_INVALID_ARG, "a step with dv needs q_half");
    if (dvbar_accum && !dv) return fail(RAM_E_INVALID_ARG, "dvbar needs dv");
    if (qbar_in == qbar_out || qbar_in == q_fwd || qbar_in == q_half || qbar_in == dv)
        return fail(RAM_E_INVALID_ARG, "qbar_in must not alias an input");
    if ((st = enter(ctx)) != RAM_OK) return st;
    if (layout->edges_shared &&
        use_fast_adjoint(ctx, layout, dtype, {q_fwd, q_half, dv, qbar_out, qbar_in, dvbar_accum}))
        return limited_adjoint_fast(ctx, layout, recon, q_fwd, q_half, dv, qbar_out, qbar_in,
                                    edges, v0, dt, dvbar_accum, v0bar_accum);
    if (!dv)
        return limited_adjoint_general(ctx, layout, dtype, recon, q_fwd, qbar_out, qbar_in,
                                       nullptr, edges, v0, dt, v0bar_accum);
    // the residual's transpose into qbar_in, then the limited shift's into
    // scratch, copied back over qbar_in
    if ((st = ram_residual_adjoint(ctx, layout, dtype, q_half, dv, qbar_out, qbar_in, edges, dt,
                                   dvbar_accum)) != RAM_OK)
        return st;
    return limited_adjoint_general(ctx, layout, dtype, recon, q_fwd, qbar_in, nullptr, qbar_in,
                                   edges, v0, dt, v0bar_accum);
}

// q_out == nullptr checks an in-place caller (q_in is its state)
ram_status check_radial(const ram_layout *layout, ram_dtype dtype, const void *q_in,
                        const void *q_out, const double *r_edges, const void *u, double dt,
                        bool in_place = false)
{
    ram_status st;
    if (!layout) return fail(RAM_E_INVALID_ARG, "null layout");
    if (layout->n_cols <= 0 || layout->n_rows < 1)
        return fail(RAM_E_INVALID_ARG, "radial transport needs uniform rows (n_cols > 0)");
    if (layout->n_rows > 65535) return fail(RAM_E_INVALID_ARG, "at most 65535 radial rows");
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!q_in || (!q_out && !in_place) || !r_edges || !u)
        return fail(RAM_E_INVALID_ARG, "null q, r_edges or u");
    if (q_in == q_out) return fail(RAM_E_INVALID_ARG, "q_in and q_out must not alias");
    return RAM_OK;
}

ram_status ram_radial_step(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                           const void *q_in, void *q_out, const double *r_edges,
                           const void *u, double dt)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_radial(layout, dtype, q_in, q_out, r_edges, u, dt)) != RAM_OK) return st;
    if ((st = enter(ctx)) != RAM_OK) return st;
    ram::RadialArgs r;
    r.n_rows = layout->n_rows;
    r.n_cols = layout->n_cols;
    r.r_edges = r_edges;
    r.q_in = q_in;
    r.q_out = q_out;
    r.u = u;
    r.dt = dt;
    hipError_t e = ram::launch_radial(r, dtype == RAM_F64, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "radial step launch");
    return RAM_OK;
}

// The row step inside a loop that does more than the step each time (the 2D
// split step, the step on centre values): its checks, and the tables, window
// plan and index the step kernels read, set up once per call.
struct RowStep {
    ram::StepArgs a;
    ram_scan scan = RAM_SCAN_F64;
    int recon = 0, order = 0, items = 0;
    bool f64 = false, shared = false;

    hipError_t launch(const void *in, void *out, hipStream_t st) const
    {
        ram::StepArgs b = a;
        b.q_in = in;
        b.q_out = out;
        if (recon) return ram::launch_step_shared_limited(b, f64, recon, st);
        if (shared) return ram::launch_step_shared(b, f64, (int)scan, order, items, st);
        return ram::launch_step(b, f64, (int)scan, order, st);
    }
};

// Lagrange (recon 0: scan and order) or limited (shared meshes only) row step.
ram_status check_row_step(const ram_layout *layout, ram_dtype dtype, ram_scan scan,
                          ram_recon recon, const double *edges, const double *v0, int order,
                          int64_t n_steps)
{
    ram_status st;
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if (recon == 0) {
        if ((st = check_scan(dtype, scan)) != RAM_OK) return st;
        if ((st = check_order(layout, order)) != RAM_OK) return st;
    } else {
        if ((st = check_dtype(dtype)) != RAM_OK) return st;
        if ((st = check_recon(layout, recon)) != RAM_OK) return st;
        if (!layout->edges_shared || layout->n_cols <= 0)
            return fail(RAM_E_UNSUPPORTED, "limited steps in a loop need a shared mesh");
    }
    if (!v0) return fail(RAM_E_INVALID_ARG, "null v0");
    if (n_steps < 0) return fail(RAM_E_INVALID_ARG, "n_steps must be >= 0");
    return RAM_OK;
}

// After the caller has taken its own buffers from cv (and called enter).
ram_status setup_row_step(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                          ram_scan scan, ram_recon recon, const double *edges,
                          const double *v0, const void *dv, double dt, int order, Carve &cv,
                          RowStep &rs)
{
    ram_status st;
    if (recon) scan = RAM_SUM_DIRECT;
    rs.scan = scan;
    rs.recon = (int)recon;
    rs.order = order;
    rs.f64 = dtype == RAM_F64;
    rs.items = recon ? ram::kItems : sched_items(ctx, layout, scan);
    const int plan_order = recon == 0 ? order : (recon == RAM_RECON_PLM ? 3 : 5);
    const bool fast = recon == 0 ? use_fast(ctx, layout, dtype, scan)
                                 : use_fast_lim(ctx, layout, dtype);
    RowsPlan rp = plan_rows(cv, layout,
                            fast ? ram::kFastTile : ram::step_tile_for(rs.items, dv != nullptr),
                            plan_order);
    rp.uniform = (dtype == RAM_F32 && (recon != 0 || scan == RAM_SUM_DIRECT)) || fast;
    const int64_t nt = tiles_of(layout, rp.tile);
    const size_t wlo_off = cv.take(sizeof(int64_t) * nt), w_off = cv.take(plan_w_bytes(nt));
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    std::memset(&rs.a, 0, sizeof(rs.a));   // graph keys compare raw bytes
    if ((st = make_rows(ctx, layout, edges, rp, rs.a.rows)) != RAM_OK) return st;
    rs.a.v0 = v0;
    rs.a.dv = dv;
    rs.a.dt = dt;
    rs.shared = rs.a.rows.has_tab != 0 && rs.a.rows.n_cols > 0;
    if (rs.shared) {
        hipError_t e = plan_shared(rs.a, plan_order, fast, (char *)ctx->scratch + wlo_off,
                                   (char *)ctx->scratch + w_off, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "window plan launch");
        if (scan == RAM_SUM_DIRECT && recon == 0)
            rs.a.dens = make_density(ctx->density, rs.a.rows.n_cols);
    }
    return RAM_OK;
}

ram_status ram_step_split2d(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                            ram_scan scan, ram_recon recon, void *q, const double *edges,
                            const double *v0, const void *dv, const double *r_edges,
                            const void *u, double dt, int order, int64_t n_steps)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_row_step(layout, dtype, scan, recon, edges, v0, order, n_steps)) != RAM_OK)
        return st;
    if ((st = check_radial(layout, dtype, q, nullptr, r_edges, u, dt, true)) != RAM_OK) return st;
    if (n_steps == 0) return RAM_OK;
    if ((st = enter(ctx)) != RAM_OK) return st;
    Carve cv;
    const size_t tmp_off = cv.take(elem_size(dtype) * (size_t)layout_cells(layout));
    RowStep rs;
    if ((st = setup_row_step(ctx, layout, dtype, scan, recon, edges, v0, dv, dt, order, cv,
                             rs)) != RAM_OK)
        return st;
    ram::RadialArgs r;
    std::memset(&r, 0, sizeof(r));
    r.n_rows = layout->n_rows;
    r.n_cols = layout->n_cols;
    r.r_edges = r_edges;
    r.u = u;
    r.dt = dt;
    void *tmp = (char *)ctx->scratch + tmp_off;
    // per step: the RAM step along the rows (q -> tmp), then the radial step
    // across them (tmp -> q)
    auto loop = [&](hipStream_t st) -> hipError_t {
        ram::RadialArgs c = r;
        for (int64_t k = 0; k < n_steps; ++k) {
            hipError_t e = rs.launch(q, tmp, st);
            if (e != hipSuccess) return e;
            c.q_in = tmp;
            c.q_out = q;
            e = ram::launch_radial(c, rs.f64, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    const int64_t extra[4] = {(int64_t)dtype * 16 + (int64_t)rs.scan + 256 * (int64_t)recon +
                                  4096 * (int64_t)rs.items,
                              order, n_steps, (int64_t)(intptr_t)q};
    return run_graphed(ctx, key_of(rs.a, r, extra, tmp), n_steps, loop);
}

// Uniform rows sharing one mesh.
bool shared_rows(const ram_layout *L) { return L->edges_shared && L->n_cols > 0; }

ram_status ram_cell_average(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                            const void *q_in, void *q_out, const double *edges, int to_centre)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if (to_centre != 0 && to_centre != 1)
        return fail(RAM_E_INVALID_ARG, "to_centre must be 0 or 1");
    if (!q_in || !q_out) return fail(RAM_E_INVALID_ARG, "null q_in or q_out");
    if (q_in == q_out) return fail(RAM_E_INVALID_ARG, "q_in and q_out must not alias");
    if ((st = enter(ctx)) != RAM_OK) return st;
    Carve cv;
    RowsPlan rp = plan_rows(cv, layout, ram::kAvgTile, 0);
    const bool tab = shared_rows(layout);
    const size_t w_off = tab ? cv.take(2 * elem_size(dtype) * (size_t)layout->n_cols) : 0;
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    ram::Rows R;
    if ((st = make_rows(ctx, layout, edges, rp, R)) != RAM_OK) return st;
    const bool f64 = dtype == RAM_F64;
    void *w = tab ? (char *)ctx->scratch + w_off : nullptr;
    hipError_t e = hipSuccess;
    if (tab) e = ram::launch_average4_weights(edges, layout->n_cols, f64, w, ctx->stream);
    if (e == hipSuccess)
        e = ram::launch_average4(R, f64, to_centre != 0, q_in, q_out, w, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "cell average launch");
    return RAM_OK;
}

ram_status ram_step_point4(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                           ram_scan scan, ram_recon recon, void *q, const double *edges,
                           const double *v0, const void *dv, double dt, int order,
                           int64_t n_steps)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_row_step(layout, dtype, scan, recon, edges, v0, order, n_steps)) != RAM_OK)
        return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!q) return fail(RAM_E_INVALID_ARG, "null q");
    if (n_steps == 0) return RAM_OK;
    if ((st = enter(ctx)) != RAM_OK) return st;
    const size_t state_bytes = elem_size(dtype) * (size_t)layout_cells(layout);
    Carve cv;
    const size_t t1_off = cv.take(state_bytes), t2_off = cv.take(state_bytes);
    RowsPlan rc = plan_rows(cv, layout, ram::kAvgTile, 0);
    const bool tab = shared_rows(layout);
    const size_t w_off = tab ? cv.take(2 * elem_size(dtype) * (size_t)layout->n_cols) : 0;
    RowStep rs;
    if ((st = setup_row_step(ctx, layout, dtype, scan, recon, edges, v0, dv, dt, order, cv,
                             rs)) != RAM_OK)
        return st;
    ram::Rows RC;
    std::memset(&RC, 0, sizeof(RC));
    if ((st = make_rows(ctx, layout, edges, rc, RC)) != RAM_OK) return st;
    void *t1 = (char *)ctx->scratch + t1_off;
    void *t2 = (char *)ctx->scratch + t2_off;
    void *w = tab ? (char *)ctx->scratch + w_off : nullptr;
    if (tab) {
        hipError_t e = ram::launch_average4_weights(edges, layout->n_cols, rs.f64, w,
                                                    ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "cell average weights launch");
    }
    // centre values -> averages (q -> t1); per step the step (t1 -> t2),
    // then, between steps, back to centre values and on to averages in one
    // pass (t2 -> t1); after the last, back to centre values (t2 -> q)
    auto loop = [&](hipStream_t st) -> hipError_t {
        hipError_t e = ram::launch_average4(RC, rs.f64, false, q, t1, w, st);
        if (e != hipSuccess) return e;
        for (int64_t k = 0; k < n_steps; ++k) {
            if ((e = rs.launch(t1, t2, st)) != hipSuccess) return e;
            e = k + 1 < n_steps ? ram::launch_average4_between(RC, rs.f64, t2, t1, w, st)
                                : ram::launch_average4(RC, rs.f64, true, t2, q, w, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    const int64_t extra[4] = {(int64_t)dtype * 16 + (int64_t)rs.scan + 256 * (int64_t)recon +
                                  4096 * (int64_t)rs.items + (1 << 20),
                              order, n_steps, (int64_t)(intptr_t)q};
    return run_graphed(ctx, key_of(rs.a, RC, extra, t1), n_steps, loop);
}

ram_status ram_step_tile_paths(ram_ctx *ctx, const ram_layout *layout, const double *edges,
                               const double *v0, double dt, int order, int with_residual,
                               int32_t *paths, int64_t cap, int64_t *n_tiles)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_order(layout, order)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!layout->edges_shared || layout->n_cols <= 0)
        return fail(RAM_E_UNSUPPORTED, "tile paths exist for shared meshes only");
    if (!v0 || !paths || !n_tiles) return fail(RAM_E_INVALID_ARG, "null v0, paths or n_tiles");
    const int64_t nt = tiles_of(layout, ram::kFastTile);
    *n_tiles = nt;
    if (cap < nt) return fail(RAM_E_INVALID_ARG, "paths holds %lld entries, %lld tiles",
                              (long long)cap, (long long)nt);
    if ((st = enter(ctx)) != RAM_OK) return st;
    Carve cv;
    RowsPlan rp = plan_rows(cv, layout, ram::kFastTile, order);
    rp.uniform = true;
    const size_t rec_off = cv.take(ram::fast_plan_bytes(nt));
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    ram::StepArgs a;
    std::memset(&a, 0, sizeof(a));
    if ((st = make_rows(ctx, layout, edges, rp, a.rows)) != RAM_OK) return st;
    a.v0 = v0;
    a.dt = dt;
    // only its being non-null matters to the plan (the halo)
    a.dv = with_residual ? (const void *)edges : nullptr;
    const ram::FastPlan fp = ram::fast_plan_at((char *)ctx->scratch + rec_off, nt);
    hipError_t e = ram::launch_plan_fast(a, order, fp, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "tile plan launch");
    // the kind is the record's first word
    e = hipMemcpy2DAsync(paths, sizeof(int32_t), fp.rec, sizeof(ram::FastTile), sizeof(int32_t),
                         (size_t)nt, hipMemcpyDeviceToDevice, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "tile path copy");
    return RAM_OK;
}

ram_status ram_row_norms(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                         const void *q, const void *q_ref, const double *edges,
                         double *out)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if (!q || !out) return fail(RAM_E_INVALID_ARG, "null q or out");
    if ((st = enter(ctx)) != RAM_OK) return st;
    ram::Rows R;
    R.n_rows = layout->n_rows;
    R.n_cols = layout->n_cols;
    R.row_ptr = layout->n_cols > 0 ? nullptr : layout->row_ptr;
    R.edges = edges;
    R.shared = layout->edges_shared ? 1 : 0;
    hipError_t e = ram::launch_row_norms(R, dtype == RAM_F64, q, q_ref, out, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "row norms launch");
    return RAM_OK;
}

ram_status ram_shift_adjoint(ram_ctx *ctx, const ram_layout *layout,
                             ram_dtype dtype, ram_scan scan,
                             const void *q_fwd, const void *qbar_out,
                             void *qbar_in, const double *edges,
                             const double *v0, double dt, int order,
                             double *v0bar_accum)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_scan(dtype, scan)) != RAM_OK) return st;
    if ((st = check_order(layout, order)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!qbar_out || !qbar_in || !v0) return fail(RAM_E_INVALID_ARG, "null qbar_out, qbar_in or v0");
    if (qbar_in == qbar_out) return fail(RAM_E_INVALID_ARG, "qbar_in and qbar_out must not alias");
    if (v0bar_accum && !q_fwd) return fail(RAM_E_INVALID_ARG, "v0bar needs the forward state q_fwd");
    if ((st = enter(ctx)) != RAM_OK) return st;
    if (layout->edges_shared)
        return step_adjoint_shared(ctx, layout, dtype, q_fwd, nullptr, nullptr, qbar_out,
                                   qbar_in, edges, v0, dt, order, nullptr, v0bar_accum);
    Carve cv;
    RowsPlan rp = plan_rows(cv, layout, ram::kAdjTile, 0);
    const int64_t nt = tiles_of(layout, ram::kAdjTile);
    const size_t v0_off = cv.take(v0bar_accum ? sizeof(double) * nt : 0);
    const size_t edge_off = cv.take(ram::adj_edge_bytes(nt, order, elem_size(dtype)));
    const size_t ws_off = cv.take(sizeof(int64_t) * nt);
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    ram::ShiftAdjArgs a;
    if ((st = make_rows(ctx, layout, edges, rp, a.rows)) != RAM_OK) return st;
    a.q_fwd = q_fwd;
    a.qbar_out = qbar_out;
    a.qbar_in = qbar_in;
    a.v0 = v0;
    a.dt = dt;
    a.v0bar = v0bar_accum;
    a.v0part = (double *)((char *)ctx->scratch + v0_off);
    a.edge = (char *)ctx->scratch + edge_off;
    a.wstart = (int64_t *)((char *)ctx->scratch + ws_off);
    hipError_t e = ram::launch_shift_adjoint(a, dtype == RAM_F64, order, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "shift adjoint launch");
    return RAM_OK;
}

ram_status ram_residual_adjoint(ram_ctx *ctx, const ram_layout *layout,
                                ram_dtype dtype, const void *q_fwd,
                                const void *dv, const void *qbar_out,
                                void *qbar_in, const double *edges, double dt,
                                void *dvbar_accum)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!q_fwd || !dv || !qbar_out || !qbar_in)
        return fail(RAM_E_INVALID_ARG, "null q_fwd, dv, qbar_out or qbar_in");
    if (qbar_in == qbar_out) return fail(RAM_E_INVALID_ARG, "qbar_in and qbar_out must not alias");
    if ((st = enter(ctx)) != RAM_OK) return st;
    Carve cv;
    RowsPlan rp = plan_rows(cv, layout, ram::kAdjTile, 0);
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    ram::ResidualAdjArgs a;
    if ((st = make_rows(ctx, layout, edges, rp, a.rows)) != RAM_OK) return st;
    a.q_fwd = q_fwd;
    a.dv = dv;
    a.qbar_out = qbar_out;
    a.qbar_in = qbar_in;
    a.dvbar = dvbar_accum;
    a.dt = dt;
    hipError_t e = ram::launch_residual_adjoint(a, dtype == RAM_F64, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "residual adjoint launch");
    return RAM_OK;
}

ram_status ram_step_record(ram_ctx *ctx, const ram_layout *layout,
                           ram_dtype dtype, ram_scan scan, void *q_traj,
                           void *q_half, const double *edges, const double *v0,
                           const void *dv, double dt, int order, int64_t n_steps)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_scan(dtype, scan)) != RAM_OK) return st;
    if ((st = check_order(layout, order)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!q_traj || !v0) return fail(RAM_E_INVALID_ARG, "null q_traj or v0");
    if (dv && !q_half) return fail(RAM_E_INVALID_ARG, "a step with dv needs q_half");
    if (n_steps < 0) return fail(RAM_E_INVALID_ARG, "n_steps must be >= 0");
    if (n_steps == 0) return RAM_OK;
    if ((st = enter(ctx)) != RAM_OK) return st;
    const size_t state_bytes = elem_size(dtype) * (size_t)layout_cells(layout);
    Carve cv;
    const int items = sched_items(ctx, layout, scan);
    const bool fast = use_fast(ctx, layout, dtype, scan);
    RowsPlan rp = plan_rows(cv, layout,
                            fast ? ram::kFastTile : ram::step_tile_for(items, dv != nullptr),
                            order);
    rp.uniform = wants_uniform(dtype, scan) || use_fast(ctx, layout, dtype, scan);
    const int64_t nt = tiles_of(layout, rp.tile);
    const size_t wlo_off = cv.take(sizeof(int64_t) * nt), w_off = cv.take(plan_w_bytes(nt));
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    ram::StepArgs a;
    if ((st = make_rows(ctx, layout, edges, rp, a.rows)) != RAM_OK) return st;
    a.v0 = v0;
    a.dv = dv;
    a.dt = dt;
    const bool f64 = dtype == RAM_F64;
    const bool shared = a.rows.has_tab != 0 && a.rows.n_cols > 0;
    hipError_t e;
    if (shared) {
        e = plan_shared(a, order, fast, (char *)ctx->scratch + wlo_off,
                        (char *)ctx->scratch + w_off, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "window plan launch");
    }
    for (int64_t k = 0; k < n_steps; ++k) {
        a.q_in = (const char *)q_traj + k * state_bytes;
        a.q_out = (char *)q_traj + (k + 1) * state_bytes;
        a.q_mid = dv ? (char *)q_half + k * state_bytes : nullptr;
        e = shared ? ram::launch_step_shared(a, f64, (int)scan, order, items, ctx->stream)
                   : ram::launch_step(a, f64, (int)scan, order, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "step launch");
    }
    return RAM_OK;
}

ram_status ram_step_adjoint(ram_ctx *ctx, const ram_layout *layout,
                            ram_dtype dtype, const void *q_fwd,
                            const void *q_half, const void *dv,
                            const void *qbar_out, void *qbar_in,
                            const double *edges, const double *v0, double dt,
                            int order, void *dvbar_accum, double *v0bar_accum)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_order(layout, order)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!qbar_out || !qbar_in || !v0) return fail(RAM_E_INVALID_ARG, "null qbar_out, qbar_in or v0");
    if (dv && !q_half) return fail(RAM_E_INVALID_ARG, "a step with dv needs q_half");
    if (v0bar_accum && !q_fwd) return fail(RAM_E_INVALID_ARG, "v0bar needs the forward state q_fwd");
    if (dvbar_accum && !dv) return fail(RAM_E_INVALID_ARG, "dvbar needs dv");
    if (qbar_in == qbar_out || qbar_in == q_fwd || qbar_in == q_half || qbar_in == dv)
        return fail(RAM_E_INVALID_ARG, "qbar_in must not alias an input");
    if ((st = enter(ctx)) != RAM_OK) return st;
    if (layout->edges_shared)
        return step_adjoint_shared(ctx, layout, dtype, q_fwd, q_half, dv, qbar_out, qbar_in,
                                   edges, v0, dt, order, dvbar_accum, v0bar_accum);
    // per-row meshes: the residual transpose into scratch, then the shift's
    const size_t state_bytes = elem_size(dtype) * (size_t)layout_cells(layout);
    Carve cv;
    const size_t mid_off = dv ? cv.take(state_bytes) : 0;
    RowsPlan rp = plan_rows(cv, layout, ram::kAdjTile, 0);
    const int64_t nt = tiles_of(layout, ram::kAdjTile);
    const size_t v0_off = cv.take(v0bar_accum ? sizeof(double) * nt : 0);
    const size_t edge_off = cv.take(ram::adj_edge_bytes(nt, order, elem_size(dtype)));
    const size_t ws_off = cv.take(sizeof(int64_t) * nt);
    if ((st = ensure_scratch(ctx, cv.off)) != RAM_OK) return st;
    ram::Rows rows;
    if ((st = make_rows(ctx, layout, edges, rp, rows)) != RAM_OK) return st;
    const void *qb = qbar_out;
    hipError_t e;
    if (dv) {
        ram::ResidualAdjArgs r;
        r.rows = rows;
        r.q_fwd = q_half;
        r.dv = dv;
        r.qbar_out = qbar_out;
        r.qbar_in = (char *)ctx->scratch + mid_off;
        r.dvbar = dvbar_accum;
        r.dt = dt;
        e = ram::launch_residual_adjoint(r, dtype == RAM_F64, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "residual adjoint launch");
        qb = r.qbar_in;
    }
    ram::ShiftAdjArgs a;
    a.rows = rows;
    a.q_fwd = q_fwd;
    a.qbar_out = qb;
    a.qbar_in = qbar_in;
    a.v0 = v0;
    a.dt = dt;
    a.v0bar = v0bar_accum;
    a.v0part = (double *)((char *)ctx->scratch + v0_off);
    a.edge = (char *)ctx->scratch + edge_off;
    a.wstart = (int64_t *)((char *)ctx->scratch + ws_off);
    e = ram::launch_shift_adjoint(a, dtype == RAM_F64, order, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "shift adjoint launch");
    return RAM_OK;
}

ram_status ram_step_adjoint_steps(ram_ctx *ctx, const ram_layout *layout,
                                  ram_dtype dtype, const void *q_traj,
                                  const void *q_half, const void *dv, void *qbar,
                                  void *qbar_work, const double *edges,
                                  const double *v0, double dt, int order,
                                  int64_t n_steps, void *dvbar_accum,
                                  double *v0bar_accum)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_order(layout, order)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if (!q_traj || !qbar || !qbar_work || !v0)
        return fail(RAM_E_INVALID_ARG, "null q_traj, qbar, qbar_work or v0");
    if (dv && !q_half) return fail(RAM_E_INVALID_ARG, "steps with dv need q_half");
    if (dvbar_accum && !dv) return fail(RAM_E_INVALID_ARG, "dvbar needs dv");
    if (n_steps < 0) return fail(RAM_E_INVALID_ARG, "n_steps must be >= 0");
    const size_t state_bytes = elem_size(dtype) * (size_t)layout_cells(layout);
    auto hits = [&](const void *p, const void *base, size_t bytes) {
        return base && (const char *)p + state_bytes > (const char *)base &&
               (const char *)p < (const char *)base + bytes;
    };
    const size_t traj_bytes = state_bytes * (size_t)n_steps;
    for (const void *p : {(const void *)qbar, (const void *)qbar_work})
        if (hits(p, q_traj, traj_bytes) || hits(p, q_half, traj_bytes) ||
            hits(p, dv, state_bytes) || hits(p, dvbar_accum, state_bytes))
            return fail(RAM_E_INVALID_ARG, "qbar and qbar_work must not overlap an input");
    if (hits(qbar, qbar_work, state_bytes))
        return fail(RAM_E_INVALID_ARG, "qbar and qbar_work must not overlap");
    if (n_steps == 0) return RAM_OK;
    if ((st = enter(ctx)) != RAM_OK) return st;
    void *cur = qbar, *oth = qbar_work;
    auto at = [&](const void *base, int64_t k) {
        return base ? (const void *)((const char *)base + (size_t)k * state_bytes) : nullptr;
    };
    if (layout->edges_shared &&
        use_fast_adjoint(ctx, layout, dtype, {q_traj, q_half, dv, qbar, qbar_work, dvbar_accum}) &&
        state_bytes % 16 == 0) {
        // one plan for every step: the shift is the same at each
        ram::StepAdjArgs a;
        if ((st = plan_adjoint_fast(ctx, layout, edges, v0, dt, order, dv, dvbar_accum,
                                    v0bar_accum, a)) != RAM_OK)
            return st;
        for (int64_t k = n_steps - 1; k >= 0; --k) {
            a.q_fwd = at(q_traj, k);
            a.q_half = dv ? at(q_half, k) : nullptr;
            a.qbar_out = cur;
            a.qbar_in = oth;
            const hipError_t e = ram::launch_step_adjoint_fast(a, order, ctx->stream);
            if (e != hipSuccess) return hip_fail(e, "step adjoint launch");
            std::swap(cur, oth);
        }
    } else {
        for (int64_t k = n_steps - 1; k >= 0; --k) {
            if ((st = ram_step_adjoint(ctx, layout, dtype, at(q_traj, k),
                                       dv ? at(q_half, k) : nullptr, dv, cur, oth, edges, v0,
                                       dt, order, dvbar_accum, v0bar_accum)) != RAM_OK)
                return st;
            std::swap(cur, oth);
        }
    }
    if (cur != qbar) {
        const hipError_t e = ram::launch_copy(cur, qbar, (int64_t)state_bytes, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "copy launch");
    }
    return RAM_OK;
}

ram_status ram_validate(ram_ctx *ctx, const ram_layout *layout,
                        ram_dtype dtype, const double *edges, const void *dv,
                        double dt)
{
    ram_status st;
    g_last_error.clear();
    if ((st = check_layout(layout, edges)) != RAM_OK) return st;
    if ((st = check_dtype(dtype)) != RAM_OK) return st;
    if ((st = check_dt(dt)) != RAM_OK) return st;
    if ((st = enter(ctx)) != RAM_OK) return st;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    const int64_t n_rows = layout->n_rows;
    std::vector<int64_t> rp(n_rows + 1);
    if (layout->n_cols > 0) {
        for (int64_t r = 0; r <= n_rows; ++r) rp[r] = r * layout->n_cols;
    } else {
        e = hipMemcpy(rp.data(), layout->row_ptr, sizeof(int64_t) * (n_rows + 1),
                      hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "copy row_ptr");
        for (int64_t r = 0; r < n_rows; ++r)
            if (rp[r + 1] < rp[r] + 1)
                return fail(RAM_E_INVALID_ARG, "row %lld is empty or row_ptr decreases", (long long)r);
        if (rp[0] != 0 || rp[n_rows] != layout->n_cells)
            return fail(RAM_E_INVALID_ARG, "row_ptr must start at 0 and end at n_cells");
    }
    const bool shared = layout->edges_shared != 0;
    const int64_t n_nodes = shared ? layout->n_cols + 1 : rp[n_rows] + n_rows;
    std::vector<double> x(n_nodes);
    e = hipMemcpy(x.data(), edges, sizeof(double) * n_nodes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "copy edges");
    std::vector<double> v;
    if (dv) {
        v.resize(rp[n_rows]);
        if (dtype == RAM_F64) {
            e = hipMemcpy(v.data(), dv, sizeof(double) * rp[n_rows], hipMemcpyDeviceToHost);
        } else {
            std::vector<float> vf(rp[n_rows]);
            e = hipMemcpy(vf.data(), dv, sizeof(float) * rp[n_rows], hipMemcpyDeviceToHost);
            for (size_t i = 0; i < vf.size(); ++i) v[i] = vf[i];
        }
        if (e != hipSuccess) return hip_fail(e, "copy dv");
    }
    for (int64_t r = 0; r < n_rows; ++r) {
        const int64_t n = rp[r + 1] - rp[r];
        const double *xr = shared ? x.data() : x.data() + rp[r] + r;
        for (int64_t j = 0; j <= n; ++j)
            if (!std::isfinite(xr[j]))
                return fail(RAM_E_MESH, "row %lld node %lld is not finite", (long long)r, (long long)j);
        for (int64_t j = 0; j < n; ++j)
            if (!(xr[j + 1] > xr[j]))
                return fail(RAM_E_MESH, "row %lld nodes not strictly increasing at %lld",
                            (long long)r, (long long)j);
        if (!dv) continue;
        for (int64_t f = 0; f < n; ++f) {
            const double a = std::fabs(v[rp[r] + f]);
            if (!std::isfinite(a))
                return fail(RAM_E_CFL, "row %lld face %lld: dv not finite", (long long)r, (long long)f);
            const int64_t fm = (f + n - 1) % n;
            const double lim = std::fmin(xr[f + 1] - xr[f], xr[fm + 1] - xr[fm]);
            if (a * std::fabs(dt) > lim)
                return fail(RAM_E_CFL, "row %lld face %lld: |dv| dt = %g exceeds %g",
                            (long long)r, (long long)f, a * std::fabs(dt), lim);
        }
    }
    return RAM_OK;
}

} // extern "C"
