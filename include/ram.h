/*
 * ram.h -- C ABI of the RAM advection library for AMD MI355X (gfx950).
 *
 * RAM (Rapid Advection Algorithm on Arbitrary Meshes) solves the advection
 * equation  dQ/dt + d(Q v)/dx = 0  with  v = v0 + dv  by operator splitting
 * (paper Section 1, Eqs. advection_bulk, splitting_first, splitting_second):
 * first an exact shift of every periodic row by s = v0*dt, evaluated as a
 * conservative remap of a piecewise reconstruction (Section 3, Steps 1-3), then
 * a standard upwind step for the residual velocity dv.
 *
 * Data model (paper Section 2):
 *   row      one periodic 1D line of N cells bounded by N+1 strictly increasing
 *            nodes x[0..N]; node N is identified with node 0 of the next
 *            period (period L = x[N] - x[0]).
 *   Q        cell averages (Eq. cellaverage_assumption), row-major, rows back
 *            to back.  FP64 or FP32 (ram_dtype).
 *   edges    node coordinates, always FP64: either one array x[0..n_cols]
 *            shared by all rows, or every row's N_r+1 nodes concatenated (row r
 *            at offset row_ptr[r] + r).
 *   v0       bulk velocity per row, FP64 [n_rows] (constant along the row,
 *            Section 1).
 *   dv       residual velocity on faces, same shape and dtype as Q: entry i of
 *            a row is the face between cells i-1 and i (periodic).
 *
 * Conventions
 *   * Every array pointer is a DEVICE pointer owned by the caller, except where
 *     a parameter says "host".  The library never frees caller memory.
 *   * Calls are asynchronous on the context's stream (ram_set_stream); errors
 *     detected on the host are returned before anything is launched, device
 *     launch errors map to RAM_E_HIP.  ram_sync waits for the stream.
 *   * Nothing throws across the ABI.  ram_last_error returns a detail message
 *     for the calling thread's most recent failure.
 *   * order (the degree p of the cumulative interpolant) must be 1, 3 or 5;
 *     every row needs N_r >= order + 1 cells.
 *   * Input and output arrays of one call must not alias.
 */
#ifndef RAM_H
#define RAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RAM_OK = 0,
    RAM_E_INVALID_ARG = -1,  /* null pointer, bad size, bad dt, aliasing      */
    RAM_E_UNSUPPORTED = -2,  /* order not in {1,3,5}, dtype/scan combination  */
    RAM_E_MESH = -3,         /* non-monotone or non-finite nodes (validate)    */
    RAM_E_CFL = -4,          /* |dv| dt exceeds an adjacent cell (validate)     */
    RAM_E_HIP = -5,          /* a HIP runtime call failed                       */
    RAM_E_NOMEM = -6         /* device scratch allocation failed                */
} ram_status;

typedef enum { RAM_F64 = 0, RAM_F32 = 1 } ram_dtype;

/* How the shift forms differences of the node cumulative C_j = sum_{m<j} M_m
 * (Eq. mass_shift_algo: whole-cell sums and partial integrals).  The prefix
 * modes build a window prefix sum and subtract; RAM_SUM_DIRECT sums the masses
 * between the two nodes instead (at most p masses for a partial integral),
 * so no prefix and no cancellation arise.  On per-row meshes RAM_SUM_DIRECT
 * uses the FP64 prefix, except on the streaming path of ram_step (below),
 * which sums directly.  FP64 state requires RAM_SCAN_F64 or RAM_SUM_DIRECT. */
typedef enum {
    RAM_SCAN_F64 = 0,         /* FP64 prefix sums                              */
    RAM_SCAN_F32_TWOSUM = 1,  /* compensated FP32 prefix (hi, lo) pairs        */
    RAM_SCAN_F32 = 2,         /* plain FP32 prefix (shows the cancellation)    */
    RAM_SUM_DIRECT = 3        /* no prefix: direct sums in the state's type    */
} ram_scan;

/* Limited (monotone) reconstructions for the bulk shift (Section 3.1; App. A):
 *   RAM_RECON_PLM  q_c(x) = Q_c + sigma_c (x - x_c), x_c the cell centre, with
 *                  the van Leer harmonic slope of the centre-gap differences;
 *   RAM_RECON_PPM  Colella & Woodward's parabola QL + xi (QR - QL) + Q6 xi (1-xi),
 *                  xi from the cell's left node, Q6 = 6 Q_c - 3 (QL + QR), with
 *                  the App. A interface values (neighbouring sizes summed in the
 *                  weights, as in Colella & Woodward's Eq. 1.6), the limited
 *                  slope (sign of the unlimited one) and the three constraints
 *                  that flatten extrema and make every parabola monotone.
 * Neither creates new extrema on a uniform mesh; both are nonlinear in Q. */
typedef enum { RAM_RECON_PLM = 1, RAM_RECON_PPM = 2 } ram_recon;

typedef struct {
    int64_t n_rows;           /* number of rows (>= 1)                          */
    int64_t n_cols;           /* > 0: every row has n_cols cells; 0: ragged     */
    const int64_t *row_ptr;   /* ragged: device, n_rows+1 cell offsets; else NULL */
    int64_t n_cells;          /* ragged: total cells, = row_ptr[n_rows] (host)  */
    int32_t edges_shared;     /* 1: one edges[n_cols+1] for every row (n_cols>0) */
} ram_layout;

typedef struct ram_ctx ram_ctx;

/* Create a context on HIP device `device`, issuing work on `stream` (a
 * hipStream_t; NULL = the null stream).  The context owns device scratch that
 * it grows on demand.  Returns RAM_E_HIP if the device cannot be selected. */
ram_status ram_create(ram_ctx **ctx, int device, void *stream);
/* Release the context and its scratch (after waiting for its stream). */
ram_status ram_destroy(ram_ctx *ctx);
/* Launch schedule of the shared-mesh step kernel.  0, the default, runs the
 * FP32 streaming kernels for every cumulative mode (tiles of 256 destination
 * cells, one a wave, four consecutive cells a lane; a tile in a uniform run
 * of the mesh is a fixed stencil on the cell values, whose cumulative
 * differences cancel exactly, so the mode governs the other tiles; rows whose
 * length is not a multiple of four, or arrays not 16-byte aligned, sum those
 * tiles' cumulative differences directly whatever the mode); FP64 runs the
 * streaming FP64 kernel on the same tile plan (every node's Lagrange weights
 * formed in FP64 from its source cell's stencil data, RAM_SCAN_F64 or
 * RAM_SUM_DIRECT; a tile whose source window exceeds 768 cells sums from
 * global memory); rows of 2^26 cells or more run the general kernel with 4
 * shifted nodes per thread instead.  In a multi-step call's captured graph
 * the FP32 step's two kernels (uniform-run tiles, searching tiles) are
 * parallel branches on a second stream of the context.  2..5 select the general
 * kernel with that many shifted nodes per thread (RAM_SUM_DIRECT; the prefix
 * modes then take 4): each workgroup of 256
 * threads shifts 256 * items_per_thread nodes, a tile of
 * 256 * items_per_thread - 1 destination cells (4 fewer when the residual
 * step is fused in).  Larger tiles mean fewer workgroups and less overlap
 * between neighbouring tiles' windows, smaller ones more waves in flight;
 * the best choice depends on the row length and the GPU, which is what an
 * autotuner measures.  Other values than 0 and 2..5 give RAM_E_UNSUPPORTED.
 * The schedule is per context and applies to later ram_shift, ram_step and
 * ram_step_record calls on shared meshes.  Every cell
 * goes through the same operations under any schedule; results agree to
 * rounding, not bit for bit (each variant is compiled on its own, and the
 * compiler may fuse multiply-adds differently in each). */
typedef struct {
    int32_t items_per_thread;
} ram_schedule;
ram_status ram_set_schedule(ram_ctx *ctx, const ram_schedule *sched);
ram_status ram_get_schedule(const ram_ctx *ctx, ram_schedule *sched);

/* Mesh-density index (paper Section 3.2.1, Eqs. index_u, norm_mesh, mesh, u;
 * the periodic bump of App. B, Eq. Inorm).  When the shared mesh was built from
 * a mesh density psi, i.e. its nodes satisfy F(x_j) = j with
 * F(x) = N int_{x_min}^{x} psi / int_{x_min}^{x_max} psi, the source cell of a
 * shifted node is floor(F(x~)), a closed form instead of a search.  After
 * ram_set_mesh_density, ram_shift / ram_step / ram_step_record on a shared mesh
 * with RAM_SUM_DIRECT and the default schedule take the cell from the closed
 * form and then check it against the nodes (stepping to the right cell if
 * F is off), so every node gets the same source cell as with the bucket index
 * for any parameters (good ones only make it cheaper); results agree with the
 * bucket-index path to rounding (a kernel variant compiled on its own, whose
 * multiply-adds may be fused differently).  NULL or RAM_DENSITY_NONE
 * switches it off.  RAM_DENSITY_PERIODIC_BUMP needs
 * xmin <= -b < -a < 0 < a < b <= xmax and c > -1: psi = 1 + c on |s| <= a,
 * 1 + c cos^2(pi/2 (|s| - a)/(b - a)) on a < |s| < b, 1 beyond. */
typedef enum { RAM_DENSITY_NONE = 0, RAM_DENSITY_PERIODIC_BUMP = 1 } ram_density_kind;
typedef struct {
    int32_t kind;
    double xmin, xmax;
    double a, b, c;
} ram_mesh_density;
ram_status ram_set_mesh_density(ram_ctx *ctx, const ram_mesh_density *density);
/* floor(F(x_i)) for m device points x (clamped to [0, n-1]), into int32 cells
 * (device), without the check against any nodes: the closed form alone. */
ram_status ram_mesh_density_cells(ram_ctx *ctx, const ram_mesh_density *density,
                                  int64_t n, const double *x, int64_t m,
                                  int32_t *cells);

/* Change the stream later calls are issued on.  The context's calls share its
 * device scratch, so the new stream first waits for everything already issued
 * on the old one (an event recorded there): calls made on different streams
 * run one after the other, in the order they were issued.  Streams under graph
 * capture take no part in that hand-off; the capturing caller orders captured
 * calls against uncaptured ones.  Setting the current stream again does
 * nothing.  Errors: RAM_E_INVALID_ARG (null context), RAM_E_HIP (the event
 * record or wait failed; the context keeps its old stream). */
ram_status ram_set_stream(ram_ctx *ctx, void *stream);
/* Wait until every call issued so far on the context's stream has finished;
 * reports asynchronous device errors as RAM_E_HIP. */
ram_status ram_sync(ram_ctx *ctx);

/* Bulk shift (paper Section 3, Steps 1-3; Eqs. Qmass_i, mass_advected,
 * condition_p, mass_shift_algo, step3): q_out = Q(x - v0[r]*dt) as the exact
 * conservative remap of the piecewise reconstruction whose cumulative is the
 * degree-`order` Lagrange interpolant of the node cumulative C_j = sum_{m<j}
 * Q_m dx_m.  dt and v0 may have any sign and size (the remap is unbounded,
 * Section 3.2).  q_in and q_out: `dtype`, n_cells each, must not alias. */
ram_status ram_shift(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                     ram_scan scan, const void *q_in, void *q_out,
                     const double *edges, const double *v0, double dt,
                     int order);
/* For callers that cannot allocate device memory (code under stream or graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * bulk shift as ram_shift, same arguments, same layouts, but its mesh tables,
 * window plan or ragged tile table live in a static device buffer of 16 MiB
 * that the library holds on each GPU it runs on until the process ends (its
 * address is looked up once per device, by ram_create).  The call allocates
 * nothing: no hipMalloc, hipFree or allocating library routine.  It always
 * runs the general shift kernels (the schedule of ram_set_schedule, 0 meaning
 * 4 nodes a thread), never the streaming FP32 kernel whose per-call plan is
 * far larger; results agree with ram_shift under the same schedule bit for
 * bit, and with the default schedule to rounding.  Layouts needing more than
 * the buffer (a shared mesh's tables take about 560 bytes a cell, so meshes
 * beyond about 29000 cells; a ragged batch's tile table 4 bytes a tile and 8
 * a row) return RAM_E_NOMEM with the required size in ram_last_error, before
 * any device work.  Every call on a GPU shares that GPU's buffer and rewrites all
 * of what it reads (nothing must start at zero): calls that overlap on one GPU
 * (other streams, other contexts, other host threads) race and must be
 * ordered by the caller. */
ram_status ram_shift_noalloc(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                             ram_scan scan, const void *q_in, void *q_out,
                             const double *edges, const double *v0, double dt, int order);

/* Residual upwind step (paper Eq. splitting_second): finite-volume update with
 * the PLM reconstruction and van Leer harmonic slope of Section 3.1; the face
 * value is the upwind profile averaged over the swept interval.  dv: faces, same
 * shape and dtype as q.  Requires |dv_f| dt <= the adjacent cell sizes for
 * stability (ram_validate checks it; this call does not). */
ram_status ram_residual(ram_ctx *ctx, const ram_layout *layout,
                        ram_dtype dtype, const void *q_in, void *q_out,
                        const double *edges, const void *dv, double dt);

/* n_steps operator-split steps (paper Section 1): shift, then residual; q is
 * updated in place (the context's scratch holds the intermediate state).
 * dv == NULL means dv = 0 (shift only).  On per-row meshes an FP32 call
 * without dv of at least 4 steps at the default schedule plans every shifted
 * node's Lagrange weights and source cell once (the shift is the same at
 * every step of a call) and then streams the steps; its scratch holds that
 * plan, about 24 bytes a cell.  Results agree with the other path to
 * rounding. */
ram_status ram_step(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                    ram_scan scan, void *q, const double *edges,
                    const double *v0, const void *dv, double dt, int order,
                    int64_t n_steps);

/* Bulk shift with a limited reconstruction (paper Section 3, Steps 1-3, with
 * Step 1 as in Section 3.1 / App. A): q_out = the conservative remap of the PLM
 * or PPM profile of q_in shifted by v0[r]*dt (any sign and size).  The whole-
 * cell masses are summed directly in `dtype` (no prefix sums); the PPM mesh
 * weights of a shared mesh are tabulated once per call.  Every row needs
 * N_r >= 4 cells (PLM) or >= 6 (PPM).  q_in and q_out: `dtype`, n_cells each,
 * must not alias.  RAM_E_UNSUPPORTED for another recon value. */
ram_status ram_shift_limited(ram_ctx *ctx, const ram_layout *layout,
                             ram_dtype dtype, ram_recon recon, const void *q_in,
                             void *q_out, const double *edges, const double *v0,
                             double dt);

/* n_steps operator-split steps (paper Section 1) with the limited shift:
 * ram_shift_limited, then (dv != NULL) ram_residual; q updated in place, the
 * context's scratch holds the intermediate state.  Loops of four or more steps
 * are captured into a graph once and replayed while the arguments match. */
ram_status ram_step_limited(ram_ctx *ctx, const ram_layout *layout,
                            ram_dtype dtype, ram_recon recon, void *q,
                            const double *edges, const double *v0,
                            const void *dv, double dt, int64_t n_steps);

/* n_steps limited steps keeping the trajectory, as ram_step_record does for
 * the Lagrange shift: q_traj holds n_steps+1 states (slot 0 the input), q_half
 * (when dv != NULL) each step's post-shift state, the state its residual step
 * read.  Results equal ram_step_limited's bit for bit. */
ram_status ram_step_limited_record(ram_ctx *ctx, const ram_layout *layout,
                                   ram_dtype dtype, ram_recon recon, void *q_traj,
                                   void *q_half, const double *edges,
                                   const double *v0, const void *dv, double dt,
                                   int64_t n_steps);

/* Adjoint of ram_shift_limited.  The limited shift is nonlinear in Q, so this
 * is the transpose of its Jacobian at the forward state q_fwd (required),
 * each limiter differentiated on the branch it takes there -- a zero slope
 * where the one-sided differences do not share a sign, as in
 * ram_residual_adjoint:
 *   qbar_in = (dS/dQ at q_fwd)^T qbar_out (overwritten),
 *   v0bar_accum[r] += dt * d<qbar_out, S(s) q_fwd>/ds at s = v0[r] dt (when
 *   non-NULL; the derivative is minus the reconstruction at each shifted
 *   node, FP64).
 * Any layout; FP64 arithmetic inside, the result rounded to dtype. */
ram_status ram_shift_limited_adjoint(ram_ctx *ctx, const ram_layout *layout,
                                     ram_dtype dtype, ram_recon recon,
                                     const void *q_fwd, const void *qbar_out,
                                     void *qbar_in, const double *edges,
                                     const double *v0, double dt,
                                     double *v0bar_accum);

/* Adjoint of one limited step Q^{n+1} = Res(ShiftLimited(Q^n)) (the
 * transposes of ram_residual_adjoint and ram_shift_limited_adjoint composed,
 * in one pass over the data on a shared mesh):
 *   qbar_in = (dS/dQ at q_fwd)^T R_q^T qbar_out (overwritten),
 *   dvbar_accum += R_dv^T qbar_out      (when non-NULL, dtype of q),
 *   v0bar_accum[r] += dt d<R^T qbar_out, S(s) q_fwd>/ds at s = v0[r] dt
 *                                        (when non-NULL, FP64).
 * q_fwd: the state the limited shift read (required); q_half: the state the
 * residual read (needed when dv != NULL; ram_step_limited_record writes it);
 * dv == NULL: the step had no residual (then this is
 * ram_shift_limited_adjoint).  Conventions at kinks as the two adjoints
 * composed.  The residual part computes in dtype; the limited shift's
 * Jacobian rows in FP64 (positions in cells, limiter branches, mesh weights),
 * accumulated in FP64 and rounded to dtype on the store.  qbar_in must not
 * alias any input. */
ram_status ram_step_limited_adjoint(ram_ctx *ctx, const ram_layout *layout,
                                    ram_dtype dtype, ram_recon recon,
                                    const void *q_fwd, const void *q_half,
                                    const void *dv, const void *qbar_out,
                                    void *qbar_in, const double *edges,
                                    const double *v0, double dt,
                                    void *dvbar_accum, double *v0bar_accum);

/* Adjoint of ram_shift: the bulk shift of paper Section 3, Steps 1-3 (Eqs.
 * Qmass_i, mass_advected, step3), is linear in Q, so qbar_in = S^T qbar_out,
 * overwritten.  When v0bar_accum != NULL, also accumulates per row
 *   v0bar_accum[r] += dt * d<qbar_out, S(s) q_fwd>/ds  at s = v0[r] dt,
 * which needs the forward input q_fwd (else q_fwd may be NULL). */
ram_status ram_shift_adjoint(ram_ctx *ctx, const ram_layout *layout,
                             ram_dtype dtype, ram_scan scan,
                             const void *q_fwd, const void *qbar_out,
                             void *qbar_in, const double *edges,
                             const double *v0, double dt, int order,
                             double *v0bar_accum);

/* Adjoint of ram_residual (the residual upwind step of paper Eq.
 * splitting_second with the van Leer slope of Section 3.1) at the forward
 * state q_fwd (the state the residual step read): qbar_in = J_q^T qbar_out (overwritten); when dvbar_accum != NULL
 * it accumulates J_dv^T qbar_out (same dtype as q).  At the limiter's kink the
 * slope derivative is taken as zero and at dv = 0 the dv >= 0 branch is used. */
ram_status ram_residual_adjoint(ram_ctx *ctx, const ram_layout *layout,
                                ram_dtype dtype, const void *q_fwd,
                                const void *dv, const void *qbar_out,
                                void *qbar_in, const double *edges, double dt,
                                void *dvbar_accum);

/* n_steps operator-split steps, keeping the trajectory (what a reverse pass
 * over the steps needs; paper Section 1 with Section 3 and Eq.
 * splitting_second).  q_traj holds n_steps+1 states of n_cells each, back to
 * back: slot 0 is the input, slot k+1 is written with step k's result.  When
 * dv != NULL, q_half (n_steps states) receives each step's state after the
 * shift, i.e. the state its residual step read; with dv == NULL it is unused
 * and may be NULL.  Results equal ram_step's bit for bit. */
ram_status ram_step_record(ram_ctx *ctx, const ram_layout *layout,
                           ram_dtype dtype, ram_scan scan, void *q_traj,
                           void *q_half, const double *edges, const double *v0,
                           const void *dv, double dt, int order, int64_t n_steps);

/* Adjoint of one step Q^{n+1} = Res(Shift(Q^n)) (the transposes of
 * ram_residual_adjoint and ram_shift_adjoint composed, in one pass over the
 * data on a shared mesh):
 *   qbar_in = S^T R_q^T qbar_out (overwritten),
 *   dvbar_accum += R_dv^T qbar_out           (when non-NULL, dtype of q),
 *   v0bar_accum[r] += dt d<R^T qbar_out, S(s) q_fwd>/ds at s = v0[r] dt
 *                                             (when non-NULL, FP64).
 * q_fwd is Q^n (needed only for v0bar), q_half the state after the shift
 * (needed when dv != NULL; ram_step_record writes it).  dv == NULL: the step
 * had no residual.  Same conventions at kinks as ram_residual_adjoint.  The
 * residual part computes in dtype; the shift part accumulates in FP64 and
 * rounds to dtype on the store (an FP32 state on a shared mesh: the
 * transposed stencil of the mesh's uniform runs sums its p+1 terms in FP32).
 * qbar_in must not alias any input. */
ram_status ram_step_adjoint(ram_ctx *ctx, const ram_layout *layout,
                            ram_dtype dtype, const void *q_fwd,
                            const void *q_half, const void *dv,
                            const void *qbar_out, void *qbar_in,
                            const double *edges, const double *v0, double dt,
                            int order, void *dvbar_accum, double *v0bar_accum);

/* The adjoint of n_steps recorded steps (ram_step_record's trajectory),
 * walked from the last step to the first: on entry qbar holds the gradient of
 * Q^{n_steps}, on return the gradient of Q^0 (overwritten), with
 * dvbar_accum and v0bar_accum accumulating every step's terms as
 * ram_step_adjoint does.  q_traj: states Q^0 .. Q^{n_steps-1} back to back
 * (n_cells each; ram_step_record's q_traj, whose last slot is not read);
 * q_half: the post-shift states of the same steps (needed when dv != NULL).
 * qbar_work: caller-owned device memory for one state (the other half of the
 * ping-pong), overwritten.  Results equal n_steps calls of ram_step_adjoint
 * bit for bit; the steps share one tile plan (the shift is the same at each),
 * which is what makes the call cheaper than those calls.  Neither qbar nor
 * qbar_work may overlap an input or each other (RAM_E_INVALID_ARG). */
ram_status ram_step_adjoint_steps(ram_ctx *ctx, const ram_layout *layout,
                                  ram_dtype dtype, const void *q_traj,
                                  const void *q_half, const void *dv, void *qbar,
                                  void *qbar_work, const double *edges,
                                  const double *v0, double dt, int order,
                                  int64_t n_steps, void *dvbar_accum,
                                  double *v0bar_accum);

/* Which path each tile of the FP32 step with RAM_SUM_DIRECT on a shared mesh
 * takes under the default schedule (tiles of 256 destination cells, one a
 * wave, row by row): RAM_TILE_WINDOW (source window staged in LDS, every shifted node
 * located by search, Eq. condition_p), RAM_TILE_UNIFORM (nodes and window in
 * one uniformly spaced run of the mesh, where the shift is one stencil on the
 * cell values, the FARGO limit of Section 4.1) or RAM_TILE_DIRECT (window
 * wider than the on-chip buffer; sums from global memory).  The tiles are
 * planned exactly as ram_step / ram_shift plan them for these arguments
 * (with_residual: the step's two-cell halo a side).  paths: device int32
 * array of at least n_tiles entries (n_tiles = n_rows * ceil(n_cols / 256)),
 * capacity `cap`; *n_tiles (host) receives the count.  RAM_E_INVALID_ARG if
 * cap is too small, RAM_E_UNSUPPORTED for layouts without a shared mesh.  For
 * tests and profiles: the step itself never needs it. */
typedef enum { RAM_TILE_WINDOW = 0, RAM_TILE_UNIFORM = 1, RAM_TILE_DIRECT = 2 } ram_tile_path;
ram_status ram_step_tile_paths(ram_ctx *ctx, const ram_layout *layout, const double *edges,
                               const double *v0, double dt, int order, int with_residual,
                               int32_t *paths, int64_t cap, int64_t *n_tiles);

/* Per-row checks of a state (not part of a step): for every row r, in FP64
 * whatever the state's dtype,
 *   out[3r]     = sum_i Q_i dx_i, the row's mass (Eq. Qmass_i summed; the
 *                 shift and the residual conserve it, Eq. qmass_total),
 *   out[3r + 1] = sum_i |Q_i - Qref_i| dx_i (0 when q_ref == NULL),
 *   out[3r + 2] = max_i |Q_i|.
 * q and q_ref: `dtype`, n_cells each; out: device, 3 * n_rows doubles.  The
 * summation order is fixed, so results are reproducible. */
ram_status ram_row_norms(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                         const void *q, const void *q_ref, const double *edges,
                         double *out);

/* Radial transport of a polar grid: the standard-upwind half of a 2D
 * dimensionally split step (paper Section 3: RAM along the direction of the
 * bulk velocity, standard transport across it).  Rows are radii bounded by
 * r_edges[0..n_rows] (FP64, device, increasing); every column (azimuthal
 * cell) is advected along r by the radial velocity u on the radial faces
 * ([n_rows + 1][n_cols], dtype; face j between rows j-1 and j) with the
 * residual's upwind scheme (PLM, van Leer slope from centre gaps,
 * swept-interval face value) in polar geometry:
 *   q'_j = q_j - dt (r_{j+1/2} F_{j+1/2} - r_{j-1/2} F_{j-1/2}) / A_j,
 *   F = u q*, A_j = (r_{j+1/2}^2 - r_{j-1/2}^2) / 2,
 * with no flux through the inner and outer edges (u there is ignored) and a
 * zero slope in the first and last rows, so sum_j A_j q_j of every column is
 * conserved.  Uniform rows (n_cols > 0, at most 65535 rows); q_in, q_out
 * must not alias.  Requires |u| dt <= the adjacent radial widths (not
 * checked). */
ram_status ram_radial_step(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                           const void *q_in, void *q_out, const double *r_edges,
                           const void *u, double dt);

/* n_steps 2D dimensionally split steps on a polar grid (Section 3), q in
 * place.  Each step: the step along the rows (the bulk shift by v0[r] dt,
 * then the residual with dv) -- ram_step's with recon = 0 (order, scan, its
 * schedule and mesh density), or ram_step_limited's with recon = PLM / PPM
 * (shared azimuthal mesh only; order and scan unused) -- then
 * ram_radial_step across the rows with u.  Arguments as for those calls;
 * loops of four or more steps are captured into a graph. */
ram_status ram_step_split2d(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                            ram_scan scan, ram_recon recon, void *q, const double *edges,
                            const double *v0, const void *dv, const double *r_edges,
                            const void *u, double dt, int order, int64_t n_steps);

/* Centre values <-> cell averages with the fourth-order correction (Section
 * 3.1: reading the state as cell averages is a second-order assumption; the
 * paper names <Q>_i = Q_i + (Q_{i+1} - 2 Q_i + Q_{i-1}) / 24 on a uniform
 * mesh).  to_centre = 0: q_in holds values at the cell centres and q_out gets
 *   <Q>_i = Q_i + dx_i^2 Q''_i / 24,
 * Q'' the three-point second derivative through the centres of cells i-1, i,
 * i+1 of the periodic row (the printed formula on a uniform mesh);
 * to_centre = 1: the inverse, Q_i = <Q>_i - dx_i^2 <Q>''_i / 24.  Both are
 * fourth-order accurate on smooth meshes; on a uniform periodic row they
 * conserve sum_i Q_i, on other meshes sum_i Q_i dx_i only to that order.  Any
 * layout; q_in and q_out must not alias. */
ram_status ram_cell_average(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                            const void *q_in, void *q_out, const double *edges,
                            int to_centre);

/* n_steps on a state of cell-centre values, q in place: each step converts
 * the values to cell averages (ram_cell_average), takes the split step
 * (recon = 0: ram_step's, with order and scan; RAM_RECON_PLM / _PPM:
 * ram_step_limited's, shared meshes only), and converts back.  This lifts
 * the second-order cap that taking centre values as averages puts on the
 * shift of smooth data on non-uniform meshes.  Between two steps the
 * conversion back and the next conversion to averages run as one pass (the
 * centre values in between are not stored), so results agree with n single
 * calls to rounding.  Loops of four or more steps are captured into a
 * graph. */
ram_status ram_step_point4(ram_ctx *ctx, const ram_layout *layout, ram_dtype dtype,
                           ram_scan scan, ram_recon recon, void *q, const double *edges,
                           const double *v0, const void *dv, double dt, int order,
                           int64_t n_steps);

/* Host-side check of the inputs (synchronous; copies to the host): strictly
 * increasing finite nodes (RAM_E_MESH; the mesh of paper Section 2), and when
 * dv != NULL the residual Courant condition |dv_f| dt <= min(dx_{f-1}, dx_f)
 * (RAM_E_CFL: information carried by the residual moves less than the
 * smaller neighbouring cell in a step, the limit the paper's Section 1
 * describes for upwind fluxes and Eq. cfl's advective terms apply). */
ram_status ram_validate(ram_ctx *ctx, const ram_layout *layout,
                        ram_dtype dtype, const double *edges, const void *dv,
                        double dt);

/* Static description of a status code. */
const char *ram_status_string(ram_status status);
/* Detail of the calling thread's last failure ("" when none). */
const char *ram_last_error(void);
/* Library version string. */
const char *ram_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RAM_H */
