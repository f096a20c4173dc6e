// ram_internal.h -- private declarations shared by the host API and the HIP
// kernels of the RAM library (not installed, not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ram {

// Destination cells per workgroup tile, threads per workgroup, and the
// capacity (in source cells) of the LDS window that holds a tile's sources.
constexpr int kTile = 256;
constexpr int kBlock = 256;
constexpr int kWindowCap = 2048;

enum ScanMode { kScanF64 = 0, kScanTwoSum = 1, kScanF32 = 2 };

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
    const double *edges = nullptr;
    int shared = 1;                   // one node array for every row
};

struct ShiftArgs {
    Rows rows;
    const void *q_in = nullptr;
    void *q_out = nullptr;
    const double *v0 = nullptr;
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
inline int64_t ragged_tile_bound(int64_t n_cells, int64_t n_rows)
{
    return n_cells / kTile + n_rows + 1;
}

hipError_t launch_tiles_prep(const int64_t *row_ptr, int64_t n_rows,
                             int64_t *tile_ptr, int32_t *tile_row,
                             hipStream_t stream);
hipError_t launch_shift(const ShiftArgs &a, bool f64, int scan, int order,
                        hipStream_t stream);
hipError_t launch_residual(const ResidualArgs &a, bool f64,
                           hipStream_t stream);
hipError_t launch_shift_adjoint(const ShiftAdjArgs &a, bool f64, int order,
                                hipStream_t stream);
hipError_t launch_residual_adjoint(const ResidualAdjArgs &a, bool f64,
                                   hipStream_t stream);
hipError_t launch_copy(const void *src, void *dst, int64_t bytes,
                       hipStream_t stream);

} // namespace ram
