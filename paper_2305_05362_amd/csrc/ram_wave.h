// ram_wave.h -- wave-level helpers of the kernels that run one tile of
// kFastTile destination cells a wave (the FP32 streaming step and its
// adjoint): LDS visibility inside a wave, DPP prefix sums, records read with
// scalar loads, tile positions.
#pragma once

#include "ram_device.h"

namespace ram {
namespace dev {

constexpr int kLanes = 64;
constexpr int kWaves = kBlock / kLanes;             // tiles per workgroup

// Every lane's LDS writes visible to the whole wave (a wave executes its LDS
// instructions in order; the fences keep the compiler from moving accesses
// across).
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int wrap1f(int j, int n) { return j < 0 ? j + n : (j >= n ? j - n : j); }

// Tile id -> row and first cell (tiles of kFastTile cells, row by row).
struct TilePos {
    int row, i0, nd;
    bool inner;          // the tile and its halo do not wrap the row
};
__device__ inline TilePos tile_pos(int tile, int n, int H)
{
    const int tpr = (n + kFastTile - 1) / kFastTile;
    TilePos p;
    p.row = tile / tpr;
    p.i0 = (tile - p.row * tpr) * kFastTile;
    p.nd = min(kFastTile, n - p.i0);
    p.inner = (p.i0 - H >= 0) && (p.i0 + p.nd + H < n);
    return p;
}

// Record i, read through the constant address space: with a wave-uniform i
// these are scalar loads (the host pass, which only checks device code, reads
// it plainly).
__device__ inline FastTile load_rec(const FastTile *rec, int i)
{
    FastTile r;
#if defined(__HIP_DEVICE_COMPILE__)
    typedef const __attribute__((address_space(4))) int32_t *CI;
    const CI c = (CI)(rec + i);
    int32_t *o = (int32_t *)&r;
#pragma unroll
    for (int k = 0; k < (int)(sizeof(FastTile) / 4); ++k) o[k] = c[k];
#else
    r = rec[i];
#endif
    return r;
}

// Wave index inside the workgroup, in a scalar register (so that what it
// selects is read with scalar loads).
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane((int)threadIdx.x / kLanes); }

// Load / store at a 32-bit byte offset from a wave-uniform base: the access
// takes the scalar-base form (base in SGPRs, one 32-bit offset a lane)
// instead of a 64-bit address formed in every lane.  The streaming kernels
// run on rows of fewer than kFastMaxCols cells, so no offset wraps.
template <class T>
__device__ __forceinline__ T ld_at(const void *base, uint32_t byte_off)
{
    return *(const T *)((const char *)base + byte_off);
}
template <class T>
__device__ __forceinline__ void st_at(void *base, uint32_t byte_off, const T &v)
{
    *(T *)((char *)base + byte_off) = v;
}

// Inclusive scan of one value a lane over the wave in DPP steps (row shifts,
// then the row-15 and row-31 broadcasts; lanes without a source read zero),
// and lane 63's value read back as a scalar.
template <class AC>
__device__ __forceinline__ typename AC::A wave_inclusive(typename AC::A inc)
{
    inc = AC::comb(AC::template dpp<kDppRowShr1, 0xf, 0xf>(inc), inc);
    inc = AC::comb(AC::template dpp<kDppRowShr2, 0xf, 0xf>(inc), inc);
    inc = AC::comb(AC::template dpp<kDppRowShr4, 0xf, 0xf>(inc), inc);
    inc = AC::comb(AC::template dpp<kDppRowShr8, 0xf, 0xf>(inc), inc);
    inc = AC::comb(AC::template dpp<kDppBcast15, 0xa, 0xf>(inc), inc);
    inc = AC::comb(AC::template dpp<kDppBcast31, 0xc, 0xf>(inc), inc);
    return inc;
}
__device__ __forceinline__ float lane63(float v)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), kLanes - 1));
}
__device__ __forceinline__ float2 lane63(float2 v) { return make_float2(lane63(v.x), lane63(v.y)); }
__device__ __forceinline__ double lane63(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), kLanes - 1);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), kLanes - 1);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Moves a small per-lane array down one slot (v[0] = v[1], ...), for loops
// over slots that are not unrolled: they read slot 0 each trip, since an
// array indexed at run time is placed in scratch memory, whose stores reach
// HBM.
template <class T, int N>
__device__ __forceinline__ void slot_down(T (&v)[N])
{
#pragma unroll
    for (int i = 0; i + 1 < N; ++i) v[i] = v[i + 1];
}

} // namespace dev
} // namespace ram
