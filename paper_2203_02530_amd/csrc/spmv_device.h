// Device helpers shared by the gfx950 kernels: cross-lane reductions on
// DPP row moves and the gfx950 permlane swaps, and XCD-aware tile order.
#pragma once

#include <hip/hip_runtime.h>

namespace spmv {

constexpr int kXcds = 8;   // MI355X: 8 XCDs, workgroups dispatched round-robin

// Block b of nb is dispatched to XCD b % 8.  With remap 1, XCD x processes
// the contiguous tile range [x*per + min(x, rem), ...) instead of every 8th
// tile, so x entries shared by neighbouring tiles stay in that XCD's L2.
// Remap 3 is remap 1 with the last XCD's range taken from its end, so that
// the last tiles, which hold a contiguous row block's high boundary rows,
// start first on their XCD rather than close the launch.  Bijective for
// any nb (the last XCD's range has per tiles).
__device__ __forceinline__ int tile_of_block(int b, int nb, int remap)
{
    if (remap != 1 && remap != 3) return b;
    const int xcd = b % kXcds, local = b / kXcds;
    const int per = nb / kXcds, rem = nb % kXcds;
    const int first = xcd * per + min(xcd, rem);
    if (remap == 3 && xcd == kXcds - 1) return first + per - 1 - local;
    return first + local;
}

// Block b of 8 * (longest range) blocks, for tiles given to the XCDs in
// contiguous ranges: XCD x runs [xr[x], xr[x + 1]), the last XCD from the
// end of its range as with remap 3; -1 for a block past its XCD's range.
__device__ __forceinline__ int tile_of_range(int b, const int32_t *xr)
{
    const int xcd = b % kXcds, local = b / kXcds;
    int lo = 0, hi = 0;
#pragma unroll
    for (int k = 0; k < kXcds; ++k)   // selects: xcd is uniform, no indexed kernarg
        if (k == xcd) {
            lo = xr[k];
            hi = xr[k + 1];
        }
    if (local >= hi - lo) return -1;
    return xcd == kXcds - 1 ? hi - 1 - local : lo + local;
}

template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    return __builtin_amdgcn_update_dpp(0.0, v, CTRL, 0xF, 0xF, false);
}

// v_permlane{16,32}_swap with both operands v: each lane ends up holding its
// own value and the partner's (16 or 32 lanes away), in some order; their sum
// is the xor-16 / xor-32 butterfly step.
__device__ __forceinline__ double swap_sum16(double v)
{
    const long long b = __double_as_longlong(v);
    auto lo = __builtin_amdgcn_permlane16_swap(unsigned(b), unsigned(b), false, false);
    auto hi = __builtin_amdgcn_permlane16_swap(unsigned(b >> 32), unsigned(b >> 32), false, false);
    const double a0 = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
    const double a1 = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
    return a0 + a1;
}

__device__ __forceinline__ double swap_sum32(double v)
{
    const long long b = __double_as_longlong(v);
    auto lo = __builtin_amdgcn_permlane32_swap(unsigned(b), unsigned(b), false, false);
    auto hi = __builtin_amdgcn_permlane32_swap(unsigned(b >> 32), unsigned(b >> 32), false, false);
    const double a0 = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
    const double a1 = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
    return a0 + a1;
}

// Sum over each aligned group of LPR lanes (power of two <= 64); afterwards
// every lane of the group holds the group sum.  Steps: pairs (quad_perm
// 1,0,3,2), quads (2,3,0,1), 8 lanes (row_half_mirror), 16 (row_mirror),
// 32 (permlane16 swap), 64 (permlane32 swap).  The order is fixed, so the
// result depends only on the lane values.
template <int LPR>
__device__ __forceinline__ double group_sum(double v)
{
    if constexpr (LPR >= 2) v += dpp<0xB1>(v);
    if constexpr (LPR >= 4) v += dpp<0x4E>(v);
    if constexpr (LPR >= 8) v += dpp<0x141>(v);
    if constexpr (LPR >= 16) v += dpp<0x140>(v);
    if constexpr (LPR >= 32) v = swap_sum16(v);
    if constexpr (LPR >= 64) v = swap_sum32(v);
    return v;
}

}  // namespace spmv
