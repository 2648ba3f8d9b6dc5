// rt_wave.hpp -- wavefront sums by DPP moves (device code only).
#pragma once

#include <hip/hip_runtime.h>

namespace rtk {

// Sum of v over aligned groups of `width` lanes (a power of two <= 64), all
// by DPP moves, every lane of the wavefront taking part, in a fixed order.
// Within a 16-lane row the lanes 1, 2, 4, 8 apart are paired (quad permutes
// and the row mirrors, which pair the same sets), so every lane of a group of
// up to 16 holds its sum; a 32-lane group adds row 0's sum into row 1 (lanes
// 16..31 hold it), a 64-lane group then row 1's into row 3 (lanes 48..63).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}
// the DPP move into the rows of ROWS only (0 elsewhere)
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_rows(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double seg_sum(double v, int width)
{
    if (width > 1) v += dpp_move<0xB1>(v);        // quad_perm [1,0,3,2]
    if (width > 2) v += dpp_move<0x4E>(v);        // quad_perm [2,3,0,1]
    if (width > 4) v += dpp_move<0x141>(v);       // row_half_mirror
    if (width > 8) v += dpp_move<0x140>(v);       // row_mirror
    if (width > 16) v += dpp_rows<0x142, 0xA>(v); // row_bcast:15 into rows 1, 3
    if (width > 32) v += dpp_rows<0x143, 0xC>(v); // row_bcast:31 into rows 2, 3
    return v;
}

// Two sums over groups of W lanes (W a power of two, 8..64, fixed at compile
// time: no branches between the steps), the steps of the two interleaved.  Each
// is the same sequence of moves and additions as seg_sum(v, W), so the sums are
// bitwise those of seg_sum.
template <int W>
__device__ __forceinline__ void seg_sum2(double &u, double &v)
{
    static_assert(W >= 8 && W <= 64 && (W & (W - 1)) == 0, "group width");
    u += dpp_move<0xB1>(u);
    v += dpp_move<0xB1>(v);
    u += dpp_move<0x4E>(u);
    v += dpp_move<0x4E>(v);
    u += dpp_move<0x141>(u);
    v += dpp_move<0x141>(v);
    if constexpr (W > 8) {
        u += dpp_move<0x140>(u);
        v += dpp_move<0x140>(v);
    }
    if constexpr (W > 16) {
        u += dpp_rows<0x142, 0xA>(u);
        v += dpp_rows<0x142, 0xA>(v);
    }
    if constexpr (W > 32) {
        u += dpp_rows<0x143, 0xC>(u);
        v += dpp_rows<0x143, 0xC>(v);
    }
}

// The same with the width (8..64) known only at run time: branches between
// the steps.
__device__ __forceinline__ void seg_sum2(double &u, double &v, int width)
{
    u += dpp_move<0xB1>(u);
    v += dpp_move<0xB1>(v);
    u += dpp_move<0x4E>(u);
    v += dpp_move<0x4E>(v);
    u += dpp_move<0x141>(u);
    v += dpp_move<0x141>(v);
    if (width > 8) {
        u += dpp_move<0x140>(u);
        v += dpp_move<0x140>(v);
    }
    if (width > 16) {
        u += dpp_rows<0x142, 0xA>(u);
        v += dpp_rows<0x142, 0xA>(v);
    }
    if (width > 32) {
        u += dpp_rows<0x143, 0xC>(u);
        v += dpp_rows<0x143, 0xC>(v);
    }
}

}  // namespace rtk
