// Cross-lane moves inside one wavefront with no LDS traffic: DPP moves
// within a row of 16 lanes, and the gfx950 permlane swaps across rows.  A
// cross-lane shuffle (__shfl_xor) compiles to ds_bpermute, an LDS
// instruction with the LDS latency; in the transform by F^{(x)s} of a CSFG
// check the move is on the frame's critical path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pbp {
namespace lanes {

// DPP move of v under control CTRL (a pattern inside each row of 16 lanes)
template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF,
                                                 false);
}

// v of lane i + H, in the lanes whose bit H is clear (the other lanes get
// unspecified values); H a power of two below 64
template <int H>
__device__ __forceinline__ uint32_t down_u32(uint32_t v)
{
    static_assert(H >= 1 && H <= 32 && (H & (H - 1)) == 0, "H: 1, 2, 4, ..., 32");
    if constexpr (H == 1) {
        return dpp<0xB1>(v);                        // quad_perm [1, 0, 3, 2]
    } else if constexpr (H == 2) {
        return dpp<0x4E>(v);                        // quad_perm [2, 3, 0, 1]
    } else if constexpr (H == 4) {
        return dpp<0x104>(v);                       // row_shl:4: lane i + 4
    } else if constexpr (H == 8) {
        return dpp<0x128>(v);                       // row_ror:8: lane i ^ 8
    } else if constexpr (H == 16) {
        // odd rows of the first operand swap with even rows of the second:
        // the second comes back holding row r + 1 in each even row r
        return __builtin_amdgcn_permlane16_swap(v, v, false, false)[1];
    } else {
        // rows 2 and 3 of the first operand swap with rows 0 and 1 of the
        // second: the second comes back holding lanes 32..63 in lanes 0..31
        return __builtin_amdgcn_permlane32_swap(v, v, false, false)[1];
    }
}

// The same for a distance known only after unrolling (a uniform value the
// compiler folds, else a uniform branch)
__device__ __forceinline__ uint32_t down_u32(uint32_t v, int h)
{
    switch (h) {
    case 1: return down_u32<1>(v);
    case 2: return down_u32<2>(v);
    case 4: return down_u32<4>(v);
    case 8: return down_u32<8>(v);
    case 16: return down_u32<16>(v);
    default: return down_u32<32>(v);
    }
}

// a 64-bit word of lane i + h, in the lanes whose bit h is clear
__device__ __forceinline__ uint64_t down_u64(uint64_t v, int h)
{
    const uint32_t lo = down_u32((uint32_t)v, h);
    const uint32_t hi = down_u32((uint32_t)(v >> 32), h);
    return ((uint64_t)hi << 32) | lo;
}

}  // namespace lanes
}  // namespace pbp
