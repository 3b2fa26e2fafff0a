// Wavefront-wide integer scan and sum on gfx9 DPP lane moves (no LDS traffic).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tc {

// DPP controls (GFX9): row_shr:n moves lane i-n of the same 16-lane row to lane i; row_bcast:15 adds
// lane 15 of each row to the next row, row_bcast:31 lane 31 to rows 2 and 3.  Lanes without a source
// (and rows masked off) receive `old` = 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_add(uint32_t v) {
    return v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, false);
}

// Inclusive prefix sum over the 64 lanes (every lane active).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v = dpp_add<0x111, 0xf>(v);  // row_shr:1
    v = dpp_add<0x112, 0xf>(v);  // row_shr:2
    v = dpp_add<0x114, 0xf>(v);  // row_shr:4
    v = dpp_add<0x118, 0xf>(v);  // row_shr:8
    v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Sum over the 64 lanes (every lane active), as a uniform value.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)wave_incl_scan(v), 63);
}

}  // namespace tc
