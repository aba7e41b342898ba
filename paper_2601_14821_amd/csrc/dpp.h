// Cross-lane reductions for wave64 built from DPP row operations (VALU only,
// no LDS traffic). Call with all 64 lanes of the wave active.
#pragma once

#include <hip/hip_runtime.h>

namespace potr {

// value of another lane selected by a DPP control; rows outside ROW_MASK read 0
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline float dpp_read(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, ROW_MASK == 0xf));
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ inline uint32_t dpp_read_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, ROW_MASK == 0xf);
}

// Inclusive prefix sum over the 64 lanes (lane l gets the sum of lanes 0..l):
// shifts by 1, 2, 4, 8 within each row of 16, then row 0's total into row 1
// and row 2's into row 3 (row_bcast:15), then lane 31's into rows 2 and 3
// (row_bcast:31). Six VALU operations, no LDS.
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    v += dpp_read_u32<0x111>(v);        // row_shr:1
    v += dpp_read_u32<0x112>(v);        // row_shr:2
    v += dpp_read_u32<0x114>(v);        // row_shr:4
    v += dpp_read_u32<0x118>(v);        // row_shr:8
    v += dpp_read_u32<0x142, 0xa>(v);   // row_bcast:15
    v += dpp_read_u32<0x143, 0xc>(v);   // row_bcast:31
    return v;
}

// Sum over the 64 lanes, returned in every lane:
// pairs (xor 1, xor 2) -> 8-lane mirror -> 16-lane mirror -> row 0 into row 1
// and row 2 into row 3 -> rows 0..1 into rows 2..3; lane 63 then holds the total.
__device__ inline float wave_sum(float v) {
    v += dpp_read<0xB1>(v);        // quad_perm [1,0,3,2]
    v += dpp_read<0x4E>(v);        // quad_perm [2,3,0,1]
    v += dpp_read<0x141>(v);       // row_half_mirror
    v += dpp_read<0x140>(v);       // row_mirror
    v += dpp_read<0x142, 0xa>(v);  // row_bcast:15
    v += dpp_read<0x143, 0xc>(v);  // row_bcast:31
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Sums of four values v0..v3 over the 64 lanes; lane r (r < 4) returns the sum
// of v_r. Reduce-scatter: after the xor-1 exchange each lane keeps two of the
// four values (summed over its lane pair), after the xor-2 exchange one of them
// (summed over its quad, value index = lane & 3); rotations by 4 and 8 within a
// row and two cross-row exchanges then sum the 16 quads of equal index.
__device__ inline float wave_sum4(float v0, float v1, float v2, float v3) {
    const int lane = threadIdx.x & 63;
    const bool o1 = (lane & 1) != 0, o2 = (lane & 2) != 0;
    const float a = (o1 ? v1 : v0) + dpp_read<0xB1>(o1 ? v0 : v1);   // quad_perm [1,0,3,2]
    const float b = (o1 ? v3 : v2) + dpp_read<0xB1>(o1 ? v2 : v3);
    float c = (o2 ? b : a) + dpp_read<0x4E>(o2 ? a : b);             // quad_perm [2,3,0,1]
    c += dpp_read<0x124>(c);                                          // row_ror:4
    c += dpp_read<0x128>(c);                                          // row_ror:8
    c += __shfl_xor(c, 16, 64);
    c += __shfl_xor(c, 32, 64);
    return c;
}

}  // namespace potr
