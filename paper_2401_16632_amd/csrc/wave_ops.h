// Wave-level helpers shared by the element sweep and the block-Jacobi
// inverse: uniform-lane reads and a wave-wide argmax by DPP.
#pragma once
#include <hip/hip_runtime.h>

namespace hfr {

__device__ __forceinline__ float lane_value(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double lane_value(double x, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

// Maximum of 64-bit keys and one DPP step on them (both halves moved; lanes
// the control leaves out keep their own key)
__device__ __forceinline__ unsigned long long key_max(unsigned long long a,
                                                      unsigned long long b) {
    return a > b ? a : b;
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ unsigned long long key_dpp(unsigned long long x) {
    const int lo = int(unsigned(x)), hi = int(unsigned(x >> 32));
    const unsigned l2 = unsigned(__builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xf, false));
    const unsigned h2 = unsigned(__builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xf, false));
    return (static_cast<unsigned long long>(h2) << 32) | l2;
}
// Wave-wide sum of a double by the same DPP row operations (lanes outside
// the row mask add zero), in a fixed order; every lane gets the sum.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_or_zero(double x) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROWMASK, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_sum(double x) {
    x += dpp_or_zero<0xb1, 0xf>(x);             // quad_perm [1,0,3,2]
    x += dpp_or_zero<0x4e, 0xf>(x);             // quad_perm [2,3,0,1]
    x += dpp_or_zero<0x141, 0xf>(x);            // row_half_mirror
    x += dpp_or_zero<0x140, 0xf>(x);            // row_mirror
    x += dpp_or_zero<0x142, 0xa>(x);            // row_bcast:15 into rows 1, 3
    x += dpp_or_zero<0x143, 0xc>(x);            // row_bcast:31 into rows 2, 3
    return lane_value(x, 63);
}

// Wave-wide maximum of a 32-bit key by the same DPP row operations; the
// maximum ends in lane 63 and is returned to every lane.  Lanes the DPP
// control leaves out read 0, the identity of the unsigned maximum, so each
// step is a single v_max_u32 with a DPP source.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ unsigned key32_dpp(unsigned x) {
    return unsigned(__builtin_amdgcn_update_dpp(0, int(x), CTRL, ROWMASK, 0xf, true));
}
__device__ __forceinline__ unsigned wave_max_u32(unsigned x) {
    x = max(x, key32_dpp<0xb1, 0xf>(x));        // quad_perm [1,0,3,2]
    x = max(x, key32_dpp<0x4e, 0xf>(x));        // quad_perm [2,3,0,1]
    x = max(x, key32_dpp<0x141, 0xf>(x));       // row_half_mirror
    x = max(x, key32_dpp<0x140, 0xf>(x));       // row_mirror
    x = max(x, key32_dpp<0x142, 0xa>(x));       // row_bcast:15
    x = max(x, key32_dpp<0x143, 0xc>(x));       // row_bcast:31
    return unsigned(__builtin_amdgcn_readlane(int(x), 63));
}
// 32-bit pivot key for rows below 256: |value| (FP32 bits) with its low 8
// mantissa bits replaced by the complement of the row, so the maximum is a
// largest magnitude (to 2^-15 relative) with the lowest row; 0 means no
// nonzero candidate
__device__ __forceinline__ unsigned pivot_key32(float mag, int row) {
    const unsigned b = __float_as_uint(mag) & 0xffffff00u;
    return b ? (b | unsigned(255 - row)) : 0u;
}

// The same key, never 0 for a candidate: magnitudes whose kept bits are 0
// (zero among them) rank below every other, lowest row first, so the
// maximum is always a row; a key below 0x200 marks a zero pivot.
__device__ __forceinline__ unsigned pivot_key32z(float mag, int row) {
    const unsigned b = __float_as_uint(mag) & 0xffffff00u;
    return (b ? b : 0x100u) | unsigned(255 - row);
}

// pivot key: |value| (as FP32, order-preserving bits) above the complement
// of the row, so the maximum is the largest magnitude with the lowest row
__device__ __forceinline__ unsigned long long pivot_key(float mag, int row) {
    return (static_cast<unsigned long long>(__float_as_uint(mag)) << 32) |
           (0xffffffffu - unsigned(row));
}

}  // namespace hfr
