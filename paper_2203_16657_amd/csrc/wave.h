// Wavefront-level sums and scans by DPP lane moves (gfx9 row shifts and
// broadcasts, ALU-side, no LDS permute round trip).  A double moves as its
// two 32-bit halves; lanes without a source, or in rows the row mask leaves
// out, read 0.  Every lane of the wavefront must be active where these are
// called.  The order of every sum is fixed.
#pragma once

#include <hip/hip_runtime.h>

namespace cia {

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float,
                              __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf, true));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// The six lane moves of a 64-lane inclusive scan: shifts by 1, 2, 4 and 8
// within each row of 16 lanes, then the last lane of rows 0 and 2 into rows
// 1 and 3, then lane 31 into rows 2 and 3.
#define CIA_WAVE_SCAN_STEPS(STEP) \
    STEP(0x111, 0xf)              \
    STEP(0x112, 0xf)              \
    STEP(0x114, 0xf)              \
    STEP(0x118, 0xf)              \
    STEP(0x142, 0xa)              \
    STEP(0x143, 0xc)

__device__ __forceinline__ float wave_incl_scan(float x) {
#define CIA_STEP(C, M) x += dpp_f<C, M>(x);
    CIA_WAVE_SCAN_STEPS(CIA_STEP)
#undef CIA_STEP
    return x;
}
__device__ __forceinline__ double wave_incl_scan(double x) {
#define CIA_STEP(C, M) x += dpp_d<C, M>(x);
    CIA_WAVE_SCAN_STEPS(CIA_STEP)
#undef CIA_STEP
    return x;
}
__device__ __forceinline__ double2 wave_incl_scan(double2 v) {
    return make_double2(wave_incl_scan(v.x), wave_incl_scan(v.y));
}
// the value one lane down the wavefront (lane 0 reads 0): inclusive -> exclusive
__device__ __forceinline__ double2 wave_shr1(double2 v) {
    return make_double2(dpp_d<0x138, 0xf>(v.x), dpp_d<0x138, 0xf>(v.y));   // wave_shr:1
}
// lane 63's value, in every lane
__device__ __forceinline__ float lane63(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), 63));
}
__device__ __forceinline__ double lane63(double x) {
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
// wavefront sums, identical in every lane
__device__ __forceinline__ float wave_sum(float x) { return lane63(wave_incl_scan(x)); }
__device__ __forceinline__ double wave_sum(double x) { return lane63(wave_incl_scan(x)); }
__device__ __forceinline__ double2 wave_sum(double2 v) { return make_double2(wave_sum(v.x), wave_sum(v.y)); }

}  // namespace cia
