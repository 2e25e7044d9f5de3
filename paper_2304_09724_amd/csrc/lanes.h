// lanes.h -- neighbour exchange inside a 64-lane wave without the LDS path
// (device code only).
//
// The DPP wavefront shifts of the GFX9 family move a 32-bit value one lane up
// ("wave_shr:1": lane l receives lane l - 1) or down ("wave_shl:1": lane l
// receives lane l + 1) inside the register file.  The lane left without a
// neighbour (lane 0 up, lane 63 down) receives 0 (bound_ctrl: the hardware
// writes the zero, so no old value has to be set up first); the sweeps never
// read it.
#pragma once

#include <hip/hip_runtime.h>

namespace shw {

constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;

template <int CTRL>
__device__ __forceinline__ double lane_shift(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// the value of lane l - 1 on lane l
__device__ __forceinline__ double from_lane_below(double x) { return lane_shift<DPP_WAVE_SHR1>(x); }
// the value of lane l + 1 on lane l
__device__ __forceinline__ double from_lane_above(double x) { return lane_shift<DPP_WAVE_SHL1>(x); }

} // namespace shw
