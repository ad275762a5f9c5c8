// Wavefront-level helpers shared by the kernels (wave64).
#pragma once
#include <hip/hip_runtime.h>

namespace rbl {

// ---------------------------------------------------------------------------
// Wavefront helpers
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
// lane i receives lane i-1's value; lane 0 receives `fill`
__device__ inline double shift_up(double v, double fill, int lane) {
    const double u = __shfl_up(v, 1, 64);
    return lane == 0 ? fill : u;
}
// lane i receives lane i+1's value; lane 63 receives `fill`
__device__ inline double shift_down(double v, double fill, int lane) {
    const double u = __shfl_down(v, 1, 64);
    return lane == 63 ? fill : u;
}
__device__ inline float shift_up(float v, float fill, int lane) {
    const float u = __shfl_up(v, 1, 64);
    return lane == 0 ? fill : u;
}
__device__ inline double lane_value(double v, int src) { return __shfl(v, src, 64); }

__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

}  // namespace rbl
