// Wavefront-level helpers shared by the kernels (wave64).
#pragma once
#include <hip/hip_runtime.h>

namespace rbl {

// ---------------------------------------------------------------------------
// Wavefront helpers
// ---------------------------------------------------------------------------
// A double moved across lanes by one DPP pattern (two 32-bit moves).  Lanes outside the
// row / bank masks, or whose source lane lies outside their row, receive +0.
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ inline double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, BANK_MASK, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, BANK_MASK, false);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront (all lanes active), returned to every lane.
// Row prefix sums by row shifts (1, 2, 3 on the input, then 4 and 8 on the partial sums),
// then the row totals are carried across rows with the row broadcasts of lanes 15 and 31;
// lane 63 ends with the total, read back as a wave-uniform value.  Fixed order, so the
// result is bitwise reproducible.
__device__ inline double wave_sum(double v) {
    double s = v + dpp_move<0x111>(v);    // row_shr:1
    s += dpp_move<0x112>(v);              // row_shr:2
    s += dpp_move<0x113>(v);              // row_shr:3
    s += dpp_move<0x114, 0xf, 0xe>(s);    // row_shr:4 into banks 1-3
    s += dpp_move<0x118, 0xf, 0xc>(s);    // row_shr:8 into banks 2-3
    s += dpp_move<0x142, 0xa, 0xf>(s);    // row_bcast:15 into rows 1 and 3
    s += dpp_move<0x143, 0xc, 0xf>(s);    // row_bcast:31 into rows 2 and 3
    const int lo = __builtin_amdgcn_readlane(__double2loint(s), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(s), 63);
    return __hiloint2double(hi, lo);
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
