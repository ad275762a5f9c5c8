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
// The value of lane src, per lane (src may differ between lanes; two 32-bit lane permutes).
__device__ inline double lane_permute(double v, int src) {
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
    return __hiloint2double(hi, lo);
}
// A value that is the same in every lane, moved to scalar registers.
__device__ inline double uniform(double v) {
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                            __builtin_amdgcn_readfirstlane(__double2loint(v)));
}
// The value of one lane, wave-uniform.
__device__ inline double lane_read(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}
__device__ inline float lane_read(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Sums over the 64 lanes of N doubles at once (N a multiple of 4), each returned
// wave-uniform.  Two lane-exchange levels fold the values pairwise: v_permlane32_swap
// swaps the upper 32 lanes of one register with the lower 32 of another, so one add leaves
// value a's half-sums in lanes 0-31 and value b's in lanes 32-63; v_permlane16_swap does
// the same between 16-lane rows, so four values end up in the four rows of one register
// (a in row 0, c in row 1, b in row 2, d in row 3 for the quadruple a, b, c, d).  A row
// reduction by DPP row rotations (8, 4, 2, 1) then leaves each row's total in all of its
// lanes.  About 20 vector instructions per four values instead of about 150 for four
// separate reductions; fixed order, so bitwise reproducible.
__device__ inline double swap32_add(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false, false);
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ inline double swap16_add(double a, double b) {
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false, false);
    return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
template <int CTRL>
__device__ inline double dpp_rot(double v) {  // a full-row DPP pattern: every lane has a source
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <int N>
__device__ inline void wave_sum_n(const double (&v)[N], double (&out)[N]) {
    static_assert(N % 4 == 0, "wave_sum_n takes a multiple of four values");
#pragma unroll
    for (int j = 0; j < N / 4; ++j) {
        const double p = swap32_add(v[4 * j], v[4 * j + 1]);
        const double q = swap32_add(v[4 * j + 2], v[4 * j + 3]);
        double r = swap16_add(p, q);
        r += dpp_rot<0x128>(r);  // row_ror:8
        r += dpp_rot<0x124>(r);  // row_ror:4
        r += dpp_rot<0x122>(r);  // row_ror:2
        r += dpp_rot<0x121>(r);  // row_ror:1
        out[4 * j] = lane_read(r, 0);
        out[4 * j + 1] = lane_read(r, 32);
        out[4 * j + 2] = lane_read(r, 16);
        out[4 * j + 3] = lane_read(r, 48);
    }
}

// Sum over the 16 lanes of the first row (lanes 0..15; all lanes active), wave-uniform:
// the row reduction of wave_sum_n, fixed order.
__device__ inline double row0_sum(double v) {
    v += dpp_rot<0x128>(v);  // row_ror:8
    v += dpp_rot<0x124>(v);  // row_ror:4
    v += dpp_rot<0x122>(v);  // row_ror:2
    v += dpp_rot<0x121>(v);  // row_ror:1
    return lane_read(v, 0);
}

// Whole-wave shifts by one lane (DPP wave_shr:1 / wave_shl:1).  The lane without a
// source (lane 0, resp. lane 63) receives `fill`.  All lanes must be active.
template <int CTRL>
__device__ inline double wave_shift(double v, double fill) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(fill), __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(fill), __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ inline float wave_shift(float v, float fill) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(v), CTRL, 0xf, 0xf, false));
}
// lane i receives lane i-1's value; lane 0 receives `fill`
template <class R>
__device__ inline R shift_up(R v, R fill) { return wave_shift<0x138>(v, fill); }
// lane i receives lane i+1's value; lane 63 receives `fill`
template <class R>
__device__ inline R shift_down(R v, R fill) { return wave_shift<0x130>(v, fill); }
// Neighbours across steps of 64 edges, without leaving vector registers: lane i receives
// cur[i-1], lane 0 the previous step's lane 63 (rotate prev right by one, then shift);
// resp. lane i receives cur[i+1], lane 63 the next step's lane 0.
template <class R>
__device__ inline R left_neighbour(R cur, R prev) { return shift_up(cur, wave_shift<0x13C>(prev, prev)); }
template <class R>
__device__ inline R right_neighbour(R cur, R next) { return shift_down(cur, wave_shift<0x134>(next, next)); }
__device__ inline double shift_up(double v, double fill, int) { return shift_up<double>(v, fill); }
__device__ inline float shift_up(float v, float fill, int) { return shift_up<float>(v, fill); }

__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

}  // namespace rbl
