// Unit phasors exp(-2 pi i phi) in FP64 from a kPhasorN-entry table held in LDS (shared by
// the likelihood kernels and the summary pass).
#pragma once
#include <hip/hip_runtime.h>

#include "rbl_internal.h"

namespace rbl {

// Unit phasor u = exp(-2 pi i phi) for a phase in revolutions.
//
// The walks carry phases in table units y = N phi, N = kPhasorN (an exact power-of-two
// scaling of revolutions).  FP64: y = k + t, k = rint(y), |t| <= 1/2, so
// exp(2 pi i phi) = E_k exp(2 pi i t / N) with E_k = exp(2 pi i k / N) from the table.  The
// rotation angle a = 2 pi t / N is at most pi / N = 0.0061: sin a to degree 5 and cos a
// to degree 4 of their Taylor series leave truncation errors below 1e-19 and 8e-17.
// k mod N is read from the low mantissa bits of y + 1.5 * 2^52, which holds rint(y) in its
// last place for |y| < 2^51; y - k is exact.
namespace phasor_detail {
constexpr double kW = 2.0 * 3.14159265358979323846 / kPhasorN;
constexpr double kS0 = kW, kS1 = -kW * kW * kW / 6.0, kS2 = kW * kW * kW * kW * kW / 120.0;
constexpr double kC1 = -kW * kW / 2.0, kC2 = kW * kW * kW * kW / 24.0;
constexpr double kMagic = 6755399441055744.0;  // 1.5 * 2^52
}  // namespace phasor_detail

__device__ inline void unit_phasor(double y, const double2* tab, double& c, double& s) {
    using namespace phasor_detail;
    const double m = y + kMagic;
    const double k = m - kMagic;
    const double t = y - k;
    const double2 e = tab[(unsigned)__double2loint(m) & (unsigned)(kPhasorN - 1)];
    const double t2 = t * t;
    const double sa = fma(fma(kS2, t2, kS1), t2, kS0) * t;
    const double ca = fma(fma(kC2, t2, kC1), t2, 1.0);
    c = fma(e.x, ca, -(e.y * sa));
    s = -fma(e.y, ca, e.x * sa);
}
// The table (cos, sin)(2 pi k / kPhasorN), copied into LDS by every workgroup that uses it.
__device__ inline void load_phasor_table(const double* src_pairs, double2* tab) {
    const double2* src = reinterpret_cast<const double2*>(src_pairs);
    for (int i = threadIdx.x; i < kPhasorN; i += blockDim.x) tab[i] = src[i];
    __syncthreads();
}

}  // namespace rbl
