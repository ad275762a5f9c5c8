// Device math helpers: forward-mode dual numbers (for the per-chain Jacobian of
// the gradient kernel), a small complex type, and phase helpers in revolutions.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

namespace rbl {

// ----------------------------------------------------------------------------
// Dual number with N tangents.  All operations are plain FP64.
// ----------------------------------------------------------------------------
template <int N>
struct Dual {
    double v;
    double d[N];
    __host__ __device__ Dual() : v(0.0) {
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    __host__ __device__ Dual(double x) : v(x) {
#pragma unroll
        for (int i = 0; i < N; ++i) d[i] = 0.0;
    }
    static __host__ __device__ Dual var(double x, int k) {
        Dual r(x);
        r.d[k] = 1.0;
        return r;
    }
};

template <int N> __host__ __device__ inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r; r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <int N> __host__ __device__ inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r; r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <int N> __host__ __device__ inline Dual<N> operator-(const Dual<N>& a) {
    Dual<N> r; r.v = -a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <int N> __host__ __device__ inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r; r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <int N> __host__ __device__ inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
    Dual<N> r; const double inv = 1.0 / b.v; r.v = a.v * inv;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * inv;
    return r;
}
template <int N> __host__ __device__ inline Dual<N> operator+(const Dual<N>& a, double b) { Dual<N> r = a; r.v += b; return r; }
template <int N> __host__ __device__ inline Dual<N> operator+(double b, const Dual<N>& a) { return a + b; }
template <int N> __host__ __device__ inline Dual<N> operator-(const Dual<N>& a, double b) { Dual<N> r = a; r.v -= b; return r; }
template <int N> __host__ __device__ inline Dual<N> operator-(double b, const Dual<N>& a) { return (-a) + b; }
template <int N> __host__ __device__ inline Dual<N> operator*(const Dual<N>& a, double b) {
    Dual<N> r; r.v = a.v * b;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
    return r;
}
template <int N> __host__ __device__ inline Dual<N> operator*(double b, const Dual<N>& a) { return a * b; }
template <int N> __host__ __device__ inline Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N> __host__ __device__ inline Dual<N> operator/(double a, const Dual<N>& b) {
    Dual<N> r; const double inv = 1.0 / b.v; r.v = a * inv;
    const double s = -r.v * inv;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = b.d[i] * s;
    return r;
}

// Chain rule for a unary function with value fv and derivative dfv.
template <int N> __host__ __device__ inline Dual<N> lift(const Dual<N>& a, double fv, double dfv) {
    Dual<N> r; r.v = fv;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * dfv;
    return r;
}

// Scalar overloads so that templated code works for T = double and T = Dual<N>.
__host__ __device__ inline double val(double x) { return x; }

// 1/b for a finite, normal, nonzero b to about one ulp: the hardware reciprocal estimate
// refined by two Newton steps (the IEEE division sequence costs about twice as much).
__device__ inline double rcp_nr(double b) {
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    return fma(r, e, r);
}
// f^(-1/3) for a positive, normal f below 2^100, to about one ulp: a single-precision
// estimate from the hardware log2 and exp2 (relative error near 1e-6) refined by two Newton
// steps for y^-3 = f, y <- y + (y / 3)(1 - f y^3), which square the relative error each time.
__device__ inline double inv_cbrt_nr(double f) {
    const float l = __builtin_amdgcn_logf((float)f);
    double y = (double)__builtin_amdgcn_exp2f(l * (-1.0f / 3.0f));
    double e = fma(-f, y * y * y, 1.0);
    y = fma(y * (1.0 / 3.0), e, y);
    e = fma(-f, y * y * y, 1.0);
    return fma(y * (1.0 / 3.0), e, y);
}
template <int N> __host__ __device__ inline double val(const Dual<N>& x) { return x.v; }

__host__ __device__ inline double dsin(double x) { return sin(x); }
__host__ __device__ inline double dcos(double x) { return cos(x); }
__host__ __device__ inline double dexp(double x) { return exp(x); }
__host__ __device__ inline double dlog(double x) { return log(x); }
__host__ __device__ inline double dsqrt(double x) { return sqrt(x); }
__host__ __device__ inline double dcbrt(double x) { return cbrt(x); }
__host__ __device__ inline double datan(double x) { return atan(x); }
__host__ __device__ inline double dpow(double x, double p) { return pow(x, p); }

template <int N> __host__ __device__ inline Dual<N> dsin(const Dual<N>& a) { return lift(a, sin(a.v), cos(a.v)); }
template <int N> __host__ __device__ inline Dual<N> dcos(const Dual<N>& a) { return lift(a, cos(a.v), -sin(a.v)); }
template <int N> __host__ __device__ inline Dual<N> dexp(const Dual<N>& a) { const double e = exp(a.v); return lift(a, e, e); }
template <int N> __host__ __device__ inline Dual<N> dlog(const Dual<N>& a) { return lift(a, log(a.v), 1.0 / a.v); }
template <int N> __host__ __device__ inline Dual<N> dsqrt(const Dual<N>& a) { const double s = sqrt(a.v); return lift(a, s, 0.5 / s); }
template <int N> __host__ __device__ inline Dual<N> dcbrt(const Dual<N>& a) { const double c = cbrt(a.v); return lift(a, c, 1.0 / (3.0 * c * c)); }
template <int N> __host__ __device__ inline Dual<N> datan(const Dual<N>& a) { return lift(a, atan(a.v), 1.0 / (1.0 + a.v * a.v)); }
template <int N> __host__ __device__ inline Dual<N> dpow(const Dual<N>& a, double p) {
    const double pv = pow(a.v, p);
    return lift(a, pv, p * pv / a.v);
}

// ----------------------------------------------------------------------------
// Complex numbers over a real type T.
// ----------------------------------------------------------------------------
template <class T>
struct Cx {
    T re, im;
};
template <class T> __host__ __device__ inline Cx<T> cmul(const Cx<T>& a, const Cx<T>& b) {
    return Cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> __host__ __device__ inline Cx<T> cdiv(const Cx<T>& a, const Cx<T>& b) {
    const T den = b.re * b.re + b.im * b.im;
    return Cx<T>{(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
}

// ----------------------------------------------------------------------------
// cos(2 pi phi) and sin(2 pi phi) for a phase phi in revolutions, FP64.
// Reduction: y = 4 phi (exact), k = rint(y), t = y - k in [-1/2, 1/2] (exact for
// |y| < 2^52), so 2 pi phi = (pi/2) k + (pi/2) t.  On |(pi/2) t| <= pi/4 the Taylor
// series of sin to degree 15 and of cos to degree 16 are accurate to < 1e-16;
// the quadrant k mod 4 rotates the pair.
// ----------------------------------------------------------------------------
namespace detail {
constexpr double kHalfPi = 1.57079632679489661923;
constexpr double ipow(double x, int n) { return n == 0 ? 1.0 : x * ipow(x, n - 1); }
constexpr double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }
// sin((pi/2) t) = t * sum_n S_n (t^2)^n,   cos((pi/2) t) = sum_n C_n (t^2)^n  (Taylor coefficients)
constexpr double S(int n) { return ((n & 1) ? -1.0 : 1.0) * ipow(kHalfPi, 2 * n + 1) / fact(2 * n + 1); }
constexpr double C(int n) { return ((n & 1) ? -1.0 : 1.0) * ipow(kHalfPi, 2 * n) / fact(2 * n); }
constexpr double kS0 = S(0), kS1 = S(1), kS2 = S(2), kS3 = S(3), kS4 = S(4), kS5 = S(5), kS6 = S(6), kS7 = S(7);
constexpr double kC0 = C(0), kC1 = C(1), kC2 = C(2), kC3 = C(3), kC4 = C(4), kC5 = C(5), kC6 = C(6), kC7 = C(7),
                 kC8 = C(8);
}  // namespace detail

__device__ inline void sincos_rev(double phi, double& c, double& s) {
    using namespace detail;
    const double y = 4.0 * phi;
    const double k = rint(y);
    const double t = y - k;
    const double t2 = t * t;
    double ps = kS7;
    ps = fma(ps, t2, kS6);
    ps = fma(ps, t2, kS5);
    ps = fma(ps, t2, kS4);
    ps = fma(ps, t2, kS3);
    ps = fma(ps, t2, kS2);
    ps = fma(ps, t2, kS1);
    ps = fma(ps, t2, kS0);
    const double sn = ps * t;
    double pc = kC8;
    pc = fma(pc, t2, kC7);
    pc = fma(pc, t2, kC6);
    pc = fma(pc, t2, kC5);
    pc = fma(pc, t2, kC4);
    pc = fma(pc, t2, kC3);
    pc = fma(pc, t2, kC2);
    pc = fma(pc, t2, kC1);
    const double cs = fma(pc, t2, kC0);
    const int q = ((int)k) & 3;
    const double a = (q & 1) ? sn : cs;   // cos of the rotated angle, up to sign
    const double b = (q & 1) ? cs : sn;   // sin of the rotated angle, up to sign
    c = (q == 1 || q == 2) ? -a : a;
    s = (q >= 2) ? -b : b;
}

// exp(-2 pi i phi) = c + i s for a phase in revolutions.
__device__ inline void expm2pi_rev(double phi, double& c, double& s) {
    double sn, cs;
    sincos_rev(phi, cs, sn);
    c = cs;
    s = -sn;
}

// sin and cos of an angle in radians (through revolutions), for double and duals.
constexpr double kInv2Pi = 0.15915494309189533577;
__device__ inline void dsincos(double a, double& s, double& c) { sincos_rev(a * kInv2Pi, c, s); }
template <int N>
__device__ inline void dsincos(const Dual<N>& a, Dual<N>& s, Dual<N>& c) {
    double sv, cv;
    sincos_rev(a.v * kInv2Pi, cv, sv);
    s = lift(a, sv, cv);
    c = lift(a, cv, -sv);
}

}  // namespace rbl
