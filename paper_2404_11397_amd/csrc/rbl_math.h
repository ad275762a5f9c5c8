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
// exp(-2 pi i phi) for a phase phi given in revolutions, FP64.
// The integer part is removed exactly (phi - rint(phi)), then sin/cos of pi*x.
// ----------------------------------------------------------------------------
__device__ inline void expm2pi_rev(double phi, double& c, double& s) {
    const double r = phi - rint(phi);
    double sn, cs;
    sincospi(2.0 * r, &sn, &cs);
    c = cs;
    s = -sn;
}

}  // namespace rbl
