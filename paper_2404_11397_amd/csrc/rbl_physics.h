// Waveform physics evaluated per chain: TaylorF2 phase coefficients in a
// separable frequency basis, leading-order amplitude, and the detector
// projection (antenna patterns, geocentre delay).  Templated on the scalar
// type so the same code runs in FP64 (likelihood) and with dual numbers
// (Jacobian for the gradient).
#pragma once
#include "rbl_math.h"

namespace rbl {

// Physical constants (SI, IAU 2015 nominal solar mass parameter).
constexpr double kC = 299792458.0;
constexpr double kGMsun = 1.3271244e20;
constexpr double kTsun = kGMsun / (kC * kC * kC);   // G Msun / c^3 [s]
constexpr double kMpc = 3.085677581491367e22;        // [m]
constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;

// ---------------------------------------------------------------------------
// TaylorF2 (stationary-phase inspiral, Sec. II B of the paper).
//
// Psi_int(f) = -pi/4 + 3/(128 eta) sum_k (p_k + l_k ln v) v^(k-5)
//   over k = 0, 2..7 (3.5PN point particle, spin-orbit 1.5-3.5PN, spin-spin
//   2PN and 3PN) and k = 10, 12 (tidal 5PN and 6PN), v = (pi M Tsun f)^(1/3).
//
// With v = s x, s = (pi M Tsun)^(1/3), x = f^(1/3), ln v = ln s + ln x, the
// phase in revolutions is exactly linear in per-chain coefficients:
//   Psi_int / 2pi = c_const + sum_b c_b B_b(x),
//   B = { x^-5, x^-3, x^-2, x^-1, ln x, x, x ln x, x^2, x^5, x^7 }.
// ---------------------------------------------------------------------------
constexpr int kTf2Basis = 10;

template <class T>
struct Tf2Coeffs {
    T c[kTf2Basis];  // basis coefficients [rev]
    T c_const;       // constant part [rev]
    T amp;           // sqrt(5/24) pi^(-2/3) (Mc Tsun)^(5/6) c / Mpc  (times f^(-7/6) -> strain/Hz at 1 Mpc)
};

// Post-Newtonian ingredients of the TaylorF2 phase: the bracket coefficients p_k of
// v^k (k = 0, 2..7) with the log coefficients of k = 5, 6, and the tidal k = 10, 12.
template <class T>
struct Tf2Pn {
    T eta, x1, x2, mtot;     // symmetric mass ratio, mass fractions, total mass [Msun]
    T lmc, lmtot;            // ln Mc, ln M
    T p[8];                  // p_0 .. p_7 (p_1 = 0)
    T l5;                    // log coefficient of k = 5 (l6 is a constant)
    T p10, p12;              // tidal
};
constexpr double kTf2L6 = -6848.0 / 21.0;

template <class T>
__host__ __device__ inline void tf2_pn(const T& mc, const T& q, const T& chi1, const T& chi2, const T& lam1,
                                       const T& lam2, Tf2Pn<T>& o) {
    // Masses: eta = q/(1+q)^2, M = Mc eta^(-3/5), X1 = 1/(1+q), X2 = q/(1+q).
    const T opq = 1.0 + q;
    const T x1 = 1.0 / opq;
    const T x2 = q * x1;
    const T eta = x1 * x2;
    o.eta = eta;
    o.x1 = x1;
    o.x2 = x2;
    o.lmc = dlog(mc);
    o.lmtot = o.lmc - 0.6 * dlog(eta);
    o.mtot = dexp(o.lmtot);
    const T dm = x1 - x2;  // signed (m1 - m2)/M
    const T cs = 0.5 * (chi1 + chi2);
    const T ca = 0.5 * (chi1 - chi2);
    const T e2 = eta * eta;
    const T e3 = e2 * eta;
    const double pi2 = kPi * kPi;
    o.p[0] = T(1.0);
    o.p[1] = T(0.0);
    o.p[2] = 3715.0 / 756.0 + (55.0 / 9.0) * eta;
    o.p[3] = -16.0 * kPi + (113.0 / 3.0) * dm * ca + (113.0 / 3.0 - (76.0 / 3.0) * eta) * cs;
    o.p[4] = 15293365.0 / 508032.0 + (27145.0 / 504.0) * eta + (3085.0 / 72.0) * e2
           + (-405.0 / 8.0 + 200.0 * eta) * ca * ca - (405.0 / 4.0) * dm * ca * cs
           + (-405.0 / 8.0 + 2.5 * eta) * cs * cs;
    // 2.5PN: (1 + 3 ln(v / v_lso)) g5, v_lso = 6^(-1/2)
    const T g5 = kPi * (38645.0 / 756.0 - (65.0 / 9.0) * eta)
               - ((732985.0 / 2268.0 - (24260.0 / 81.0) * eta - (340.0 / 9.0) * e2) * cs
                  + (732985.0 / 2268.0 + (140.0 / 9.0) * eta) * dm * ca);
    const double ln_vlso = -0.5 * log(6.0);
    o.p[5] = g5 * (1.0 - 3.0 * ln_vlso);
    o.l5 = 3.0 * g5;
    o.p[6] = 11583231236531.0 / 4694215680.0 - (640.0 / 3.0) * pi2
           - (6848.0 / 21.0) * kEulerGamma - (6848.0 / 21.0) * log(4.0)
           + (-15737765635.0 / 3048192.0 + (2255.0 / 12.0) * pi2) * eta
           + (76055.0 / 1728.0) * e2 - (127825.0 / 1296.0) * e3
           + kPi * ((2270.0 / 3.0) * dm * ca + (2270.0 / 3.0 - 520.0 * eta) * cs)
           + (75515.0 / 144.0 - (8225.0 / 18.0) * eta) * dm * ca * cs
           + (75515.0 / 288.0 - (263245.0 / 252.0) * eta - 480.0 * e2) * ca * ca
           + (75515.0 / 288.0 - (232415.0 / 504.0) * eta + (1255.0 / 9.0) * e2) * cs * cs;
    o.p[7] = kPi * (77096675.0 / 254016.0 + (378515.0 / 1512.0) * eta - (74045.0 / 756.0) * e2)
           + (-25150083775.0 / 3048192.0 + (10566655595.0 / 762048.0) * eta
              - (1042165.0 / 3024.0) * e2 + (5345.0 / 36.0) * e3) * cs
           + (-25150083775.0 / 3048192.0 + (26804935.0 / 6048.0) * eta
              - (1985.0 / 48.0) * e2) * dm * ca;
    // Tidal, each body A with companion B (Vines-Flanagan-Hinderer 5PN + 6PN).
    const T x1_4 = (x1 * x1) * (x1 * x1);
    const T x2_4 = (x2 * x2) * (x2 * x2);
    o.p10 = -24.0 * ((1.0 + 11.0 * x2) * x1_4 * lam1 + (1.0 + 11.0 * x1) * x2_4 * lam2);
    o.p12 = (-5.0 / 28.0) *
            ((3179.0 - 919.0 * x1 - 2286.0 * x1 * x1 + 260.0 * x1 * x1 * x1) * x1_4 * lam1 +
             (3179.0 - 919.0 * x2 - 2286.0 * x2 * x2 + 260.0 * x2 * x2 * x2) * x2_4 * lam2);
}

template <class T>
__host__ __device__ inline T tf2_amp(const T& mc) {
    // sqrt(5/24) pi^(-2/3) (Mc Tsun)^(5/6) c/Mpc
    return dexp((5.0 / 6.0) * dlog(mc * kTsun)) * (sqrt(5.0 / 24.0) * pow(kPi, -2.0 / 3.0) * (kC / kMpc));
}

template <class T>
__host__ __device__ inline void tf2_coeffs(const T& mc, const T& q, const T& chi1, const T& chi2,
                                           const T& lam1, const T& lam2, Tf2Coeffs<T>& out) {
    Tf2Pn<T> pn;
    tf2_pn<T>(mc, q, chi1, chi2, lam1, lam2, pn);
    // v = s x: fold powers of s into the coefficients; divide by 2 pi for revolutions.
    // ln s = (ln(pi Tsun) + ln M) / 3 from the logarithms already at hand (no cube root).
    const T ls = (1.0 / 3.0) * (pn.lmtot + log(kPi * kTsun));
    const T s = dexp(ls);
    const T is = 1.0 / s;
    const T s2 = s * s;
    const T s5 = s2 * s2 * s;
    const T s7 = s5 * s2;
    const T is2 = is * is;
    const T is3 = is2 * is;
    const T P = (3.0 / (128.0 * 2.0 * kPi)) / pn.eta;
    out.c[0] = P * (is3 * is2);                // x^-5   (k = 0)
    out.c[1] = P * pn.p[2] * is3;              // x^-3   (k = 2)
    out.c[2] = P * pn.p[3] * is2;              // x^-2   (k = 3)
    out.c[3] = P * pn.p[4] * is;               // x^-1   (k = 4)
    out.c[4] = P * pn.l5;                      // ln x   (k = 5, log)
    out.c[5] = P * (pn.p[6] + kTf2L6 * ls) * s;  // x    (k = 6)
    out.c[6] = P * (kTf2L6 * s);               // x ln x (k = 6, log)
    out.c[7] = P * pn.p[7] * s2;               // x^2    (k = 7)
    out.c[8] = P * pn.p10 * s5;                // x^5    (tidal 5PN)
    out.c[9] = P * pn.p12 * s7;                // x^7    (tidal 6PN)
    out.c_const = P * (pn.p[5] + pn.l5 * ls) - 0.125;
    // tf2_amp from ln Mc: (Mc Tsun)^(5/6) = exp(5/6 (ln Mc + ln Tsun))
    out.amp = dexp((5.0 / 6.0) * (pn.lmc + log(kTsun))) * (sqrt(5.0 / 24.0) * pow(kPi, -2.0 / 3.0) * (kC / kMpc));
}

// Basis values at x = f^(1/3) given x, 1/x and ln x.
__device__ inline void tf2_basis(double x, double ix, double lx, double b[kTf2Basis]) {
    const double ix2 = ix * ix;
    const double ix3 = ix2 * ix;
    const double x2 = x * x;
    const double x5 = x2 * x2 * x;
    b[0] = ix3 * ix2;
    b[1] = ix3;
    b[2] = ix2;
    b[3] = ix;
    b[4] = lx;
    b[5] = x;
    b[6] = x * lx;
    b[7] = x2;
    b[8] = x5;
    b[9] = x5 * x2;
}

// ---------------------------------------------------------------------------
// Detector projection.  Source direction n at hour angle phi = ra - gmst and
// declination dec; polarisation axes p = cos(psi) e_th + sin(psi) e_ph,
// q = sin(psi) e_th - cos(psi) e_ph; F+ = D:(pp - qq), Fx = D:(pq + qp);
// dt = -(r . n)/c;  C = (1+cos^2 iota)/2 F+ - i cos(iota) Fx.
// ---------------------------------------------------------------------------
template <class T>
struct Proj {
    Cx<T> C;  // complex response
    T dt;     // arrival delay relative to the geocentre [s]
};

// The source frame, shared by all detectors: n, the polarisation axes p, q and cos(iota).
template <class T>
struct SkyFrame {
    T n[3], p[3], q[3], ci;
};

template <class T>
__device__ inline void sky_frame(const T& iota, const T& psi, const T& ra, const T& dec, double gmst, SkyFrame<T>& s) {
    const T ph = ra - gmst;
    T sph, cph, sd, cd, sp, cp, si, ci;
    dsincos(ph, sph, cph);
    dsincos(dec, sd, cd);
    dsincos(psi, sp, cp);
    dsincos(iota, si, ci);
    s.n[0] = cd * cph;
    s.n[1] = cd * sph;
    s.n[2] = sd;
    const T eth[3] = {sd * cph, sd * sph, -cd};
    const T eph[3] = {-sph, cph, T(0.0)};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        s.p[i] = cp * eth[i] + sp * eph[i];
        s.q[i] = sp * eth[i] - cp * eph[i];
    }
    s.ci = ci;
}

// One detector's response and delay in a source frame.
template <class T>
__device__ inline void project(const SkyFrame<T>& s, const double* D /*[9]*/, const double* r /*[3]*/, Proj<T>& out) {
    const T* p = s.p;
    const T* qv = s.q;
    // D p and D q, then the contractions.
    T Dp[3], Dq[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Dp[i] = D[3 * i + 0] * p[0] + D[3 * i + 1] * p[1] + D[3 * i + 2] * p[2];
        Dq[i] = D[3 * i + 0] * qv[0] + D[3 * i + 1] * qv[1] + D[3 * i + 2] * qv[2];
    }
    const T pDp = p[0] * Dp[0] + p[1] * Dp[1] + p[2] * Dp[2];
    const T qDq = qv[0] * Dq[0] + qv[1] * Dq[1] + qv[2] * Dq[2];
    const T pDq = p[0] * Dq[0] + p[1] * Dq[1] + p[2] * Dq[2];
    const T qDp = qv[0] * Dp[0] + qv[1] * Dp[1] + qv[2] * Dp[2];
    const T fplus = pDp - qDq;
    const T fcross = pDq + qDp;
    out.C.re = 0.5 * (1.0 + s.ci * s.ci) * fplus;
    out.C.im = -(s.ci * fcross);
    out.dt = -(r[0] * s.n[0] + r[1] * s.n[1] + r[2] * s.n[2]) / kC;
}

template <class T>
__device__ inline void project(const T& iota, const T& psi, const T& ra, const T& dec, double gmst,
                               const double* D /*[9]*/, const double* r /*[3]*/, Proj<T>& out) {
    SkyFrame<T> s;
    sky_frame(iota, psi, ra, dec, gmst, s);
    project(s, D, r, out);
}

}  // namespace rbl
