// IMRPhenomD_NRTidalv2-structured waveform on the device (Sec. II B of the paper names
// the model; its calibration tables are not available, so the coefficients follow the
// stated rules below).
//
// Point-particle phase, piecewise in Mf = M f (M total mass in seconds):
//   Mf < 0.018        TaylorF2 point particle with aligned spins (no tidal terms);
//   0.018 <= Mf < f2  (b0 + b1 Mf + b2 ln Mf - b3 / (3 Mf^3)) / eta, b0..b3 matching the
//                     inspiral phase and its first three Mf-derivatives at 0.018;
//   Mf >= f2          (a0 + a1 Mf - a2 / Mf + 4/3 a3 Mf^(3/4)) / eta, a0..a3 matching the
//                     intermediate phase and its first three derivatives at f2 = f_RD / 2.
// Ringdown: final spin of Barausse & Rezzolla (2009), radiated energy (1 - sqrt(8/9)) eta,
// l = m = 2 quasinormal fits of Berti, Cardoso & Will (2006), f_damp = f_RD / (2 Q).
// Tidal phase (NRTidal Pade form), x = (pi Mf)^(2/3), kappa = 3/16 of the paper's
// Eq. (8) Lambda-tilde:  Psi_T = -(39/16) kappa / (X1 X2) x^(5/2) N(x) / D(x).
// Amplitude: A_0PN(f) (a_pp + a_T) w(f); a_pp = 1 below f_peak = f_RD - f_damp and
// exp(-(Mf - f_peak) / f_damp) above; a_T = -9 kappa x^5 (1 + 449/108 x + 22672/9 x^2.89)
// / (1 + 13477.8 x^4); w the Planck taper from f_merger to 1.2 f_merger with
// M f_merger = 0.3586/(2 pi) sqrt(X_min/X_max) (1 + 3.354e-2 k + 4.315e-5 k^2)
// / (1 + 7.542e-2 k + 2.236e-4 k^2).
// The fit constants are restated from the publications named above (the NRTidalv2 Pade and
// amplitude fits: Dietrich, Samajdar, Khan et al. 2019; the merger frequency: Dietrich,
// Bernuzzi & Tichy 2017); with no calibration tables at hand this is a structural stand-in
// of IMRPhenomD_NRTidalv2 whose agreement with the published model is not established.
#pragma once
#include "rbl_physics.h"

namespace rbl {

constexpr double kNrtF1 = 0.018;
// PN tidal series 1 + c1 x + c32 x^1.5 + c2 x^2 + c52 x^2.5 and the Pade fit (n52, n3, d1, d2)
constexpr double kTc1 = 3115.0 / 1248.0;
constexpr double kTc32 = -kPi;
constexpr double kTc2 = 28024205.0 / 3302208.0;
constexpr double kTc52 = -4283.0 * kPi / 1092.0;
constexpr double kTn52 = 312.48173;
constexpr double kTn3 = -342.15498;
constexpr double kTd1 = -20.2372;
constexpr double kTd2 = -5.36163;
constexpr double kTd32 = (kTn52 - kTc52 - kTc32 * kTd1) / kTc1;
constexpr double kTn1 = kTc1 + kTd1;
constexpr double kTn32 = kTc32 + kTd32;
constexpr double kTn2 = kTc2 + kTc1 * kTd1 + kTd2;

template <class T>
struct NrtParams {
    T ms, lnms, s, lns;   // M Tsun [s], its log, s = (pi M Tsun)^(1/3), ln s
    T c[8];               // inspiral: TaylorF2 point-particle coefficients of x^-5 .. x^2 (x = f^(1/3)) [rev]
    T cconst;             // inspiral constant [rev]
    T b[4];               // intermediate coefficients / (2 pi eta) [rev]
    T a[4];               // merger-ringdown coefficients / (2 pi eta) [rev]
    T f2;                 // intermediate / merger-ringdown boundary (Mf)
    T tp;                 // tidal phase prefactor -(39/16) kappa / (X1 X2) / (2 pi) [rev]
    T m9k;                // -9 kappa
    T fpk, fdp;           // amplitude peak and damping frequency (Mf)
    T fm;                 // taper start [Hz]
    T amp;                // 0PN amplitude scale (see tf2_amp)
    T s578;               // exp(5.78 ln s) = s^5.78: with the edge table x^5.78 it gives xt^2.89
};
constexpr int kNrtParams = 29;  // doubles in NrtParams<double>
static_assert(sizeof(NrtParams<double>) == kNrtParams * sizeof(double), "NrtParams layout");

namespace nrt_detail {
// d^n/dx^n x^p = F(p, n) x^(p - n);  d^n/dx^n (x^p ln x) = x^(p - n) (F(p, n) ln x + G(p, n))
constexpr double F(double p, int n) { return n == 0 ? 1.0 : (p - (n - 1)) * F(p, n - 1); }
constexpr double binom(int n, int k) { return k == 0 ? 1.0 : binom(n, k - 1) * (n - k + 1) / k; }
constexpr double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }
constexpr double G(double p, int n) {
    double s = 0.0;
    for (int k = 1; k <= n; ++k) s += binom(n, k) * F(p, n - k) * ((k - 1) % 2 ? -1.0 : 1.0) * fact(k - 1);
    return s;
}
// The inspiral phase terms used in the matching: PN orders k = 0, 2..7 (p_k = (k - 5) / 3).
constexpr int kMatchK[7] = {0, 2, 3, 4, 5, 6, 7};
struct FGTable {
    double F[7][4], G[7][4];
};
constexpr FGTable make_fg() {
    FGTable t{};
    for (int i = 0; i < 7; ++i)
        for (int n = 0; n < 4; ++n) {
            const double p = (kMatchK[i] - 5) / 3.0;
            t.F[i][n] = F(p, n);
            t.G[i][n] = G(p, n);
        }
    return t;
}
constexpr FGTable kFG = make_fg();
}  // namespace nrt_detail

// Parameter-independent powers used by the phase matching at Mf = 0.018, computed once on
// the host: pi^(p_k), X^(p_k - n) with X = 0.018, ln X and ln(pi) / 3.
struct NrtConsts {
    double pip[7];
    double xp[7][4];
    double lX, lpi3;
};
__host__ inline NrtConsts nrt_consts() {
    NrtConsts c{};
    for (int i = 0; i < 7; ++i) {
        const double p = (nrt_detail::kMatchK[i] - 5) / 3.0;
        c.pip[i] = std::pow(kPi, p);
        for (int n = 0; n < 4; ++n) c.xp[i][n] = std::pow(kNrtF1, p - n);
    }
    c.lX = std::log(kNrtF1);
    c.lpi3 = std::log(kPi) / 3.0;
    return c;
}

template <class T>
__device__ inline void nrt_params(const T& mc, const T& q, const T& chi1, const T& chi2, const T& lam1,
                                  const T& lam2, const NrtConsts& nc, NrtParams<T>& o) {
    using namespace nrt_detail;
    Tf2Pn<T> pn;
    const T zero(0.0);
    tf2_pn<T>(mc, q, chi1, chi2, zero, zero, pn);
    const T eta = pn.eta, x1 = pn.x1, x2 = pn.x2;
    o.ms = pn.mtot * kTsun;
    o.lnms = dlog(o.ms);
    o.lns = (log(kPi) + o.lnms) * (1.0 / 3.0);
    o.s = dexp(o.lns);
    // inspiral basis coefficients (as in tf2_coeffs, without the tidal terms)
    {
        const T s = o.s, ls = o.lns;
        const T s2 = s * s, s3 = s2 * s, s5 = s3 * s2;
        const T P = (3.0 / (128.0 * 2.0 * kPi)) / eta;
        o.c[0] = P / s5;
        o.c[1] = P * pn.p[2] / s3;
        o.c[2] = P * pn.p[3] / s2;
        o.c[3] = P * pn.p[4] / s;
        o.c[4] = P * pn.l5;
        o.c[5] = P * (pn.p[6] + kTf2L6 * ls) * s;
        o.c[6] = P * (kTf2L6 * s);
        o.c[7] = P * pn.p[7] * s2;
        o.cconst = P * (pn.p[5] + pn.l5 * ls) - 0.125;
    }
    // eta times the inspiral phase [rad] and its Mf-derivatives at F1, from the power form
    // Psi = -pi/4 + sum_k (A_k + B_k ln Mf) Mf^p_k, p_k = (k-5)/3
    const double X = kNrtF1, lX = nc.lX;
    T y[4];
    {
        const T P3 = 3.0 / 128.0;  // eta * 3 / (128 eta)
        const double lpi3 = nc.lpi3;
        for (int n = 0; n < 4; ++n) y[n] = T(n == 0 ? -0.25 * kPi : 0.0) * eta;
#pragma unroll
        for (int i = 0; i < 7; ++i) {
            const int k = kMatchK[i];
            const double pip = nc.pip[i];
            T A = P3 * pn.p[k] * pip;
            T Bc = T(0.0);
            if (k == 5) {
                A = A + P3 * pn.l5 * (lpi3 * pip);
                Bc = P3 * pn.l5 * (pip / 3.0);
            } else if (k == 6) {
                A = A + P3 * (kTf2L6 * lpi3 * pip);
                Bc = T(P3 * (kTf2L6 * pip / 3.0));
            }
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const double xp = nc.xp[i][n];
                const double Fn = kFG.F[i][n], Gn = kFG.G[i][n];
                y[n] = y[n] + (A * Fn + Bc * (Fn * lX + Gn)) * xp;
            }
        }
    }
    const double X3 = X * X * X;
    const T b3 = X3 * X3 * (y[3] + 2.0 * y[2] / X) / 12.0;
    const T b2 = -X * X * y[2] - 4.0 * b3 / X3;
    const T b1 = y[1] - b2 / X - b3 / (X3 * X);
    const T b0 = y[0] - b1 * X - b2 * lX + b3 / (3.0 * X3);
    // ringdown frequencies
    const T q2 = q * q;
    const T chit = (chi1 + q2 * chi2) / (1.0 + q2);
    const T e2 = eta * eta;
    const T af = chit - 0.1229 * chit * chit * eta + 0.4537 * chit * e2 - 2.8904 * chit * eta
               + 2.0 * sqrt(3.0) * eta - 3.5171 * e2 + 2.5763 * e2 * eta;
    const T erad = (1.0 - sqrt(8.0 / 9.0)) * eta;
    const T l1a = dlog(1.0 - af);
    const T om = 1.5251 - 1.1568 * dexp(0.1292 * l1a);
    const T qf = 0.7 + 1.4187 * dexp(-0.4990 * l1a);
    const T frd = om / ((2.0 * kPi) * (1.0 - erad));
    const T fdamp = frd / (2.0 * qf);
    const T f2 = 0.5 * frd;
    o.f2 = f2;
    // merger-ringdown coefficients from the intermediate form at f2
    const T lf2 = dlog(f2);
    const T i2 = 1.0 / f2;
    const T i3 = i2 * i2 * i2;
    const T Y0 = b0 + b1 * f2 + b2 * lf2 - b3 * i3 / 3.0;
    const T Y1 = b1 + b2 * i2 + b3 * i3 * i2;
    const T Y2 = -b2 * i2 * i2 - 4.0 * b3 * i3 * i2 * i2;
    const T Y3 = 2.0 * b2 * i3 + 20.0 * b3 * i3 * i3;
    const T a3 = -(16.0 / 7.0) * dexp(2.25 * lf2) * (Y3 + 3.0 * Y2 * i2);
    const T a2 = -0.5 * f2 * f2 * f2 * (Y2 + 0.25 * a3 * dexp(-1.25 * lf2));
    const T a1 = Y1 - a2 * i2 * i2 - a3 * dexp(-0.25 * lf2);
    const T a0 = Y0 - a1 * f2 + a2 * i2 - (4.0 / 3.0) * a3 * dexp(0.75 * lf2);
    const T g = 1.0 / ((2.0 * kPi) * eta);
    o.b[0] = b0 * g; o.b[1] = b1 * g; o.b[2] = b2 * g; o.b[3] = b3 * g;
    o.a[0] = a0 * g; o.a[1] = a1 * g; o.a[2] = a2 * g; o.a[3] = a3 * g;
    // tides
    const T kappa = (3.0 / 13.0) * ((x1 + 12.0 * x2) * (x1 * x1) * (x1 * x1) * lam1 +
                                    (x2 + 12.0 * x1) * (x2 * x2) * (x2 * x2) * lam2);
    o.tp = (-(39.0 / 16.0) / (2.0 * kPi)) * kappa / (x1 * x2);
    o.m9k = -9.0 * kappa;
    o.fpk = frd - fdamp;
    o.fdp = fdamp;
    const T ratio = (val(x1) >= val(x2)) ? x2 / x1 : x1 / x2;
    const T mfm = (0.3586 / (2.0 * kPi)) * dsqrt(ratio) * (1.0 + 3.354e-2 * kappa + 4.315e-5 * kappa * kappa) /
                  (1.0 + 7.542e-2 * kappa + 2.236e-4 * kappa * kappa);
    o.fm = mfm / o.ms;
    o.amp = tf2_amp<T>(mc);
    o.s578 = dexp(5.78 * o.lns);
}

// Quotients of one edge that the adjoint reuses: num/den and 1/den of the tidal phase,
// 1/(1 + 13477.8 xt^4) of the tidal amplitude.
struct NrtShared {
    double rat, iden, idd;
};

// Phase [rev] and amplitude factor a = (a_pp + a_T) w at one frequency, given
// x = f^(1/3), 1/x, ln x and x^5.78 (so that (s x)^5.78 = s578 x^5.78 needs no exp).
__device__ inline void nrt_node(const NrtParams<double>& p, double f, double x, double ix, double lx, double x578,
                                bool taper, double& phi, double& a, NrtShared* sh = nullptr) {
    const double mf = p.ms * f;
    double ph;
    if (mf < kNrtF1) {
        const double ix2 = ix * ix, ix3 = ix2 * ix;
        ph = p.cconst + p.c[0] * (ix3 * ix2) + p.c[1] * ix3 + p.c[2] * ix2 + p.c[3] * ix + p.c[4] * lx
           + p.c[5] * x + p.c[6] * (x * lx) + p.c[7] * (x * x);
    } else {
        const double lnmf = p.lnms + 3.0 * lx;
        if (mf < p.f2) {
            const double im = rcp_nr(mf);
            ph = p.b[0] + p.b[1] * mf + p.b[2] * lnmf - p.b[3] * (im * im * im) * (1.0 / 3.0);
        } else {
            ph = p.a[0] + p.a[1] * mf - p.a[2] * rcp_nr(mf) + (4.0 / 3.0) * p.a[3] * exp(0.75 * lnmf);
        }
    }
    const double sx = p.s * x;
    const double xt = sx * sx;
    const double xt2 = xt * xt;
    const double num = 1.0 + kTn1 * xt + kTn32 * xt * sx + kTn2 * xt2 + kTn52 * xt2 * sx + kTn3 * xt2 * xt;
    const double den = 1.0 + kTd1 * xt + kTd32 * xt * sx + kTd2 * xt2;
    const double iden = rcp_nr(den);
    const double rat = num * iden;
    phi = ph + p.tp * xt2 * sx * rat;
    const double app = mf < p.fpk ? 1.0 : exp(-(mf - p.fpk) * rcp_nr(p.fdp));
    const double idd = rcp_nr(1.0 + 13477.8 * xt2 * xt2);
    const double at = p.m9k * (xt2 * xt2 * xt) * (1.0 + (449.0 / 108.0) * xt + (22672.0 / 9.0) * (p.s578 * x578)) * idd;
    a = app + at;
    if (sh) *sh = NrtShared{rat, iden, idd};
    if (taper) {
        const double fe = 1.2 * p.fm;
        if (f >= fe) {
            a = 0.0;
        } else if (f > p.fm) {
            const double wd = fe - p.fm;
            double z = wd * rcp_nr(f - p.fm) + wd * rcp_nr(f - fe);
            z = fmin(fmax(z, -700.0), 700.0);
            a *= 1.0 - rcp_nr(exp(z) + 1.0);
        }
    }
}

// Adjoint of one edge: acc[k] += gphi dPhi/dp_k + ga da/dp_k for the node parameters
// p_k in the order of NrtParams without f2 and amp (kNrtAdj of them; index k is field k
// for k < kNrtAdjSkip and field k + 1 above).  gphi = d lnL / dPhi [per revolution],
// ga = d lnL / da.  The region and taper branches are taken as in nrt_node; derivatives
// of the branch conditions are zero almost everywhere.
constexpr int kNrtAdj = 26;
constexpr int kNrtAdjSkip = 21;  // f2
constexpr int kAdjMs = 0, kAdjLnMs = 1, kAdjS = 2, kAdjLnS = 3, kAdjC = 4, kAdjCc = 12, kAdjB = 13, kAdjA = 17,
              kAdjTp = 21, kAdjM9k = 22, kAdjFpk = 23, kAdjFdp = 24, kAdjFm = 25;

__device__ inline void nrt_node_adjoint(const NrtParams<double>& p, double f, double x, double ix, double lx,
                                        double x578, const NrtShared& sh, double gphi, double ga, double* acc) {
    const double mf = p.ms * f;
    if (mf < kNrtF1) {
        const double ix2 = ix * ix, ix3 = ix2 * ix;
        acc[kAdjC + 0] = fma(gphi, ix3 * ix2, acc[kAdjC + 0]);
        acc[kAdjC + 1] = fma(gphi, ix3, acc[kAdjC + 1]);
        acc[kAdjC + 2] = fma(gphi, ix2, acc[kAdjC + 2]);
        acc[kAdjC + 3] = fma(gphi, ix, acc[kAdjC + 3]);
        acc[kAdjC + 4] = fma(gphi, lx, acc[kAdjC + 4]);
        acc[kAdjC + 5] = fma(gphi, x, acc[kAdjC + 5]);
        acc[kAdjC + 6] = fma(gphi, x * lx, acc[kAdjC + 6]);
        acc[kAdjC + 7] = fma(gphi, x * x, acc[kAdjC + 7]);
        acc[kAdjCc] += gphi;
    } else {
        const double lnmf = p.lnms + 3.0 * lx;
        const double im = rcp_nr(mf);
        if (mf < p.f2) {
            const double im3 = im * im * im;
            acc[kAdjB + 0] += gphi;
            acc[kAdjB + 1] = fma(gphi, mf, acc[kAdjB + 1]);
            acc[kAdjB + 2] = fma(gphi, lnmf, acc[kAdjB + 2]);
            acc[kAdjB + 3] = fma(gphi, -(1.0 / 3.0) * im3, acc[kAdjB + 3]);
            acc[kAdjMs] = fma(gphi, f * (p.b[1] + p.b[3] * (im3 * im)), acc[kAdjMs]);
            acc[kAdjLnMs] = fma(gphi, p.b[2], acc[kAdjLnMs]);
        } else {
            const double e = exp(0.75 * lnmf);
            acc[kAdjA + 0] += gphi;
            acc[kAdjA + 1] = fma(gphi, mf, acc[kAdjA + 1]);
            acc[kAdjA + 2] = fma(gphi, -im, acc[kAdjA + 2]);
            acc[kAdjA + 3] = fma(gphi, (4.0 / 3.0) * e, acc[kAdjA + 3]);
            acc[kAdjMs] = fma(gphi, f * (p.a[1] + p.a[2] * (im * im)), acc[kAdjMs]);
            acc[kAdjLnMs] = fma(gphi, p.a[3] * e, acc[kAdjLnMs]);
        }
    }
    // tidal phase tp sx^5 N(sx) / D(sx), sx = s x
    const double sx = p.s * x;
    const double xt = sx * sx;
    const double xt2 = xt * xt;
    const double sx5 = xt2 * sx;
    const double dnum = sx * (2.0 * kTn1 + 3.0 * kTn32 * sx + 4.0 * kTn2 * xt + 5.0 * kTn52 * xt * sx + 6.0 * kTn3 * xt2);
    const double dden = sx * (2.0 * kTd1 + 3.0 * kTd32 * sx + 4.0 * kTd2 * xt);
    const double rat = sh.rat;
    acc[kAdjTp] = fma(gphi, sx5 * rat, acc[kAdjTp]);
    const double dtid = p.tp * (5.0 * xt2 * rat + sx5 * (dnum - rat * dden) * sh.iden);  // d tidal / d sx
    double gs = gphi * dtid * x;                                                      // -> d / ds
    // amplitude a = (a_pp + a_T) w
    double w = 1.0, dw = 0.0;  // taper and its derivative with respect to f_merger
    const double fe = 1.2 * p.fm;
    if (f >= fe) {
        w = 0.0;
    } else if (f > p.fm) {
        const double wd = fe - p.fm;
        const double u1 = rcp_nr(f - p.fm), u2 = rcp_nr(f - fe);
        double z = wd * u1 + wd * u2;
        const bool clip = z > 700.0 || z < -700.0;
        z = fmin(fmax(z, -700.0), 700.0);
        const double ez = exp(z);
        w = 1.0 - rcp_nr(ez + 1.0);
        if (!clip) {
            const double dz = 0.2 * u1 + wd * u1 * u1 + 0.2 * u2 + 1.2 * wd * u2 * u2;
            dw = w * (1.0 - w) * dz;
        }
    }
    const double gA = ga * w;  // d lnL / d(a_pp + a_T)
    double app = 1.0;
    if (mf >= p.fpk) {
        const double id = rcp_nr(p.fdp);
        app = exp(-(mf - p.fpk) * id);
        const double g = gA * app * id;
        acc[kAdjMs] = fma(-g, f, acc[kAdjMs]);
        acc[kAdjFpk] += g;
        acc[kAdjFdp] = fma(g, (mf - p.fpk) * id, acc[kAdjFdp]);
    }
    const double e289 = p.s578 * x578;  // xt^2.89
    const double xt4 = xt2 * xt2;
    const double nn = 1.0 + (449.0 / 108.0) * xt + (22672.0 / 9.0) * e289;
    const double idd = sh.idd;
    const double base = xt4 * xt * nn * idd;  // a_T / m9k
    acc[kAdjM9k] = fma(gA, base, acc[kAdjM9k]);
    const double dat_dxt = p.m9k * (5.0 * xt4 * nn * idd + xt4 * xt * ((449.0 / 108.0) - nn * idd * (4.0 * 13477.8) * xt2 * xt) * idd);
    gs = fma(gA * dat_dxt, 2.0 * sx * x, gs);
    acc[kAdjS] += gs;
    acc[kAdjLnS] = fma(gA, p.m9k * xt4 * xt * (22672.0 / 9.0) * 2.89 * e289 * idd * 2.0, acc[kAdjLnS]);
    const double at = p.m9k * base;
    acc[kAdjFm] = fma(ga * (app + at), dw, acc[kAdjFm]);
}

}  // namespace rbl
