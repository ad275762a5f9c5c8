// HIP kernels of the relative-binned likelihood (gfx950, wave64).
//
//  k_ref_setup      reference (fiducial) constants for theta0            [1 thread]
//  k_chain_setup    per-chain record                                     [1 thread / (chain, half)]
//  k_chain_setup_grad  record and partial derivatives (dual numbers)    [1 lane / (chain, tangent)]
//  k_summary_bins   summary data of one bin                              [1 workgroup / bin]
//  k_node_tables    per-edge coefficient tables of the binned sum        [1 thread / node]
//  (k_loglike_fwd and k_loglike_grad, the likelihood kernels, are in likelihood.hip)
//  (the full-band likelihood kernels are in fullband.hip)
//  k_strain         projected strain on a grid (injections)              [1 thread / grid point]
//
// All reductions are in a fixed order, so results are bitwise reproducible.
#include "rbl_launch.h"
#include "rbl_phasor.h"
#include "rbl_wave.h"

namespace rbl {

// ---------------------------------------------------------------------------
// Reference constants
// ---------------------------------------------------------------------------
__global__ void k_ref_setup(Theta13 th, Network net, int32_t waveform, NrtConsts nc, RefConsts* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    RefConsts r{};
    const double* t = th.v;
    bool ok = t[0] > 0.0 && t[1] > 0.0 && t[6] > 0.0 && fabs(t[2]) < 1.0 && fabs(t[3]) < 1.0 &&
              t[4] >= 0.0 && t[5] >= 0.0;
    for (int i = 0; i < 13; ++i) ok = ok && isfinite(t[i]);
    r.status = ok ? 1 : 0;
    r.waveform = waveform;
    Tf2Coeffs<double> c;
    tf2_coeffs<double>(t[0], t[1], t[2], t[3], t[4], t[5], c);
    for (int b = 0; b < kTf2Basis; ++b) r.c0[b] = c.c[b];
    r.c0_const = c.c_const;
    r.amp0 = c.amp;
    if (waveform == kWfNrtv2) {
        // the edge phase is taken absolutely: no constant phase in h0fac
        nrt_params<double>(t[0], t[1], t[2], t[3], t[4], t[5], nc, r.nrt);
        r.c0_const = 0.0;
        c.c_const = 0.0;
    }
    r.mc0 = t[0];
    r.dl0 = t[6];
    r.tc0 = t[7];
    r.phic0 = t[8];
    // exp(2i phic0) exp(-2 pi i c0_const), the constant reduced to one revolution first
    const double cr = c.c_const - rint(c.c_const);
    const double ang = 2.0 * t[8] - 2.0 * kPi * cr;
    const double ce = cos(ang), se = sin(ang);
    for (int d = 0; d < net.n_det; ++d) {
        Proj<double> p;
        project<double>(t[9], t[10], t[11], t[12], net.gmst, net.D[d], net.r[d], p);
        const double den = p.C.re * p.C.re + p.C.im * p.C.im;
        r.invC0_re[d] = p.C.re / den;
        r.invC0_im[d] = -p.C.im / den;
        r.tau0[d] = t[7] + p.dt;
        const double are = p.C.re / t[6], aim = p.C.im / t[6];
        r.h0fac_re[d] = are * ce - aim * se;
        r.h0fac_im[d] = are * se + aim * ce;
    }
    r.nc = nc;
    *out = r;
}

// ---------------------------------------------------------------------------
// Per-chain setup: record (and, for the gradient, d record / d theta).
// ---------------------------------------------------------------------------
__device__ inline int theta_status(const double* t) {
    bool nan = false;
    for (int i = 0; i < 13; ++i) nan = nan || isnan(t[i]);
    if (nan) return -1;
    bool fin = true;
    for (int i = 0; i < 13; ++i) fin = fin && isfinite(t[i]);
    const bool ok = fin && t[0] > 0.0 && t[1] > 0.0 && t[6] > 0.0 && fabs(t[2]) < 1.0 &&
                    fabs(t[3]) < 1.0 && t[4] >= 0.0 && t[5] >= 0.0;
    return ok ? 1 : 0;
}

// Record for the likelihood alone.  Two kinds of blocks, one thread per chain in each:
// intrinsic blocks write the status, the TaylorF2 coefficients (or the IMRPhenomD_NRTidalv2
// node parameters), G and dL; extrinsic blocks write P_d and the delays.  The two halves of a
// chain's setup run concurrently (the kernel is latency-bound); the likelihood kernels form
// K_d = P_d G.
__global__ __launch_bounds__(64) void k_chain_setup(const double* __restrict__ theta, int64_t B, Network net,
                                                    RefConsts ref, double* __restrict__ rec, int64_t n_int_blocks) {
    const bool intrinsic = (int64_t)blockIdx.x < n_int_blocks;
    // XCD-aware, as in k_chain_setup_grad: workgroup i of each half (n_int_blocks a multiple of
    // 8) takes the 8-chain blocks 64 (i / 8) + i % 8 + 8 j, j = 0..7, which the likelihood
    // kernels' 8-chain workgroups read on the same XCD.
    const int64_t wi = (int64_t)blockIdx.x - (intrinsic ? 0 : n_int_blocks);
    const int64_t blk = 64 * (wi / 8) + wi % 8 + 8 * (threadIdx.x / 8);
    const int64_t b = blk * 8 + threadIdx.x % 8;
    if (b >= B) return;
    double t[13];
#pragma unroll
    for (int i = 0; i < 13; ++i) t[i] = theta[b * 13 + i];
    double* out = rec + b * kRecStride;
    const int st = theta_status(t);
    if (intrinsic) {
        if (st != 1) {
            out[kRecStatus] = st < 0 ? __builtin_nan("") : 0.0;
            for (int i = kRecDc; i < kRecDc + kTf2Basis; ++i) out[i] = 0.0;
            out[kRecG] = out[kRecG + 1] = out[kRecDl] = 0.0;
            return;
        }
        out[kRecStatus] = 1.0;
        double dconst = 0.0, amp;
        if (ref.waveform == kWfNrtv2) {
            for (int k = 0; k < kTf2Basis; ++k) out[kRecDc + k] = 0.0;
            amp = tf2_amp<double>(t[0]);
            NrtParams<double> np;
            nrt_params<double>(t[0], t[1], t[2], t[3], t[4], t[5], ref.nc, np);
            const double* src = reinterpret_cast<const double*>(&np);
            for (int i = 0; i < kNrtParams; ++i) out[kRecNrt + i] = src[i];
        } else {
            Tf2Coeffs<double> c;
            tf2_coeffs<double>(t[0], t[1], t[2], t[3], t[4], t[5], c);
            for (int k = 0; k < kTf2Basis; ++k) out[kRecDc + k] = (c.c[k] - ref.c0[k]) * (double)kPhasorN;
            dconst = c.c_const - ref.c0_const;
            dconst -= rint(dconst);  // whole revolutions removed
            amp = c.amp;
        }
        // G = (dL0/dL)(amp/amp0) exp(2i(phic - phic0)) exp(-2 pi i dconst)
        const double ang = 2.0 * (t[8] - ref.phic0) - (2.0 * kPi) * dconst;
        const double mag = (ref.dl0 / t[6]) * (amp / ref.amp0);
        double sa, ca;
        dsincos(ang, sa, ca);
        out[kRecG] = mag * ca;
        out[kRecG + 1] = mag * sa;
        out[kRecDl] = t[6];
    } else {
        if (st != 1) {
            for (int i = kRecK; i < kRecTau + kMaxDet; ++i) out[i] = 0.0;
            return;
        }
        SkyFrame<double> sky;
        sky_frame<double>(t[9], t[10], t[11], t[12], net.gmst, sky);
        for (int d = 0; d < kMaxDet; ++d) {
            double pr = 0.0, pi = 0.0, tau = 0.0;
            if (d < net.n_det) {
                Proj<double> p;
                project<double>(sky, net.D[d], net.r[d], p);
                const Cx<double> P = cmul(p.C, Cx<double>{ref.invC0_re[d], ref.invC0_im[d]});
                pr = P.re;
                pi = P.im;
                tau = ((t[7] + p.dt) - ref.tau0[d]) * (double)kPhasorN;
            }
            out[kRecK + 2 * d] = pr;
            out[kRecK + 2 * d + 1] = pi;
            out[kRecTau + d] = tau;
        }
    }
}

// Record and partial derivatives for the gradient.  Two kinds of blocks:
//   intrinsic blocks: 8 lanes per chain, lane t < 6 differentiates the TaylorF2
//     coefficients with respect to parameter t (one dual component per lane);
//   extrinsic blocks: 4 lanes per chain, lane a differentiates the projection with
//     respect to angle a of (iota, psi, ra, dec).
// Lane 0 of each group writes the values.  The blocks of the two kinds are
// disjoint, so no wavefront mixes the two code paths.  One-wavefront blocks: the kernel
// is latency-bound with 1.5 waves per SIMD, and single-wave blocks spread evenly over the
// CUs (measured 9.5 -> 8.0 us at 8192 chains against 4-wave blocks).
constexpr int kIntLanes = 8;
constexpr int kExtLanes = 4;

// The MALA proposal z' = z + (s/2) gz + sqrt(s) xi of chain b, formed by the chain's L lanes
// together (lane r of the group, the groups aligned in the wavefront): lane r loads and forms
// components r, r + L, ...; every lane then receives all 13 components by lane permutes.
// theta is z', or NaN in every component outside the prior box.
//
// With WRITE (the intrinsic groups, L = 8) the lanes also fill the chain's accept record for
// the gradient kernel's epilogue (kMalaRec* rows of 16): with h = s/2, k = 1/sqrt(2 s) and f
// the factor from d lnL/dtheta to d lnL/dz (1, or -1/sin iota and 1/cos dec), component i's
// term of log q(z|z') - log q(z'|z) is rq_i - u_i^2 with u_i = dq_i - aq_i g_i(theta'), where
//   rq = ((z' - z - h gz) k)^2,  dq = (z - z') k,  aq = h k f,
// and the spare slots of the rq row hold lnL(z) + log u and the two factors f.
template <int L, bool WRITE>
__device__ inline void mala_proposal(const MalaProp& mp, int64_t b, int r, double (&t)[13]) {
    constexpr int S = (13 + L - 1) / L;
    // Every load first, unconditionally (a slot past component 12 reads component 12 and is
    // not used), so that they are in flight together: one memory round trip.
    double z[S], gz[S], xi[S], lnl = 0.0, logu = 0.0;
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const int64_t o = b * 13 + min(k * L + r, 12);
        z[k] = mp.z[o];
        gz[k] = mp.gz[o];
        xi[k] = mp.xi[o];
    }
    if (WRITE) {
        lnl = mp.lnl[b];
        logu = mp.logu[b];
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of their first use
    double q[S];
#pragma unroll
    for (int k = 0; k < S; ++k) {
        const int i0 = k * L, i = i0 + r;
        double s = mp.s[i0], sq = mp.sq[i0], kk = mp.k[i0], hk = mp.hk[i0];
#pragma unroll
        for (int rr = 1; rr < L && i0 + rr < 13; ++rr) {
            s = r == rr ? mp.s[i0 + rr] : s;
            sq = r == rr ? mp.sq[i0 + rr] : sq;
            kk = r == rr ? mp.k[i0 + rr] : kk;
            hk = r == rr ? mp.hk[i0 + rr] : hk;
        }
        q[k] = fma(sq, xi[k], fma(0.5 * s, gz[k], z[k]));
        if (WRITE && i < 13) {
            double* rec = mp.rec + b * kMalaRecStride;
            double f = 1.0;
            if (i == kMalaIota || i == kMalaDec) {
                f = (i == kMalaIota ? -1.0 : 1.0) / sqrt(fma(-q[k], q[k], 1.0));
                rec[i == kMalaIota ? kMalaRecFIota : kMalaRecFDec] = f;
            }
            const double rf = (q[k] - z[k] - 0.5 * s * gz[k]) * kk;
            rec[kMalaRecZp + i] = q[k];
            rec[kMalaRecDq + i] = (z[k] - q[k]) * kk;
            rec[kMalaRecAq + i] = hk * f;
            rec[kMalaRecRq + i] = rf * rf;
        }
    }
    if (WRITE && r == L - 1) mp.rec[b * kMalaRecStride + kMalaRecThr] = lnl + logu;
    const int base = (int)(threadIdx.x & 63) & ~(L - 1);
    bool in = true;
#pragma unroll
    for (int i = 0; i < 13; ++i) {
        t[i] = lane_permute(q[i / L], base + i % L);
        in = in && t[i] >= mp.lo[i] && t[i] <= mp.hi[i];
    }
    if (!in)
#pragma unroll
        for (int i = 0; i < 13; ++i) t[i] = __builtin_nan("");
}

// PROP: the chain's theta is the MALA proposal theta(z') (mala_proposal); the intrinsic
// groups write the chain's accept record.
template <bool PROP>
__global__ __launch_bounds__(64) void k_chain_setup_grad(const double* __restrict__ theta, int64_t B, Network net,
                                                          RefConsts ref, double* __restrict__ rec,
                                                          double* __restrict__ jac, int64_t n_int_blocks, MalaProp mp) {
    const bool intrinsic = (int64_t)blockIdx.x < n_int_blocks;
    int64_t b;
    int tg;
    if (intrinsic) {  // workgroup w: the 8-chain block w
        const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        b = gid / kIntLanes;
        tg = (int)(gid % kIntLanes);
    } else {
        // XCD-aware: workgroups are dispatched to the 8 XCDs in turn, so block w's intrinsic
        // workgroup and the likelihood kernel's workgroup of the same 8 chains share XCD w % 8.
        // Extrinsic workgroup p (n_int_blocks is a multiple of 8) takes blocks
        // 16 (p / 8) + p % 8 and that + 8, both of its own XCD, in lanes 0-31 and 32-63.
        const int64_t p = (int64_t)blockIdx.x - n_int_blocks;
        const int64_t blk = 16 * (p / 8) + p % 8 + (threadIdx.x >= 32 ? 8 : 0);
        b = blk * 8 + (threadIdx.x & 31) / kExtLanes;
        tg = (int)(threadIdx.x % kExtLanes);
    }
    if (b >= B) return;
    double t[13];
    if constexpr (PROP) {
        if (intrinsic) {
            mala_proposal<kIntLanes, true>(mp, b, tg, t);
        } else {
            mala_proposal<kExtLanes, false>(mp, b, tg, t);
            if (!isnan(t[0])) {  // the intrinsic lanes use neither angle (only its finiteness)
                t[9] = acos(fmin(fmax(t[9], -1.0), 1.0));
                t[12] = asin(fmin(fmax(t[12], -1.0), 1.0));
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < 13; ++i) t[i] = theta[b * 13 + i];
    }
    double* out = rec + b * kRecStride;
    double* J = jac + b * kJacStride;
    const int st = theta_status(t);
    using D1 = Dual<1>;
    if (intrinsic) {
        if (tg >= 6) return;
        if (st != 1) {
            if (tg == 0) {
                out[kRecStatus] = st < 0 ? __builtin_nan("") : 0.0;
                for (int i = kRecDc; i < kRecDc + kTf2Basis; ++i) out[i] = 0.0;
                out[kRecG] = out[kRecG + 1] = out[kRecDl] = 0.0;
            }
            for (int k = 0; k < kJacExt / 6; ++k) J[kJacInt + k * 6 + tg] = 0.0;
            return;
        }
        D1 ti[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            ti[i] = D1(t[i]);
            ti[i].d[0] = (i == tg) ? 1.0 : 0.0;
        }
        if (ref.waveform == kWfNrtv2) {
            NrtParams<D1> np;
            nrt_params<D1>(ti[0], ti[1], ti[2], ti[3], ti[4], ti[5], ref.nc, np);
            const D1* pv = reinterpret_cast<const D1*>(&np);
            for (int k = 0; k < kNrtAdj; ++k) J[kJacInt + k * 6 + tg] = pv[k < kNrtAdjSkip ? k : k + 1].d[0];
            const D1 amp = tf2_amp<D1>(ti[0]);
            J[kJacInt + kJacAmpNrt * 6 + tg] = amp.d[0] / amp.v;
            if (tg == 0) {
                out[kRecStatus] = 1.0;
                for (int k = 0; k < kTf2Basis; ++k) out[kRecDc + k] = 0.0;
                const double ang = 2.0 * (t[8] - ref.phic0);
                const double mag = (ref.dl0 / t[6]) * (amp.v / ref.amp0);
                double sa, ca;
                dsincos(ang, sa, ca);
                out[kRecG] = mag * ca;
                out[kRecG + 1] = mag * sa;
                out[kRecDl] = t[6];
                for (int i = 0; i < kNrtParams; ++i) out[kRecNrt + i] = pv[i].v;
            }
            return;
        }
        Tf2Coeffs<D1> c;
        tf2_coeffs<D1>(ti[0], ti[1], ti[2], ti[3], ti[4], ti[5], c);
        for (int k = 0; k < kTf2Basis; ++k) J[kJacInt + k * 6 + tg] = c.c[k].d[0];
        J[kJacInt + 10 * 6 + tg] = c.c_const.d[0];
        J[kJacInt + kJacAmpTf2 * 6 + tg] = c.amp.d[0] / c.amp.v;
        if (tg == 0) {
            out[kRecStatus] = 1.0;
            for (int k = 0; k < kTf2Basis; ++k) out[kRecDc + k] = (c.c[k].v - ref.c0[k]) * (double)kPhasorN;
            double dconst = c.c_const.v - ref.c0_const;
            dconst -= rint(dconst);
            const double ang = 2.0 * (t[8] - ref.phic0) - (2.0 * kPi) * dconst;
            const double mag = (ref.dl0 / t[6]) * (c.amp.v / ref.amp0);
            double sa, ca;
            dsincos(ang, sa, ca);
            out[kRecG] = mag * ca;
            out[kRecG + 1] = mag * sa;
            out[kRecDl] = t[6];
        }
    } else {
        if (st != 1) {
            if (tg == 0)
                for (int i = kRecK; i < kRecTau + kMaxDet; ++i) out[i] = 0.0;
            for (int i = 0; i < 36; ++i)
                if (i % 4 == tg) J[kJacExt + i] = 0.0;
            return;
        }
        D1 ang[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            ang[a] = D1(t[9 + a]);
            ang[a].d[0] = (a == tg) ? 1.0 : 0.0;
        }
        SkyFrame<D1> sky;
        sky_frame<D1>(ang[0], ang[1], ang[2], ang[3], net.gmst, sky);
        for (int d = 0; d < kMaxDet; ++d) {
            if (d < net.n_det) {
                Proj<D1> p;
                project<D1>(sky, net.D[d], net.r[d], p);
                const Cx<D1> inv0{D1(ref.invC0_re[d]), D1(ref.invC0_im[d])};
                const Cx<D1> P = cmul(p.C, inv0);
                J[kJacExt + (d * 3 + 0) * 4 + tg] = P.re.d[0];
                J[kJacExt + (d * 3 + 1) * 4 + tg] = P.im.d[0];
                J[kJacExt + (d * 3 + 2) * 4 + tg] = p.dt.d[0];
                if (tg == 0) {
                    out[kRecK + 2 * d] = P.re.v;
                    out[kRecK + 2 * d + 1] = P.im.v;
                    out[kRecTau + d] = ((t[7] + p.dt.v) - ref.tau0[d]) * (double)kPhasorN;
                }
            } else {
                J[kJacExt + (d * 3 + 0) * 4 + tg] = J[kJacExt + (d * 3 + 1) * 4 + tg] =
                    J[kJacExt + (d * 3 + 2) * 4 + tg] = 0.0;
                if (tg == 0) out[kRecK + 2 * d] = out[kRecK + 2 * d + 1] = out[kRecTau + d] = 0.0;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Summary data: one workgroup per bin, T threads taking up to PPT grid points each per pass
// (point base + p T + t for thread t), as many passes as the bin needs.  A pass issues all of
// its data and PSD loads before its arithmetic, and the first pass's loads go out before the
// unit-phasor table is copied into LDS, so that the two memory round trips overlap.  The
// reference waveform is generated inline, once per point, and projected onto every detector
// with the unit phasors from the LDS table.  Each thread adds its points in order, the 7 ND
// sums are reduced across each wavefront (wave_sum_n) and the wavefront totals added in wave
// order: the summary data are bitwise reproducible, and the pass is one kernel with no
// partial sums in memory.  Workgroup w takes bin order[w]: bins sorted by size, the largest
// first, the order reversed for every next group of as many workgroups as the device has
// CUs, so that the workgroups that share a CU pair large bins with small ones (the largest
// bins, up to a few thousand points, bound the pass).
// ---------------------------------------------------------------------------
template <int ND, int WF>
__device__ inline void summary_point(const SummaryArgs& a, const double2* tab, int64_t k, double fm, const double* dre,
                                     const double* dim, const double* ps, double (&acc)[ND][7]) {
    const RefConsts& ref = a.ref;
    const double w = 4.0 * a.delta_f;
    const double f = a.f_low + (double)k * a.delta_f;
    const double ix = inv_cbrt_nr(f);  // f^(-1/3)
    const double x = f * ix * ix;
    const double lx = log(f) * (1.0 / 3.0);
    double phi = 0.0;
    double amp = ref.amp0 * (ix * ix * ix) * sqrt(ix);  // f^(-7/6)
    if constexpr (WF == kWfNrtv2) {
        double a0;
        nrt_node(ref.nrt, f, x, ix, lx, exp(5.78 * lx), a.ref_taper != 0, phi, a0);
        amp *= a0;
    } else {
        double bas[kTf2Basis];
        tf2_basis(x, ix, lx, bas);
#pragma unroll
        for (int j = 0; j < kTf2Basis; ++j) phi = fma(ref.c0[j], bas[j], phi);
    }
    const double df = f - fm;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        double cu, su;
        unit_phasor(fma(f, ref.tau0[d], phi) * (double)kPhasorN, tab, cu, su);
        const double hre = amp * (ref.h0fac_re[d] * cu - ref.h0fac_im[d] * su);
        const double him = amp * (ref.h0fac_re[d] * su + ref.h0fac_im[d] * cu);
        const double wk = w * rcp_nr(ps[d]);
        // d conj(h0) w and |h0|^2 w
        const double are = (dre[d] * hre + dim[d] * him) * wk;
        const double aim = (dim[d] * hre - dre[d] * him) * wk;
        const double hh = (hre * hre + him * him) * wk;
        acc[d][0] += are;
        acc[d][1] += aim;
        acc[d][2] += are * df;
        acc[d][3] += aim * df;
        acc[d][4] += hh;
        acc[d][5] += hh * df;
        acc[d][6] += hh * df * df;
    }
}

template <int ND, int PPT>
__device__ inline void summary_loads(const SummaryArgs& a, int64_t base, int64_t hi, int t, int T,
                                     double (&re)[PPT][ND], double (&im)[PPT][ND], double (&ps)[PPT][ND]) {
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
        const int64_t k = base + (int64_t)p * T + t;
        if (k < hi) {
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                const int64_t o = (int64_t)d * a.n_freq + k;
                const double2 v = reinterpret_cast<const double2*>(a.data)[o];
                re[p][d] = v.x;
                im[p][d] = v.y;
                ps[p][d] = a.psd[o];
            }
        }
    }
}

template <int ND, int WF, int T, int PPT>
__global__ __launch_bounds__(T) void k_summary_bins(SummaryArgs a) {
    constexpr int NV = (7 * ND + 3) / 4 * 4;
    constexpr int NW = T / 64;
    __shared__ double2 tab[kPhasorN];
    __shared__ double red[NW][NV];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wid = wave_id();
    const int b = a.order[blockIdx.x];
    const int64_t lo = a.edges[b];
    const int64_t hi = (b == a.n_bins - 1) ? a.n_freq : a.edges[b + 1];
    const double fm = a.f_low + 0.5 * (double)(a.edges[b] + a.edges[b + 1]) * a.delta_f;
    double re[PPT][ND], im[PPT][ND], ps[PPT][ND];
    summary_loads<ND, PPT>(a, lo, hi, t, T, re, im, ps);
    load_phasor_table(a.phasor, tab);
    double acc[ND][7];
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
        for (int j = 0; j < 7; ++j) acc[d][j] = 0.0;
    for (int64_t base = lo;;) {
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int64_t k = base + (int64_t)p * T + t;
            if (k < hi) summary_point<ND, WF>(a, tab, k, fm, re[p], im[p], ps[p], acc);
        }
        base += (int64_t)T * PPT;
        if (base >= hi) break;
        summary_loads<ND, PPT>(a, base, hi, t, T, re, im, ps);
    }
    double part[NV], tot[NV];
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
        for (int j = 0; j < 7; ++j) part[d * 7 + j] = acc[d][j];
#pragma unroll
    for (int i = 7 * ND; i < NV; ++i) part[i] = 0.0;
    wave_sum_n<NV>(part, tot);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) red[wid][i] = tot[i];
    }
    __syncthreads();
    if (t < 7 * ND) {
        double v = red[0][t];
#pragma unroll
        for (int w = 1; w < NW; ++w) v += red[w][t];
        const int d = t / 7, j = t % 7;
        a.summary[((int64_t)d * a.n_bins + b) * 7 + j] = v;
    }
}

// ---------------------------------------------------------------------------
// Node tables.  With p = r_b, q = r_{b+1}, w = 1/(f_{b+1} - f_b) the bin term
//   Re(A0 r0* + A1 r1*) - B0|r0|^2/2 - B1 Re(r0 r1*) - B2|r1|^2/2
// equals Re(alpha p* + beta q*) - [ |p|^2 (B0/4 - B1 w + B2 w^2)
//   + |q|^2 (B0/4 + B1 w + B2 w^2) + Re(p q*) (B0/2 - 2 B2 w^2) ] / 2
// with alpha = A0/2 - A1 w, beta = A0/2 + A1 w.  Collecting by edge:
//   gamma_j = alpha_j + beta_{j-1},  mu_j = (left part of bin j) + (right part of bin j-1),
//   nu_b = B0/2 - 2 B2 w^2 multiplies Re(r_b r_{b+1}*).  The tables hold the cross
// weights of 2 lnL, xL_j = -nu_{j-1} and xR_j = -nu_j.
//
// Centre-node variant: the nodes are e_0, c_0, e_1, c_1, ..., e_Nb (edges and bin centres
// f_m interleaved), r0 = r(c_b) and r1 = (r(e_{b+1}) - r(e_b)) w.  Bin b's term
//   Re(A0 r0* + A1 r1*) - B0 |r0|^2 / 2 - B1 Re(r0 r1*)
// then gives  gamma(c_b) = A0, mu(c_b) = B0, gamma(e_b) -= A1 w, gamma(e_{b+1}) += A1 w, and the
// cross weights (2 lnL) 2 B1 w between e_b and c_b and -2 B1 w between c_b and e_{b+1}.
// ---------------------------------------------------------------------------
__device__ inline double node_frequency(const NodeArgs& a, int j) {
    if (!a.centre) return a.f_low + (double)a.edges[j] * a.delta_f;
    if ((j & 1) == 0) return a.f_low + (double)a.edges[j >> 1] * a.delta_f;
    const int b = j >> 1;  // the same expression as the bin centre of the summary pass
    return a.f_low + 0.5 * (double)(a.edges[b] + a.edges[b + 1]) * a.delta_f;
}

__global__ void k_node_tables(NodeArgs a) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;  // node index
    if (j >= a.n_nodes_pad) return;
    // lane-contiguous position (TaylorF2) or natural order (IMRPhenomD_NRTidalv2)
    const int pos = a.ref.waveform == kWfNrtv2 ? j : (j % a.L) * kNodeTile + j / a.L;
    const bool real_node = j < a.n_nodes;
    const int nb = a.centre ? (a.n_nodes - 1) / 2 : a.n_nodes - 1;
    double f = 0.0, x = 1.0, ix = 1.0, lx = 0.0;
    if (real_node) {
        f = node_frequency(a, j);
        x = cbrt(f);
        ix = 1.0 / x;
        lx = log(x);
    }
    a.node_fx[2 * pos] = f;
    a.node_fx[2 * pos + 1] = x;
    a.node_il[2 * pos] = ix;
    a.node_il[2 * pos + 1] = lx;
    if (a.ref.waveform == kWfNrtv2) {
        double phi0 = 0.0, a0 = 1.0;
        const double x578 = exp(5.78 * lx);
        a.node_x578[pos] = x578;
        if (real_node) nrt_node(a.ref.nrt, f, x, ix, lx, x578, a.ref_taper != 0, phi0, a0);
        const bool ok = a0 > 0.0 && isfinite(a0) && isfinite(phi0);
        if (!ok) *a.bad_ref = 1;
        a.phi0[pos] = phi0;
        a.ia0[pos] = ok ? 1.0 / a0 : 0.0;
        a.ia0_32[pos] = ok ? (float)(1.0 / a0) : 0.0f;
    }
    for (int d = 0; d < a.n_det; ++d) {
        double gre = 0.0, gim = 0.0, mu = 0.0, xl = 0.0, xr = 0.0;
        if (real_node && a.centre) {
            const int b = j >> 1;
            if (j & 1) {  // centre of bin b
                const double* s = a.summary + ((int64_t)d * nb + b) * 7;
                const double w = 1.0 / ((double)(a.edges[b + 1] - a.edges[b]) * a.delta_f);
                gre = s[0];
                gim = s[1];
                mu = s[4];
                xl = 2.0 * s[5] * w;
                xr = -2.0 * s[5] * w;
            } else {      // edge b
                if (b < nb) {  // bin b to the right
                    const double* s = a.summary + ((int64_t)d * nb + b) * 7;
                    const double w = 1.0 / ((double)(a.edges[b + 1] - a.edges[b]) * a.delta_f);
                    gre -= s[2] * w;
                    gim -= s[3] * w;
                    xr = 2.0 * s[5] * w;
                }
                if (b > 0) {   // bin b - 1 to the left
                    const double* s = a.summary + ((int64_t)d * nb + (b - 1)) * 7;
                    const double w = 1.0 / ((double)(a.edges[b] - a.edges[b - 1]) * a.delta_f);
                    gre += s[2] * w;
                    gim += s[3] * w;
                    xl = -2.0 * s[5] * w;
                }
            }
        } else if (real_node) {
            if (j < nb) {  // bin j lies to the right of edge j
                const double* s = a.summary + ((int64_t)d * nb + j) * 7;
                const double w = 1.0 / ((double)(a.edges[j + 1] - a.edges[j]) * a.delta_f);
                const double b2 = a.keep_b2 ? s[6] : 0.0;
                gre += 0.5 * s[0] - s[2] * w;
                gim += 0.5 * s[1] - s[3] * w;
                mu += 0.25 * s[4] - s[5] * w + b2 * w * w;
                xr = 2.0 * b2 * w * w - 0.5 * s[4];
            }
            if (j > 0) {  // bin j-1 lies to the left
                const double* s = a.summary + ((int64_t)d * nb + (j - 1)) * 7;
                const double w = 1.0 / ((double)(a.edges[j] - a.edges[j - 1]) * a.delta_f);
                const double b2 = a.keep_b2 ? s[6] : 0.0;
                gre += 0.5 * s[0] + s[2] * w;
                gim += 0.5 * s[1] + s[3] * w;
                mu += 0.25 * s[4] + s[5] * w + b2 * w * w;
                xl = 2.0 * b2 * w * w - 0.5 * s[4];
            }
        }
        const int64_t o = (int64_t)d * a.n_nodes_pad + pos;
        a.g[2 * o] = gre;
        a.g[2 * o + 1] = gim;
        a.mu[o] = mu;
        a.xL[o] = xl;
        a.xR[o] = xr;
        a.g32[2 * o] = (float)gre;
        a.g32[2 * o + 1] = (float)gim;
        a.mu32[o] = (float)mu;
        a.xL32[o] = (float)xl;
        a.xR32[o] = (float)xr;
    }
}

// Per-detector magnitude sums of the edge tables and M_d = sum_j mu_dj (one wavefront
// per detector, fixed reduction order).
__global__ __launch_bounds__(64) void k_event_scales(NodeArgs a) {
    const int d = blockIdx.x;
    const int lane = threadIdx.x;
    double gs = 0.0, hs = 0.0, ms = 0.0;
    for (int j = lane; j < a.n_nodes_pad; j += 64) {
        const int64_t o = (int64_t)d * a.n_nodes_pad + j;
        gs += sqrt(a.g[2 * o] * a.g[2 * o] + a.g[2 * o + 1] * a.g[2 * o + 1]);
        hs += fabs(a.mu[o]) + fabs(a.xL[o]);
        ms += a.mu[o];
    }
    gs = wave_sum(gs);
    hs = wave_sum(hs);
    ms = wave_sum(ms);
    if (lane == 0) {
        a.scales[2 * d] = gs;
        a.scales[2 * d + 1] = hs;
        a.mu_sum[d] = ms;
    }
}

// ---------------------------------------------------------------------------
// Projected strain on a grid for one parameter vector (its constants come from
// k_ref_setup run on that vector).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_strain(const RefConsts* __restrict__ cst, int32_t taper, int32_t n_det,
                                                double f_low, double delta_f, int64_t n_freq,
                                                double* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_freq) return;
    const RefConsts& r = *cst;
    const double f = f_low + (double)k * delta_f;
    const double x = cbrt(f), ix = 1.0 / x, lx = log(x);
    double ph = 0.0;
    double am = r.amp0 * (ix * ix * ix) * sqrt(ix);
    if (r.waveform == kWfNrtv2) {
        double af;
        nrt_node(r.nrt, f, x, ix, lx, exp(5.78 * lx), taper != 0, ph, af);
        am *= af;
    } else {
        double bas[kTf2Basis];
        tf2_basis(x, ix, lx, bas);
        for (int j = 0; j < kTf2Basis; ++j) ph = fma(r.c0[j], bas[j], ph);
    }
    for (int d = 0; d < n_det; ++d) {
        double cu, su;
        expm2pi_rev(fma(f, r.tau0[d], ph), cu, su);
        const int64_t o = (int64_t)d * n_freq + k;
        out[2 * o] = am * (r.h0fac_re[d] * cu - r.h0fac_im[d] * su);
        out[2 * o + 1] = am * (r.h0fac_re[d] * su + r.h0fac_im[d] * cu);
    }
}

// ---------------------------------------------------------------------------
// Bin placement on the device (Sec. II C): the post-Newtonian phase-bound ansatz
//   Phi(f) = sum_g sgn(g) (f / f*_g)^g,  g in {-5/3, -2/3, 1, 5/3, 7/3},
// f*_g = f_low for g < 0 and f_high for g > 0, on every grid point (Phi increases with f);
// n_bins + 1 equally spaced targets between Phi(f_low) and Phi(f_high), each snapped to the
// grid point with the nearer Phi (the lower one on a tie); then one pass each way makes the
// indices strictly increasing with the ends at 0 and N - 1.
// ---------------------------------------------------------------------------
__global__ void k_pn_phase(double f_low, double delta_f, int64_t n, double* __restrict__ phi) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double f_high = f_low + (double)(n - 1) * delta_f;
    const double f = f_low + (double)k * delta_f;
    double s = 0.0;
    s += -pow(f / f_low, -5.0 / 3.0);
    s += -pow(f / f_low, -2.0 / 3.0);
    s += pow(f / f_high, 1.0);
    s += pow(f / f_high, 5.0 / 3.0);
    s += pow(f / f_high, 7.0 / 3.0);
    phi[k] = s;
}

__global__ void k_pn_snap(const double* __restrict__ phi, int64_t n, int32_t n_bins, int64_t* __restrict__ edges) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n_bins) return;
    const double p0 = phi[0], p1 = phi[n - 1];
    const double tgt = p0 + (p1 - p0) * (double)i / (double)n_bins;
    int64_t lo = 0, hi = n;  // first index with phi >= tgt
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (phi[mid] < tgt)
            lo = mid + 1;
        else
            hi = mid;
    }
    const int64_t pos = lo < 1 ? 1 : (lo > n - 1 ? n - 1 : lo);
    edges[i] = (tgt - phi[pos - 1] <= phi[pos] - tgt) ? pos - 1 : pos;
}

__global__ void k_pn_order(int64_t n, int32_t n_bins, int64_t* __restrict__ edges) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    edges[0] = 0;
    edges[n_bins] = n - 1;
    for (int32_t i = 1; i <= n_bins; ++i) edges[i] = edges[i] > edges[i - 1] + 1 ? edges[i] : edges[i - 1] + 1;
    edges[n_bins] = n - 1;
    for (int32_t i = n_bins - 1; i >= 0; --i) edges[i] = edges[i] < edges[i + 1] - 1 ? edges[i] : edges[i + 1] - 1;
}

hipError_t launch_bin_edges(double f_low, double delta_f, int64_t n, int32_t n_bins, double* phi, int64_t* edges,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_pn_phase, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f_low, delta_f, n, phi);
    hipLaunchKernelGGL(k_pn_snap, dim3((unsigned)((n_bins + 1 + 255) / 256)), dim3(256), 0, s, phi, n, n_bins, edges);
    hipLaunchKernelGGL(k_pn_order, dim3(1), dim3(64), 0, s, n, n_bins, edges);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_ref_setup(const double* theta, const Network& net, int32_t waveform, RefConsts* out_dev,
                            hipStream_t s) {
    Theta13 th;
    for (int i = 0; i < 13; ++i) th.v[i] = theta[i];
    hipLaunchKernelGGL(k_ref_setup, dim3(1), dim3(64), 0, s, th, net, waveform, nrt_consts(), out_dev);
    return hipGetLastError();
}

hipError_t launch_chain_setup(const double* theta, int64_t B, const Network& net, const RefConsts& ref,
                              double* rec, double* jac, hipStream_t s, KTime kt, const MalaProp* prop) {
    if (jac) {
        // intrinsic workgroups: one per 8-chain block, padded to a multiple of 8; extrinsic: two
        // blocks each, in groups of 8 workgroups covering 16 blocks (k_chain_setup_grad)
        const int64_t blocks = (B + 7) / 8;
        const int64_t n_int = (blocks + 7) / 8 * 8;
        const int64_t n_ext = (blocks + 15) / 16 * 8;
        if (prop)
            launch_k(k_chain_setup_grad<true>, dim3((unsigned)(n_int + n_ext)), dim3(64), s, kt, theta, B, net, ref,
                     rec, jac, n_int, *prop);
        else
            launch_k(k_chain_setup_grad<false>, dim3((unsigned)(n_int + n_ext)), dim3(64), s, kt, theta, B, net, ref,
                     rec, jac, n_int, MalaProp{});
    } else {
        const int64_t n_half = ((B + 7) / 8 + 63) / 64 * 8;  // groups of 8 workgroups, 64 blocks
        launch_k(k_chain_setup, dim3((unsigned)(2 * n_half)), dim3(64), s, kt, theta, B, net, ref, rec, n_half);
    }
    return hipGetLastError();
}

template <int ND>
void launch_summary_nd(const SummaryArgs& a, hipStream_t s, KTime kt) {
    const dim3 g((unsigned)a.n_bins);  // one workgroup per bin
    if (a.ref.waveform == kWfNrtv2)
        launch_k(k_summary_bins<ND, kWfNrtv2, kSumThreadsNrt, kSumPptNrt>, g, dim3(kSumThreadsNrt), s, kt, a);
    else
        launch_k(k_summary_bins<ND, kWfTaylorF2, kSumThreadsTf2, kSumPptTf2>, g, dim3(kSumThreadsTf2), s, kt, a);
}

hipError_t launch_summary(const SummaryArgs& a, hipStream_t s, KTime kt) {
    switch (a.n_det) {
        case 1: launch_summary_nd<1>(a, s, kt); break;
        case 2: launch_summary_nd<2>(a, s, kt); break;
        default: launch_summary_nd<3>(a, s, kt); break;
    }
    return hipGetLastError();
}

hipError_t launch_node_tables(const NodeArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_node_tables, dim3((unsigned)((a.n_nodes_pad + 255) / 256)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_event_scales, dim3((unsigned)a.n_det), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_strain(const RefConsts* cst_dev, int32_t waveform, int32_t taper, int32_t n_det, double f_low,
                         double delta_f, int64_t n_freq, double* out, hipStream_t s) {
    (void)waveform;
    hipLaunchKernelGGL(k_strain, dim3((unsigned)((n_freq + 255) / 256)), dim3(256), 0, s, cst_dev, taper, n_det,
                       f_low, delta_f, n_freq, out);
    return hipGetLastError();
}

}  // namespace rbl
