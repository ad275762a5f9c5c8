// HIP kernels of the relative-binned likelihood (gfx950, wave64).
//
//  k_ref_setup      reference (fiducial) constants for theta0            [1 thread]
//  k_chain_setup    per-chain record (+ Jacobian for the gradient)       [1 thread / chain]
//  k_summary_items  summary-data partial sums over (bin, chunk) items    [1 wave / item]
//  k_summary_reduce ordered sum of the partials of each bin              [1 thread / (det, bin, field)]
//  k_node_tables    per-edge coefficient tables of the binned sum        [1 thread / node]
//  k_loglike_fwd    fused ratio + bin contraction + reduction            [1 wave / chain]
//  k_loglike_grad   the same with the hand-written adjoint               [1 wave / chain]
//  k_loglike_full   full-grid likelihood (validation)                    [1 block / chain]
//  k_strain         projected strain on a grid (injections)              [1 thread / grid point]
//
// All reductions are in a fixed order, so results are bitwise reproducible.
#include "rbl_launch.h"

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
__device__ inline double lane_value(double v, int src) { return __shfl(v, src, 64); }

__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// ---------------------------------------------------------------------------
// Reference constants
// ---------------------------------------------------------------------------
__global__ void k_ref_setup(Theta13 th, Network net, RefConsts* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    RefConsts r{};
    const double* t = th.v;
    bool ok = t[0] > 0.0 && t[1] > 0.0 && t[6] > 0.0 && fabs(t[2]) < 1.0 && fabs(t[3]) < 1.0 &&
              t[4] >= 0.0 && t[5] >= 0.0;
    for (int i = 0; i < 13; ++i) ok = ok && isfinite(t[i]);
    r.status = ok ? 1 : 0;
    Tf2Coeffs<double> c;
    tf2_coeffs<double>(t[0], t[1], t[2], t[3], t[4], t[5], c);
    for (int b = 0; b < kTf2Basis; ++b) r.c0[b] = c.c[b];
    r.c0_const = c.c_const;
    r.amp0 = c.amp;
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
    *out = r;
}

// ---------------------------------------------------------------------------
// Per-chain setup: record (and, for the gradient, d record / d theta).
// ---------------------------------------------------------------------------
template <class T>
__device__ inline void chain_record(const T* th, const Network& net, const RefConsts& ref, T* rec /*[kRecUsed]*/) {
    Tf2Coeffs<T> c;
    tf2_coeffs<T>(th[0], th[1], th[2], th[3], th[4], th[5], c);
    for (int b = 0; b < kTf2Basis; ++b) rec[kRecDc + b] = c.c[b] - ref.c0[b];
    // common complex factor (dL0/dL)(amp/amp0) exp(2i(phic - phic0)) exp(-2 pi i dconst)
    T dconst = c.c_const - ref.c0_const;
    dconst = dconst - rint(val(dconst));  // whole revolutions removed (no derivative)
    const T ang = 2.0 * (th[8] - ref.phic0) - (2.0 * kPi) * dconst;
    const T mag = (ref.dl0 / th[6]) * (c.amp / ref.amp0);
    const Cx<T> common{mag * dcos(ang), mag * dsin(ang)};
    for (int d = 0; d < kMaxDet; ++d) {
        if (d < net.n_det) {
            Proj<T> p;
            project<T>(th[9], th[10], th[11], th[12], net.gmst, net.D[d], net.r[d], p);
            const Cx<T> inv0{T(ref.invC0_re[d]), T(ref.invC0_im[d])};
            const Cx<T> k = cmul(cmul(p.C, inv0), common);
            rec[kRecK + 2 * d] = k.re;
            rec[kRecK + 2 * d + 1] = k.im;
            rec[kRecTau + d] = (th[7] + p.dt) - ref.tau0[d];
        } else {
            rec[kRecK + 2 * d] = T(0.0);
            rec[kRecK + 2 * d + 1] = T(0.0);
            rec[kRecTau + d] = T(0.0);
        }
    }
}

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

template <bool GRAD>
__global__ __launch_bounds__(64) void k_chain_setup(const double* __restrict__ theta, int64_t B, Network net,
                                                    RefConsts ref, double* __restrict__ rec,
                                                    double* __restrict__ jac) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double t[13];
    for (int i = 0; i < 13; ++i) t[i] = theta[b * 13 + i];
    double* out = rec + b * kRecStride;
    const int st = theta_status(t);
    if (st != 1) {
        out[kRecStatus] = st < 0 ? __builtin_nan("") : 0.0;
        for (int i = 1; i < kRecUsed; ++i) out[i] = 0.0;
        if (GRAD)
            for (int i = 0; i < kJacRows * 13; ++i) jac[b * kJacRows * 13 + i] = 0.0;
        return;
    }
    out[kRecStatus] = 1.0;
    if (!GRAD) {
        double r[kRecUsed];
        chain_record<double>(t, net, ref, r);
        for (int i = 1; i < kRecUsed; ++i) out[i] = r[i];
    } else {
        using D13 = Dual<13>;
        D13 td[13];
        for (int i = 0; i < 13; ++i) td[i] = D13::var(t[i], i);
        D13 r[kRecUsed];
        chain_record<D13>(td, net, ref, r);
        double* J = jac + b * kJacRows * 13;
        for (int i = 1; i < kRecUsed; ++i) {
            out[i] = r[i].v;
            for (int k = 0; k < 13; ++k) J[(i - 1) * 13 + k] = r[i].d[k];
        }
    }
}

// ---------------------------------------------------------------------------
// Summary data: one wavefront per item (a run of <= chunk grid points inside
// one bin); the reference waveform is generated inline, once per point, and
// projected onto every detector.  Partials: [item][det][7].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_summary_items(SummaryArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t item = (int64_t)blockIdx.x * 4 + wave_id();
    if (item >= a.n_items) return;
    const int32_t bin = a.item_bin[item];
    const int64_t k0 = a.item_start[item];
    const int32_t cnt = a.item_count[item];
    const double fm = a.f_low + 0.5 * (double)(a.edges[bin] + a.edges[bin + 1]) * a.delta_f;
    double acc[kMaxDet][7];
    for (int d = 0; d < kMaxDet; ++d)
        for (int j = 0; j < 7; ++j) acc[d][j] = 0.0;
    const RefConsts& ref = a.ref;
    const double w = 4.0 * a.delta_f;
    for (int i = lane; i < cnt; i += 64) {
        const int64_t k = k0 + i;
        const double f = a.f_low + (double)k * a.delta_f;
        const double x = cbrt(f);
        const double ix = 1.0 / x;
        const double lx = log(x);
        double bas[kTf2Basis];
        tf2_basis(x, ix, lx, bas);
        double phi = 0.0;
#pragma unroll
        for (int j = 0; j < kTf2Basis; ++j) phi = fma(ref.c0[j], bas[j], phi);
        const double amp = ref.amp0 * (ix * ix * ix) * sqrt(ix);  // f^(-7/6)
        const double df = f - fm;
        for (int d = 0; d < a.n_det; ++d) {
            double cu, su;
            expm2pi_rev(fma(f, ref.tau0[d], phi), cu, su);
            const double hre = amp * (ref.h0fac_re[d] * cu - ref.h0fac_im[d] * su);
            const double him = amp * (ref.h0fac_re[d] * su + ref.h0fac_im[d] * cu);
            const int64_t o = (int64_t)d * a.n_freq + k;
            const double dre = a.data[2 * o], dim = a.data[2 * o + 1];
            const double wk = w / a.psd[o];
            // d conj(h0) w and |h0|^2 w
            const double are = (dre * hre + dim * him) * wk;
            const double aim = (dim * hre - dre * him) * wk;
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
    for (int d = 0; d < a.n_det; ++d)
        for (int j = 0; j < 7; ++j) {
            const double s = wave_sum(acc[d][j]);
            if (lane == 0) a.partials[(item * a.n_det + d) * 7 + j] = s;
        }
}

__global__ void k_summary_reduce(const double* __restrict__ partials, const int64_t* __restrict__ bin_first_item,
                                 int32_t n_bins, int32_t n_det, double* __restrict__ summary) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)n_det * n_bins * 7;
    if (t >= total) return;
    const int j = t % 7;
    const int b = (t / 7) % n_bins;
    const int d = t / (7 * n_bins);
    double s = 0.0;
    for (int64_t it = bin_first_item[b]; it < bin_first_item[b + 1]; ++it) s += partials[(it * n_det + d) * 7 + j];
    summary[((int64_t)d * n_bins + b) * 7 + j] = s;
}

// ---------------------------------------------------------------------------
// Node tables.  With p = r_b, q = r_{b+1}, w = 1/(f_{b+1} - f_b) the bin term
//   Re(A0 r0* + A1 r1*) - B0|r0|^2/2 - B1 Re(r0 r1*) - B2|r1|^2/2
// equals Re(alpha p* + beta q*) - [ |p|^2 (B0/4 - B1 w + B2 w^2)
//   + |q|^2 (B0/4 + B1 w + B2 w^2) + Re(p q*) (B0/2 - 2 B2 w^2) ] / 2
// with alpha = A0/2 - A1 w, beta = A0/2 + A1 w.  Collecting by edge:
//   gamma_j = alpha_j + beta_{j-1},  mu_j = (left part of bin j) + (right part of bin j-1),
//   nu_b = B0/2 - 2 B2 w^2 multiplies Re(r_b r_{b+1}*).
// ---------------------------------------------------------------------------
__global__ void k_node_tables(NodeArgs a) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n_nodes_pad) return;
    const bool real_node = j < a.n_nodes;
    const int nb = a.n_nodes - 1;
    double f = 0.0, x = 1.0, ix = 1.0, lx = 0.0;
    if (real_node) {
        f = a.f_low + (double)a.edges[j] * a.delta_f;
        x = cbrt(f);
        ix = 1.0 / x;
        lx = log(x);
    }
    a.node_f[j] = f;
    a.node_x[j] = x;
    a.node_ix[j] = ix;
    a.node_lx[j] = lx;
    for (int d = 0; d < a.n_det; ++d) {
        double gre = 0.0, gim = 0.0, mu = 0.0, nul = 0.0, nur = 0.0;
        if (real_node) {
            if (j < nb) {  // bin j lies to the right of edge j
                const double* s = a.summary + ((int64_t)d * nb + j) * 7;
                const double w = 1.0 / ((double)(a.edges[j + 1] - a.edges[j]) * a.delta_f);
                const double b2 = a.keep_b2 ? s[6] : 0.0;
                gre += 0.5 * s[0] - s[2] * w;
                gim += 0.5 * s[1] - s[3] * w;
                mu += 0.25 * s[4] - s[5] * w + b2 * w * w;
                nur = 0.5 * s[4] - 2.0 * b2 * w * w;
            }
            if (j > 0) {  // bin j-1 lies to the left
                const double* s = a.summary + ((int64_t)d * nb + (j - 1)) * 7;
                const double w = 1.0 / ((double)(a.edges[j] - a.edges[j - 1]) * a.delta_f);
                const double b2 = a.keep_b2 ? s[6] : 0.0;
                gre += 0.5 * s[0] + s[2] * w;
                gim += 0.5 * s[1] + s[3] * w;
                mu += 0.25 * s[4] + s[5] * w + b2 * w * w;
                nul = 0.5 * s[4] - 2.0 * b2 * w * w;
            }
        }
        const int64_t o = (int64_t)d * a.n_nodes_pad + j;
        a.g_re[o] = gre;
        a.g_im[o] = gim;
        a.mu[o] = mu;
        a.nuL[o] = nul;
        a.nuR[o] = nur;
    }
}

// ---------------------------------------------------------------------------
// Relative-binned likelihood, FP64.  One wavefront per chain; lane l handles
// edge j = 64 t + l of tile t.  The ratio at the edge is r = K_d exp(-2 pi i phi),
// phi = sum_b dc_b B_b(x_j) + f_j dtau_d [rev].  The cross term of bin j-1 uses
// the left neighbour's ratio (shift by one lane; the first lane takes the last
// lane of the previous tile).
// ---------------------------------------------------------------------------
__device__ inline double rec_load(const double* rec, int i) { return rec[i]; }

template <int ND>
__global__ __launch_bounds__(256) void k_loglike_fwd(EventDev ev, const double* __restrict__ recs, int64_t B,
                                                     double* __restrict__ lnl) {
    const int lane = threadIdx.x & 63;
    const int64_t chain = (int64_t)blockIdx.x * 4 + wave_id();
    if (chain >= B) return;
    const double* rec = recs + chain * kRecStride;
    const double status = rec[kRecStatus];
    if (!(status == 1.0)) {
        if (lane == 0) lnl[chain] = (status == 0.0) ? -__builtin_inf() : __builtin_nan("");
        return;
    }
    double dc[kTf2Basis];
#pragma unroll
    for (int j = 0; j < kTf2Basis; ++j) dc[j] = rec[kRecDc + j];
    double kre[ND], kim[ND], dtau[ND], carry_re[ND], carry_im[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        kre[d] = rec[kRecK + 2 * d];
        kim[d] = rec[kRecK + 2 * d + 1];
        dtau[d] = rec[kRecTau + d];
        carry_re[d] = 0.0;
        carry_im[d] = 0.0;
    }
    double acc = 0.0;
    for (int base = 0; base < ev.n_nodes_pad; base += 64) {
        const int j = base + lane;
        const bool live = j < ev.n_nodes;
        const double f = ev.node_f[j];
        double bas[kTf2Basis];
        tf2_basis(ev.node_x[j], ev.node_ix[j], ev.node_lx[j], bas);
        double ph = 0.0;
#pragma unroll
        for (int k = 0; k < kTf2Basis; ++k) ph = fma(dc[k], bas[k], ph);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            double cu, su;
            expm2pi_rev(fma(f, dtau[d], ph), cu, su);
            double rre = kre[d] * cu - kim[d] * su;
            double rim = kre[d] * su + kim[d] * cu;
            if (!live) { rre = 0.0; rim = 0.0; }
            const int64_t o = (int64_t)d * ev.n_nodes_pad + j;
            const double gre = ev.g_re[o], gim = ev.g_im[o], mu = ev.mu[o], nul = ev.nuL[o];
            const double lre = shift_up(rre, carry_re[d], lane);
            const double lim = shift_up(rim, carry_im[d], lane);
            acc += (gre * rre + gim * rim) - 0.5 * mu * (rre * rre + rim * rim)
                 - 0.5 * nul * (lre * rre + lim * rim);
            carry_re[d] = lane_value(rre, 63);
            carry_im[d] = lane_value(rim, 63);
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) lnl[chain] = acc;
}

// ---------------------------------------------------------------------------
// lnL and gradient.  Adjoint of the binned sum with respect to the edge ratios:
//   Gbar_j = gamma_j - mu_j r_j - nuR_j r_{j+1}/2 - nuL_j r_{j-1}/2,
// so that d lnL = sum Re(conj(Gbar_j) d r_j).  With r = K u, u = exp(-2 pi i phi):
//   d lnL/d phi_j = 2 pi Im(conj(Gbar_j) r_j),  d lnL/dK = sum conj(Gbar_j) u_j (as Re(W dK)).
// Accumulated per lane: Z_d = sum conj(Gbar) u, T_d = sum Im(z) f, S_b = sum_j (sum_d Im z) B_b(x_j).
// The right neighbour of a tile's last lane lives in the next tile, so each
// tile is finished one iteration later.  Epilogue: grad = J^T abar.
// ---------------------------------------------------------------------------
template <int ND>
__global__ __launch_bounds__(256) void k_loglike_grad(EventDev ev, const double* __restrict__ recs,
                                                      const double* __restrict__ jac, int64_t B,
                                                      double* __restrict__ lnl, double* __restrict__ grad) {
    const int lane = threadIdx.x & 63;
    const int64_t chain = (int64_t)blockIdx.x * 4 + wave_id();
    if (chain >= B) return;
    const double* rec = recs + chain * kRecStride;
    const double status = rec[kRecStatus];
    if (!(status == 1.0)) {
        if (lane == 0) lnl[chain] = (status == 0.0) ? -__builtin_inf() : __builtin_nan("");
        if (lane < 13) grad[chain * 13 + lane] = (status == 0.0) ? 0.0 : __builtin_nan("");
        return;
    }
    double dc[kTf2Basis];
#pragma unroll
    for (int j = 0; j < kTf2Basis; ++j) dc[j] = rec[kRecDc + j];
    double kre[ND], kim[ND], dtau[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        kre[d] = rec[kRecK + 2 * d];
        kim[d] = rec[kRecK + 2 * d + 1];
        dtau[d] = rec[kRecTau + d];
    }
    // accumulators
    double acc = 0.0;
    double zre[ND], zim[ND], tacc[ND], sacc[kTf2Basis];
#pragma unroll
    for (int d = 0; d < ND; ++d) { zre[d] = 0.0; zim[d] = 0.0; tacc[d] = 0.0; }
#pragma unroll
    for (int k = 0; k < kTf2Basis; ++k) sacc[k] = 0.0;
    // pipeline state: previous tile
    double p_rre[ND], p_rim[ND], p_cu[ND], p_su[ND];
    double cl_re[ND], cl_im[ND];  // left carry (last lane of the tile before the previous one)
#pragma unroll
    for (int d = 0; d < ND; ++d) { p_rre[d] = p_rim[d] = p_cu[d] = p_su[d] = 0.0; cl_re[d] = cl_im[d] = 0.0; }
    double p_f = 0.0, p_x = 1.0, p_ix = 1.0, p_lx = 0.0;
    int p_j = 0;
    const int ntile = ev.n_nodes_pad / 64;
    for (int t = 0; t <= ntile; ++t) {
        double c_rre[ND], c_rim[ND], c_cu[ND], c_su[ND];
        double c_f = 0.0, c_x = 1.0, c_ix = 1.0, c_lx = 0.0;
        const int j = t * 64 + lane;
        if (t < ntile) {
            const bool live = j < ev.n_nodes;
            c_f = ev.node_f[j];
            c_x = ev.node_x[j];
            c_ix = ev.node_ix[j];
            c_lx = ev.node_lx[j];
            double bas[kTf2Basis];
            tf2_basis(c_x, c_ix, c_lx, bas);
            double ph = 0.0;
#pragma unroll
            for (int k = 0; k < kTf2Basis; ++k) ph = fma(dc[k], bas[k], ph);
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                double cu, su;
                expm2pi_rev(fma(c_f, dtau[d], ph), cu, su);
                c_cu[d] = cu;
                c_su[d] = su;
                c_rre[d] = live ? kre[d] * cu - kim[d] * su : 0.0;
                c_rim[d] = live ? kre[d] * su + kim[d] * cu : 0.0;
            }
        } else {
#pragma unroll
            for (int d = 0; d < ND; ++d) c_rre[d] = c_rim[d] = c_cu[d] = c_su[d] = 0.0;
        }
        if (t > 0) {
            // finish the previous tile (edges p_j)
            double qsum = 0.0;
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                const double nx_re = lane_value(c_rre[d], 0), nx_im = lane_value(c_rim[d], 0);
                const double rre = p_rre[d], rim = p_rim[d];
                const double lre = shift_up(rre, cl_re[d], lane), lim = shift_up(rim, cl_im[d], lane);
                const double rgt_re = shift_down(rre, nx_re, lane), rgt_im = shift_down(rim, nx_im, lane);
                const int64_t o = (int64_t)d * ev.n_nodes_pad + p_j;
                const double gre = ev.g_re[o], gim = ev.g_im[o], mu = ev.mu[o];
                const double nul = ev.nuL[o], nur = ev.nuR[o];
                acc += (gre * rre + gim * rim) - 0.5 * mu * (rre * rre + rim * rim)
                     - 0.5 * nul * (lre * rre + lim * rim);
                const double gbre = gre - mu * rre - 0.5 * (nur * rgt_re + nul * lre);
                const double gbim = gim - mu * rim - 0.5 * (nur * rgt_im + nul * lim);
                // conj(Gbar) u and Im(conj(Gbar) r)
                zre[d] += gbre * p_cu[d] + gbim * p_su[d];
                zim[d] += gbre * p_su[d] - gbim * p_cu[d];
                const double imz = gbre * rim - gbim * rre;
                tacc[d] = fma(imz, p_f, tacc[d]);
                qsum += imz;
                cl_re[d] = lane_value(rre, 63);
                cl_im[d] = lane_value(rim, 63);
            }
            double bas[kTf2Basis];
            tf2_basis(p_x, p_ix, p_lx, bas);
#pragma unroll
            for (int k = 0; k < kTf2Basis; ++k) sacc[k] = fma(qsum, bas[k], sacc[k]);
        }
#pragma unroll
        for (int d = 0; d < ND; ++d) { p_rre[d] = c_rre[d]; p_rim[d] = c_rim[d]; p_cu[d] = c_cu[d]; p_su[d] = c_su[d]; }
        p_f = c_f; p_x = c_x; p_ix = c_ix; p_lx = c_lx; p_j = j;
    }
    // wave reductions
    acc = wave_sum(acc);
    double abar[kJacRows];
#pragma unroll
    for (int k = 0; k < kTf2Basis; ++k) abar[kRecDc - 1 + k] = 2.0 * kPi * wave_sum(sacc[k]);
#pragma unroll
    for (int d = 0; d < kMaxDet; ++d) {
        if (d < ND) {
            abar[kRecK - 1 + 2 * d] = wave_sum(zre[d]);
            abar[kRecK - 1 + 2 * d + 1] = -wave_sum(zim[d]);
            abar[kRecTau - 1 + d] = 2.0 * kPi * wave_sum(tacc[d]);
        } else {
            abar[kRecK - 1 + 2 * d] = 0.0;
            abar[kRecK - 1 + 2 * d + 1] = 0.0;
            abar[kRecTau - 1 + d] = 0.0;
        }
    }
    if (lane == 0) lnl[chain] = acc;
    if (lane < 13) {
        const double* J = jac + chain * kJacRows * 13;
        double g = 0.0;
#pragma unroll
        for (int r = 0; r < kJacRows; ++r) g = fma(abar[r], J[r * 13 + lane], g);
        grad[chain * 13 + lane] = g;
    }
}

// ---------------------------------------------------------------------------
// Full-grid likelihood (no binning), FP64: one block of 256 per chain.
// h_d(f) = h0fac_d K_d amp0 f^(-7/6) exp(-2 pi i (sum_b (c0_b + dc_b) B_b(x) + f (tau0_d + dtau_d)))
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_loglike_full(FullArgs a) {
    __shared__ double red[4];
    const int64_t chain = blockIdx.x;
    const double* rec = a.recs + chain * kRecStride;
    const double status = rec[kRecStatus];
    if (!(status == 1.0)) {
        if (threadIdx.x == 0) a.lnl[chain] = (status == 0.0) ? -__builtin_inf() : __builtin_nan("");
        return;
    }
    const RefConsts& ref = a.ref;
    double c[kTf2Basis];
    for (int k = 0; k < kTf2Basis; ++k) c[k] = ref.c0[k] + rec[kRecDc + k];
    double fre[kMaxDet], fim[kMaxDet], tau[kMaxDet];
    for (int d = 0; d < a.n_det; ++d) {
        const double kre = rec[kRecK + 2 * d], kim = rec[kRecK + 2 * d + 1];
        fre[d] = ref.amp0 * (ref.h0fac_re[d] * kre - ref.h0fac_im[d] * kim);
        fim[d] = ref.amp0 * (ref.h0fac_re[d] * kim + ref.h0fac_im[d] * kre);
        tau[d] = ref.tau0[d] + rec[kRecTau + d];
    }
    const double w = 4.0 * a.delta_f;
    double acc = 0.0;
    for (int64_t k = threadIdx.x; k < a.n_freq; k += blockDim.x) {
        const double f = a.f_low + (double)k * a.delta_f;
        const double x = cbrt(f), ix = 1.0 / x, lx = log(x);
        double bas[kTf2Basis];
        tf2_basis(x, ix, lx, bas);
        double ph = 0.0;
        for (int j = 0; j < kTf2Basis; ++j) ph = fma(c[j], bas[j], ph);
        const double am = (ix * ix * ix) * sqrt(ix);
        for (int d = 0; d < a.n_det; ++d) {
            double cu, su;
            expm2pi_rev(fma(f, tau[d], ph), cu, su);
            const double hre = am * (fre[d] * cu - fim[d] * su);
            const double him = am * (fre[d] * su + fim[d] * cu);
            const int64_t o = (int64_t)d * a.n_freq + k;
            const double wk = w / a.psd[o];
            acc += ((a.data[2 * o] * hre + a.data[2 * o + 1] * him) - 0.5 * (hre * hre + him * him)) * wk;
        }
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) a.lnl[chain] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ---------------------------------------------------------------------------
// Projected strain on a grid for one parameter vector (its constants come from
// k_ref_setup run on that vector).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_strain(const RefConsts* __restrict__ cst, int32_t n_det, double f_low,
                                                double delta_f, int64_t n_freq, double* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_freq) return;
    const RefConsts& r = *cst;
    const double f = f_low + (double)k * delta_f;
    const double x = cbrt(f), ix = 1.0 / x, lx = log(x);
    double bas[kTf2Basis];
    tf2_basis(x, ix, lx, bas);
    double ph = 0.0;
    for (int j = 0; j < kTf2Basis; ++j) ph = fma(r.c0[j], bas[j], ph);
    const double am = r.amp0 * (ix * ix * ix) * sqrt(ix);
    for (int d = 0; d < n_det; ++d) {
        double cu, su;
        expm2pi_rev(fma(f, r.tau0[d], ph), cu, su);
        const int64_t o = (int64_t)d * n_freq + k;
        out[2 * o] = am * (r.h0fac_re[d] * cu - r.h0fac_im[d] * su);
        out[2 * o + 1] = am * (r.h0fac_re[d] * su + r.h0fac_im[d] * cu);
    }
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_ref_setup(const double* theta, const Network& net, RefConsts* out_dev, hipStream_t s) {
    Theta13 th;
    for (int i = 0; i < 13; ++i) th.v[i] = theta[i];
    hipLaunchKernelGGL(k_ref_setup, dim3(1), dim3(64), 0, s, th, net, out_dev);
    return hipGetLastError();
}

hipError_t launch_chain_setup(const double* theta, int64_t B, const Network& net, const RefConsts& ref,
                              double* rec, double* jac, hipStream_t s) {
    const unsigned grid = (unsigned)((B + 63) / 64);
    if (jac)
        hipLaunchKernelGGL(k_chain_setup<true>, dim3(grid), dim3(64), 0, s, theta, B, net, ref, rec, jac);
    else
        hipLaunchKernelGGL(k_chain_setup<false>, dim3(grid), dim3(64), 0, s, theta, B, net, ref, rec, jac);
    return hipGetLastError();
}

hipError_t launch_summary(const SummaryArgs& a, const int64_t* bin_first_item, double* summary, hipStream_t s) {
    const unsigned g1 = (unsigned)((a.n_items + 3) / 4);
    hipLaunchKernelGGL(k_summary_items, dim3(g1), dim3(256), 0, s, a);
    const int64_t tot = (int64_t)a.n_det * a.n_bins * 7;
    hipLaunchKernelGGL(k_summary_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a.partials,
                       bin_first_item, a.n_bins, a.n_det, summary);
    return hipGetLastError();
}

hipError_t launch_node_tables(const NodeArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_node_tables, dim3((unsigned)((a.n_nodes_pad + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_loglike(const EventDev& ev, const double* rec, int64_t B, double* lnl, hipStream_t s) {
    const unsigned grid = (unsigned)((B + 3) / 4);
    switch (ev.n_det) {
        case 1: hipLaunchKernelGGL(k_loglike_fwd<1>, dim3(grid), dim3(256), 0, s, ev, rec, B, lnl); break;
        case 2: hipLaunchKernelGGL(k_loglike_fwd<2>, dim3(grid), dim3(256), 0, s, ev, rec, B, lnl); break;
        default: hipLaunchKernelGGL(k_loglike_fwd<3>, dim3(grid), dim3(256), 0, s, ev, rec, B, lnl); break;
    }
    return hipGetLastError();
}

hipError_t launch_loglike_grad(const EventDev& ev, const double* rec, const double* jac, int64_t B, double* lnl,
                               double* grad, hipStream_t s) {
    const unsigned grid = (unsigned)((B + 3) / 4);
    switch (ev.n_det) {
        case 1: hipLaunchKernelGGL(k_loglike_grad<1>, dim3(grid), dim3(256), 0, s, ev, rec, jac, B, lnl, grad); break;
        case 2: hipLaunchKernelGGL(k_loglike_grad<2>, dim3(grid), dim3(256), 0, s, ev, rec, jac, B, lnl, grad); break;
        default: hipLaunchKernelGGL(k_loglike_grad<3>, dim3(grid), dim3(256), 0, s, ev, rec, jac, B, lnl, grad); break;
    }
    return hipGetLastError();
}

hipError_t launch_loglike_full(const FullArgs& a, int64_t B, hipStream_t s) {
    hipLaunchKernelGGL(k_loglike_full, dim3((unsigned)B), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_strain(const RefConsts* cst_dev, int32_t n_det, double f_low, double delta_f, int64_t n_freq,
                         double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_strain, dim3((unsigned)((n_freq + 255) / 256)), dim3(256), 0, s, cst_dev, n_det, f_low,
                       delta_f, n_freq, out);
    return hipGetLastError();
}

}  // namespace rbl
