// Full-band likelihood (Eqs. (2)-(3) over every grid point, no binning) for a batch of chains.
//
//  k_full_consts  per-chain constants of the strain, from the setup record   [1 thread / chain]
//  k_full_tiles   partial lnL of a group of C chains over a tile of grid points
//                 [1 workgroup / (tile, chain group), one grid point per thread at a time]
//  k_full_reduce  lnL of each chain: its tile partials, lane j summing tiles j, j + 64, ... in
//                 order, then the wavefront's fixed reduction tree         [1 wavefront / chain]
//
// A workgroup loads each grid point's data and PSD, and evaluates the chain-independent part
// of the waveform there (x = f^(1/3), 1/x, ln x, f^(-7/6), the TaylorF2 basis or x^5.78),
// once for its C chains; per chain and detector it then forms
//   h_d(f) = F_d f^(-7/6) a(f) exp(-2 pi i (Phi(f) + f tau_d)),   F_d = amp0 h0fac_d K_d,
// and accumulates (Re(d h*) - |h|^2 / 2) 4 df / S.  The chain constants are wave-uniform
// (scalar loads); the unit phasors come from the LDS table as in the other kernels.
// Consecutive workgroups take the same tile for different chain groups, so a tile's data is
// read from HBM about once per XCD.  Every sum has a fixed order: bitwise reproducible.
#include "rbl_launch.h"
#include "rbl_phasor.h"
#include "rbl_wave.h"

namespace rbl {

namespace {

constexpr int kFullTileThreads = 256;

// Per-chain constants [kFullStride doubles]: status, F_d (re, im), tau_d in table units,
// TaylorF2 coefficients in table units, IMRPhenomD_NRTidalv2 node parameters.
constexpr int kFcStatus = 0, kFcFre = 1, kFcFim = 4, kFcTau = 7, kFcC = 10, kFcNrt = 20;
static_assert(kFcNrt + kNrtParams <= kFullStride, "full-band constant block");

__global__ __launch_bounds__(64) void k_full_consts(const double* __restrict__ recs, int64_t B, RefConsts ref,
                                                    int32_t n_det, double* __restrict__ out) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double* rec = recs + b * kRecStride;
    double* o = out + b * kFullStride;
    o[kFcStatus] = rec[kRecStatus];
    const double g_re = rec[kRecG], g_im = rec[kRecG + 1];
    for (int d = 0; d < kMaxDet; ++d) {
        double fre = 0.0, fim = 0.0, tau = 0.0;
        if (d < n_det) {
            const double pr = rec[kRecK + 2 * d], pi = rec[kRecK + 2 * d + 1];
            const double kre = pr * g_re - pi * g_im, kim = pr * g_im + pi * g_re;  // K_d = P_d G
            fre = ref.amp0 * (ref.h0fac_re[d] * kre - ref.h0fac_im[d] * kim);
            fim = ref.amp0 * (ref.h0fac_re[d] * kim + ref.h0fac_im[d] * kre);
            tau = ref.tau0[d] * (double)kPhasorN + rec[kRecTau + d];
        }
        o[kFcFre + d] = fre;
        o[kFcFim + d] = fim;
        o[kFcTau + d] = tau;
    }
    for (int k = 0; k < kTf2Basis; ++k) o[kFcC + k] = ref.c0[k] * (double)kPhasorN + rec[kRecDc + k];
    for (int i = 0; i < kNrtParams; ++i) o[kFcNrt + i] = rec[kRecNrt + i];
}

template <int ND, int WF, int C>
__global__ __launch_bounds__(kFullTileThreads) void k_full_tiles(FullTileArgs a) {
    __shared__ double2 tab[kPhasorN];
    __shared__ double red[kFullTileThreads / 64][C];
    load_phasor_table(a.phasor, tab);
    const int64_t g = (int64_t)blockIdx.x % a.n_groups;
    const int64_t t = (int64_t)blockIdx.x / a.n_groups;
    const int64_t c0 = g * C;
    const int nc = (int)((a.B - c0) < C ? (a.B - c0) : C);
    const int64_t k_begin = t * a.tile_points;
    const int64_t k_end = (k_begin + a.tile_points) < a.n_freq ? (k_begin + a.tile_points) : a.n_freq;
    const double w0 = 4.0 * a.delta_f;
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0;
    for (int64_t k = k_begin + threadIdx.x; k < k_end; k += kFullTileThreads) {
        const double f = a.f_low + (double)k * a.delta_f;
        const double x = cbrt(f);
        const double ix = 1.0 / x;
        const double lx = log(x);
        const double am = (ix * ix * ix) * sqrt(ix);  // f^(-7/6)
        double bas[kTf2Basis];
        double x578 = 0.0;
        if constexpr (WF == kWfNrtv2)
            x578 = exp(5.78 * lx);
        else
            tf2_basis(x, ix, lx, bas);
        double dre[ND], dim[ND], wk[ND];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const int64_t o = (int64_t)d * a.n_freq + k;
            const double2 dd = reinterpret_cast<const double2*>(a.data)[o];
            dre[d] = dd.x;
            dim[d] = dd.y;
            wk[d] = w0 / a.psd[o];
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (c >= nc) break;  // wave-uniform
            const double* cc = a.consts + (c0 + c) * kFullStride;
            if (!(cc[kFcStatus] == 1.0)) continue;
            double ph, amp;
            if constexpr (WF == kWfNrtv2) {
                double ar;
                nrt_node(*reinterpret_cast<const NrtParams<double>*>(cc + kFcNrt), f, x, ix, lx, x578, true, ph, ar);
                ph *= (double)kPhasorN;
                amp = am * ar;
            } else {
                ph = 0.0;
#pragma unroll
                for (int b = 0; b < kTf2Basis; ++b) ph = fma(cc[kFcC + b], bas[b], ph);
                amp = am;
            }
            double s = 0.0;
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                double cu, su;
                unit_phasor(fma(f, cc[kFcTau + d], ph), tab, cu, su);
                const double fr = amp * cc[kFcFre + d], fi = amp * cc[kFcFim + d];
                const double hre = fr * cu - fi * su;
                const double him = fr * su + fi * cu;
                s = fma(fma(dre[d], hre, fma(dim[d], him, -0.5 * fma(hre, hre, him * him))), wk[d], s);
            }
            acc[c] += s;
        }
    }
    constexpr int NV = (C + 3) / 4 * 4;
    double part[NV], tot[NV];
#pragma unroll
    for (int c = 0; c < NV; ++c) part[c] = c < C ? acc[c] : 0.0;
    wave_sum_n<NV>(part, tot);
    const int wid = wave_id();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int c = 0; c < C; ++c) red[wid][c] = tot[c];
    }
    __syncthreads();
    if ((int)threadIdx.x < nc)
        a.partials[(c0 + threadIdx.x) * a.n_tiles + t] =
            ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) + red[3][threadIdx.x];
}

__global__ __launch_bounds__(256) void k_full_reduce(const double* __restrict__ partials,
                                                     const double* __restrict__ consts, int64_t B, int64_t n_tiles,
                                                     double* __restrict__ lnl) {
    const int64_t b = (int64_t)blockIdx.x * 4 + wave_id();
    if (b >= B) return;  // wave-uniform
    const int lane = threadIdx.x & 63;
    const double status = consts[b * kFullStride + kFcStatus];
    if (!(status == 1.0)) {
        if (lane == 0) lnl[b] = (status == 0.0) ? -__builtin_inf() : __builtin_nan("");
        return;
    }
    const double* p = partials + b * n_tiles;
    double s = 0.0;
    for (int64_t t = lane; t < n_tiles; t += 64) s += p[t];
    s = wave_sum(s);
    if (lane == 0) lnl[b] = s;
}

template <int ND, int WF, int C>
void launch_tiles(const FullTileArgs& a, hipStream_t s, KTime kt) {
    launch_k(k_full_tiles<ND, WF, C>, dim3((unsigned)(a.n_groups * a.n_tiles)), dim3(kFullTileThreads), s, kt, a);
}

}  // namespace

FullPlan full_plan(int64_t n_freq, int64_t B, int32_t waveform) {
    FullPlan p;
    p.chains_per_group = waveform == kWfNrtv2 ? kFullGroupNrt : kFullGroupTf2;
    p.n_groups = (B + p.chains_per_group - 1) / p.chains_per_group;
    // points per thread: enough workgroups to fill the chip (about 16 per CU), at most 16
    const int64_t target = 4096;
    int64_t per_thread = (n_freq * p.n_groups + (int64_t)kFullTileThreads * target - 1) /
                         ((int64_t)kFullTileThreads * target);
    per_thread = per_thread < 1 ? 1 : (per_thread > 16 ? 16 : per_thread);
    p.tile_points = per_thread * kFullTileThreads;
    p.n_tiles = (n_freq + p.tile_points - 1) / p.tile_points;
    return p;
}

hipError_t launch_loglike_full(const FullArgs& f, int64_t B, double* consts, double* partials, hipStream_t s,
                               KTime kt) {
    const FullPlan p = full_plan(f.n_freq, B, f.ref.waveform);
    hipLaunchKernelGGL(k_full_consts, dim3((unsigned)((B + 63) / 64)), dim3(64), 0, s, f.recs, B, f.ref, f.n_det,
                       consts);
    FullTileArgs a{};
    a.consts = consts;
    a.partials = partials;
    a.phasor = f.phasor;
    a.data = f.data;
    a.psd = f.psd;
    a.B = B;
    a.n_freq = f.n_freq;
    a.f_low = f.f_low;
    a.delta_f = f.delta_f;
    a.tile_points = p.tile_points;
    a.n_tiles = p.n_tiles;
    a.n_groups = p.n_groups;
    const bool nrt = f.ref.waveform == kWfNrtv2;
    switch (f.n_det) {
        case 1: nrt ? launch_tiles<1, kWfNrtv2, kFullGroupNrt>(a, s, kt) : launch_tiles<1, kWfTaylorF2, kFullGroupTf2>(a, s, kt); break;
        case 2: nrt ? launch_tiles<2, kWfNrtv2, kFullGroupNrt>(a, s, kt) : launch_tiles<2, kWfTaylorF2, kFullGroupTf2>(a, s, kt); break;
        default: nrt ? launch_tiles<3, kWfNrtv2, kFullGroupNrt>(a, s, kt) : launch_tiles<3, kWfTaylorF2, kFullGroupTf2>(a, s, kt); break;
    }
    hipLaunchKernelGGL(k_full_reduce, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, s, partials, consts, B, p.n_tiles,
                       f.lnl);
    return hipGetLastError();
}

}  // namespace rbl
