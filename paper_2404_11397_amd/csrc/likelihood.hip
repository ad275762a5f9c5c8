// Relative-binned likelihood kernels (gfx950, wave64): lnL, and lnL with the adjoint
// gradient, each in FP64 or mixed precision.
//
// One wavefront per chain.  TaylorF2: lane l walks its L consecutive bin edges
// j = l L + k (k = 0..L-1) in the lane-contiguous table layout; IMRPhenomD_NRTidalv2:
// step k covers edges 64k .. 64k+63 (natural order).  At each edge the ratio of
// Eq. (4) is r_d = K_d exp(-2 pi i phi_d), phi_d = sum_b dc_b B_b(x_j) + f_j dtau_d
// (revolutions; times a / a0 for IMRPhenomD_NRTidalv2), and the binned sum of Eq. (5)
// is regrouped per edge:
//   2 lnL = sum_d sum_j [ 2 Re(gamma_dj r_dj*) - mu_dj |r_dj|^2 + xL_dj Re(r_d,j-1 r_dj*) ],
// xL_dj being the cross weight of the bin left of edge j.  The TaylorF2 walks keep K_d
// out of the per-edge products and apply it after the wavefront reduction.
//
// FP64 unit phasors come from a kPhasorN-entry table in LDS and a short Taylor
// rotation (unit_phasor, rbl_phasor.h).
//
// The FP64 TaylorF2 kernels and the IMRPhenomD_NRTidalv2 gradient kernels stage the
// event's edge tables in LDS per workgroup of kStageChains chains, in one memory round
// trip (stage_tf2_workgroup, stage_nrt_tables); the TaylorF2 gradient kernel stages its
// chains' Jacobian entries and records with them.
//
// Mixed precision: the phase is accumulated in FP64 and reduced to (-1/2, 1/2]
// revolutions in FP64; sin/cos (hardware, revolution argument), the ratio and the
// per-edge products are FP32; every per-edge term is added to an FP64 accumulator.
// A chain whose binned-sum magnitude bound exceeds kMixedScaleMax takes the FP64
// path (a wavefront-uniform branch).
#include "rbl_launch.h"
#include "rbl_phasor.h"
#include "rbl_wave.h"

namespace rbl {

// Mixed precision: the hardware FP32 sin / cos on the reduced phase.
__device__ inline void unit_phasor(double y, const double2*, float& c, float& s) {
    const double phi = y * (1.0 / kPhasorN);
    const float t = (float)(phi - rint(phi));  // exact reduction in FP64, then rounded once
    c = __builtin_amdgcn_cosf(t);              // v_cos_f32: cos(2 pi t)
    s = -__builtin_amdgcn_sinf(t);             // v_sin_f32: sin(2 pi t)
}

template <class R>
struct EdgeTab {
    const R *g, *mu, *xl;  // g: gamma as (re, im) pairs
};
__device__ inline EdgeTab<double> edge_tab(const EventDev& ev, double) { return {ev.g, ev.mu, ev.xL}; }
__device__ inline EdgeTab<float> edge_tab(const EventDev& ev, float) { return {ev.g32, ev.mu32, ev.xL32}; }
// xR_j = xL_{j+1}: the cross weight of the bin right of edge j
__device__ inline const double* xr_tab(const EventDev& ev, double) { return ev.xR; }
__device__ inline const float* xr_tab(const EventDev& ev, float) { return ev.xR32; }

__device__ inline void load_phasor_table(const EventDev& ev, double2* tab) { load_phasor_table(ev.phasor, tab); }

// Table load with a 32-bit byte offset: lets the compiler address every table of a step
// from its scalar base plus one shared vector offset (global_load ... saddr).
template <class T>
__device__ inline T ld(const T* base, unsigned idx) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + idx * (unsigned)sizeof(T));
}
// The idx-th (re, im) pair of an interleaved table.
__device__ inline double2 ld2(const double* base, unsigned idx) {
    return *reinterpret_cast<const double2*>(reinterpret_cast<const char*>(base) + idx * 16u);
}
__device__ inline float2 ld2(const float* base, unsigned idx) {
    return *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(base) + idx * 8u);
}

// One edge of the node table: f, x = f^(1/3), 1/x, ln x.
struct Node {
    double f, x, ix, lx;
};
__device__ inline Node ld_node(const EventDev& ev, unsigned pos) {
    const double2 a = ld2(ev.node_fx, pos), b = ld2(ev.node_il, pos);
    return {a.x, a.y, b.x, b.y};
}

// Per-chain values shared by the walks.  dc and dtau are in table units, as in the record.
template <int ND>
struct ChainVals {
    double dc[kTf2Basis];
    double kre[ND], kim[ND], dtau[ND];
    NrtParams<double> np;  // IMRPhenomD_NRTidalv2 events only
};

// Accumulation helpers of the TaylorF2 walks: fused in FP64; in the mixed form the product
// is formed in FP32 and added to the FP64 accumulator.
__device__ inline void acc_dot(double& a, double x1, double y1, double x2, double y2) { a = fma(x1, y1, fma(x2, y2, a)); }
__device__ inline void acc_dot(double& a, float x1, float y1, float x2, float y2) { a += (double)(x1 * y1 + x2 * y2); }
__device__ inline void acc_mul(double& a, double x, double y) { a = fma(x, y, a); }
__device__ inline void acc_mul(double& a, float x, double y) { a = fma((double)x, y, a); }

// The amplitude ratio of an IMRPhenomD_NRTidalv2 chain to the reference stays below
// about 1.1 in band; the bound takes it as 2.
template <int ND>
__device__ inline bool use_mixed(const EventDev& ev, const ChainVals<ND>& cv) {
    const double amax = ev.waveform == kWfNrtv2 ? 2.0 : 1.0;
    double bound = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const double k2 = (cv.kre[d] * cv.kre[d] + cv.kim[d] * cv.kim[d]) * amax * amax;
        bound += sqrt(k2) * ev.scales[2 * d] + k2 * ev.scales[2 * d + 1];
    }
    return bound <= kMixedScaleMax;
}

// Edge phase (table units, relative to the reference) and amplitude ratio.
//   TaylorF2:  sum_b dc_b B_b(x), ratio 1 (the Mc^(5/6) factor is in K);
//   IMRPhenomD_NRTidalv2:  Phi(f; theta) - Phi0_j, ratio a(f; theta) / a0_j.
template <int ND, int WF>
__device__ inline void edge_phase(const EventDev& ev, const ChainVals<ND>& cv, unsigned pos, const Node& n, double& dph,
                                  double& ar) {
    if (WF == kWfNrtv2) {
        double ph, a;
        nrt_node(cv.np, n.f, n.x, n.ix, n.lx, ld(ev.node_x578, pos), true, ph, a);
        dph = (ph - ld(ev.phi0, pos)) * (double)kPhasorN;
        ar = a * ld(ev.ia0, pos);
    } else {
        double bas[kTf2Basis];
        tf2_basis(n.x, n.ix, n.lx, bas);
        double ph = -0.0;
#pragma unroll
        for (int b = 0; b < kTf2Basis; ++b) ph = fma(cv.dc[b], bas[b], ph);
        dph = ph;
        ar = 1.0;
    }
}

// ---------------------------------------------------------------------------
// TaylorF2 forward walk.  r_dj = K_d u_dj with u_dj the unit phasor of the edge phase, so
// K_d factors out of every per-edge product: this lane's share of lnL without the quadratic
// term is
//   sum_d [ Re(K_d P_d) + |K_d|^2 X_d / 2 ],  P_d = sum_j conj(gamma_dj) u_dj,
//   X_d = sum_j xL_dj Re(u_d,j-1 u_dj*),
// and the quadratic term is -sum_d |K_d|^2 M_d / 2 (|r_dj| = |K_d|).  The cross term of the
// bin left of a lane's first edge needs the last edge of lane - 1: exchanged once at the end.
// ---------------------------------------------------------------------------
template <int ND, class R>
__device__ inline double fwd_walk(const EventDev& ev, const ChainVals<ND>& cv, const double2* tab, int lane) {
    const EdgeTab<R> T = edge_tab(ev, R(0));
    const int npad = ev.n_nodes_pad;
    R pre[ND], pim[ND], fre[ND], fim[ND];
    double Pr[ND], Pi[ND], X[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        pre[d] = pim[d] = fre[d] = fim[d] = R(0);
        Pr[d] = Pi[d] = X[d] = 0.0;
    }
    for (int k = 0; k < ev.L; ++k) {
        const unsigned pos = (unsigned)(k * 64 + lane);
        const Node n = ld_node(ev, pos);
        const double f = n.f;
        double bas[kTf2Basis];
        tf2_basis(n.x, n.ix, n.lx, bas);
        double ph = -0.0;
#pragma unroll
        for (int b = 0; b < kTf2Basis; ++b) ph = fma(cv.dc[b], bas[b], ph);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            R ur, ui;
            unit_phasor(fma(f, cv.dtau[d], ph), tab, ur, ui);
            const unsigned o = (unsigned)(d * npad) + pos;
            const auto g = ld2(T.g, o);
            const R gre = g.x, gim = g.y;
            acc_dot(Pr[d], gre, ur, gim, ui);
            acc_dot(Pi[d], gre, ui, -gim, ur);
            if (k > 0) {
                acc_mul(X[d], pre[d] * ur + pim[d] * ui, (double)ld(T.xl, o));
            } else {
                fre[d] = ur;
                fim[d] = ui;
            }
            pre[d] = ur;
            pim[d] = ui;
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const R lre = shift_up(pre[d], R(0), lane), lim = shift_up(pim[d], R(0), lane);
        acc_mul(X[d], lre * fre[d] + lim * fim[d], (double)ld(T.xl, (unsigned)(d * npad + lane)));
        const double k2 = cv.kre[d] * cv.kre[d] + cv.kim[d] * cv.kim[d];
        acc = fma(cv.kre[d], Pr[d], fma(-cv.kim[d], Pi[d], fma(0.5 * k2, X[d], acc)));
    }
    return acc;
}

// The quadratic term of a TaylorF2 chain, -sum_d |K_d|^2 M_d / 2.
template <int ND>
__device__ inline double tf2_quadratic(const EventDev& ev, const ChainVals<ND>& cv) {
    double q = 0.0;
#pragma unroll
    for (int d = 0; d < ND; ++d) q = fma(cv.kre[d] * cv.kre[d] + cv.kim[d] * cv.kim[d], ev.mu_sum[d], q);
    return -0.5 * q;
}

// IMRPhenomD_NRTidalv2 events keep their edge tables in natural order (edge j at
// position j): step k covers edges 64k .. 64k+63, so the lanes of a wavefront sit in
// the same region of the piecewise model (phase regions, taper) and branch together.
// The left neighbour of an edge is the previous lane, or for lane 0 the last lane of
// the previous step (a wave-uniform carry).
template <int ND, class R>
__device__ inline void nrt_ratio(const EventDev& ev, const ChainVals<ND>& cv, const NrtParams<double>& np,
                                 const double2* tab, unsigned pos,
                                 const R* kre, const R* kim, R* rre, R* rim, double& a, NrtShared* sh = nullptr) {
    const Node n = ld_node(ev, pos);
    const double f = n.f;
    double ph;
    nrt_node(np, f, n.x, n.ix, n.lx, ld(ev.node_x578, pos), true, ph, a, sh);
    const double dph = (ph - ld(ev.phi0, pos)) * (double)kPhasorN;
    const R ar = (R)(a * ld(ev.ia0, pos));
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        R cu, su;
        unit_phasor(fma(f, cv.dtau[d], dph), tab, cu, su);
        cu *= ar;
        su *= ar;
        rre[d] = kre[d] * cu - kim[d] * su;
        rim[d] = kre[d] * su + kim[d] * cu;
    }
}

template <int ND, class R>
__device__ inline double fwd_walk_natural(const EventDev& ev, const ChainVals<ND>& cv, const double2* tab, int lane) {
    const EdgeTab<R> T = edge_tab(ev, R(0));
    const int npad = ev.n_nodes_pad;
    R kre[ND], kim[ND], pre[ND], pim[ND];  // pre/pim: the previous step's ratios
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        kre[d] = (R)cv.kre[d];
        kim[d] = (R)cv.kim[d];
        pre[d] = pim[d] = R(0);
    }
    double acc = 0.0;
    for (int k = 0; k < ev.L; ++k) {
        const unsigned pos = (unsigned)(k * 64 + lane);
        R rre[ND], rim[ND];
        double a;
        nrt_ratio<ND, R>(ev, cv, cv.np, tab, pos, kre, kim, rre, rim, a);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const R lre = left_neighbour(rre[d], pre[d]), lim = left_neighbour(rim[d], pim[d]);
            const unsigned o = (unsigned)(d * npad) + pos;
            const auto g = ld2(T.g, o);
            const R gr = g.x * rre[d] + g.y * rim[d];
            const R h = fma(ld(T.xl, o), lre * rre[d] + lim * rim[d], -(ld(T.mu, o) * (rre[d] * rre[d] + rim[d] * rim[d])));
            acc += (double)fma(R(0.5), h, gr);
            pre[d] = rre[d];
            pim[d] = rim[d];
        }
    }
    return acc;
}

// LDS staging limits and the workgroup shape of the LDS-table kernels.
constexpr size_t kStageMaxBytes = 56 * 1024;  // with the 8 KB phasor table: two workgroups per CU
constexpr int kStageChains = 8;               // chains (wavefronts) per workgroup sharing the staged tables
constexpr size_t kNrtStageMaxBytes = 144 * 1024;  // with the phasor table and node parameters: one workgroup per CU
// TaylorF2 edge tables staged in LDS, shared by the workgroup's chains: the node pairs, the
// gamma pairs and x_L of the first ND detectors (npad (4 + 3 ND) doubles); the walk then
// reads them with LDS loads instead of vector-memory loads.  ev's pointers are redirected.
template <int ND>
__device__ inline void stage_edge_tables(EventDev& ev, double* lds) {
    const int np = ev.n_nodes_pad;
    double* fx = lds;
    double* il = fx + 2 * np;
    double* g = il + 2 * np;
    double* xl = g + 2 * ND * np;
    const double2* sfx = reinterpret_cast<const double2*>(ev.node_fx);
    const double2* sil = reinterpret_cast<const double2*>(ev.node_il);
    const double2* sg = reinterpret_cast<const double2*>(ev.g);
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        reinterpret_cast<double2*>(fx)[i] = sfx[i];
        reinterpret_cast<double2*>(il)[i] = sil[i];
    }
    for (int i = threadIdx.x; i < ND * np; i += blockDim.x) {
        reinterpret_cast<double2*>(g)[i] = sg[i];
        xl[i] = ev.xL[i];
    }
    __syncthreads();
    ev.node_fx = fx;
    ev.node_il = il;
    ev.g = g;
    ev.xL = xl;
}
// IMRPhenomD_NRTidalv2 edge tables staged in LDS for the gradient walk: the gamma pairs,
// mu, x_L and x_R of the first ND detectors (5 ND npad doubles), natural order.
template <int ND>
__device__ inline void stage_nrt_tables(EventDev& ev, double2* tab, double* lds) {
    // One memory round trip, as in stage_tf2_workgroup: every load (the unit-phasor table
    // too) is issued, at an index clamped into its array, before the first LDS write.
    constexpr int T = 64 * kStageChains;
    constexpr int NPMAX = (int)(kNrtStageMaxBytes / (sizeof(double) * (5 * ND + 3))) / kNodeTile * kNodeTile;
    constexpr int NT = (kPhasorN + T - 1) / T, NA = (ND * NPMAX + T - 1) / T, NB = (NPMAX + T - 1) / T;
    const int t = threadIdx.x, np = ev.n_nodes_pad;
    double* g = lds;
    double* mu = g + 2 * ND * np;
    double* xl = mu + ND * np;
    double* xr = xl + ND * np;
    double* p0 = xr + ND * np;
    double* a0 = p0 + np;
    double* x5 = a0 + np;
    const double2* sph = reinterpret_cast<const double2*>(ev.phasor);
    const double2* sg = reinterpret_cast<const double2*>(ev.g);
    double phx[NT], phy[NT], gx[NA], gy[NA], vmu[NA], vxl[NA], vxr[NA], vp0[NB], va0[NB], vx5[NB];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const double2 v = sph[min(k * T + t, kPhasorN - 1)];
        phx[k] = v.x;
        phy[k] = v.y;
    }
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const int i = min(k * T + t, ND * np - 1);
        const double2 v = sg[i];
        gx[k] = v.x;
        gy[k] = v.y;
        vmu[k] = ev.mu[i];
        vxl[k] = ev.xL[i];
        vxr[k] = ev.xR[i];
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int i = min(k * T + t, np - 1);
        vp0[k] = ev.phi0[i];
        va0[k] = ev.ia0[i];
        vx5[k] = ev.node_x578[i];
    }
    __builtin_amdgcn_sched_barrier(0);  // every load above is issued before the first store
#pragma unroll
    for (int k = 0; k < NT; ++k)
        if (k * T + t < kPhasorN) tab[k * T + t] = double2{phx[k], phy[k]};
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const int i = k * T + t;
        if (i < ND * np) {
            reinterpret_cast<double2*>(g)[i] = double2{gx[k], gy[k]};
            mu[i] = vmu[k];
            xl[i] = vxl[k];
            xr[i] = vxr[k];
        }
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int i = k * T + t;
        if (i < np) {
            p0[i] = vp0[k];
            a0[i] = va0[k];
            x5[i] = vx5[k];
        }
    }
    __syncthreads();
    ev.phi0 = p0;
    ev.ia0 = a0;
    ev.node_x578 = x5;
    ev.g = g;
    ev.mu = mu;
    ev.xL = xl;
    ev.xR = xr;
}
inline size_t staged_nrt_table_bytes(int nd, int np) { return sizeof(double) * (size_t)np * (5 * (size_t)nd + 3); }
// The mixed-precision walk's FP32 tables (gamma pairs, mu, x_L, x_R) and the FP64 reference
// phase, inverse amplitude and x^5.78; a chain that takes the FP64 branch reads the FP64
// tables from global memory.
template <int ND>
__device__ inline void stage_nrt_tables32(EventDev& ev, double2* tab, double* lds) {
    // One memory round trip, as in stage_nrt_tables.
    constexpr int T = 64 * kStageChains;
    constexpr int NPMAX = (int)(kNrtStageMaxBytes / (20 * ND + 24)) / kNodeTile * kNodeTile;
    constexpr int NT = (kPhasorN + T - 1) / T, NA = (ND * NPMAX + T - 1) / T, NB = (NPMAX + T - 1) / T;
    const int t = threadIdx.x, np = ev.n_nodes_pad;
    double* p0 = lds;
    double* a0 = p0 + np;
    double* x5 = a0 + np;
    float* g = reinterpret_cast<float*>(x5 + np);
    float* mu = g + 2 * ND * np;
    float* xl = mu + ND * np;
    float* xr = xl + ND * np;
    const double2* sph = reinterpret_cast<const double2*>(ev.phasor);
    const float2* sg = reinterpret_cast<const float2*>(ev.g32);
    double phx[NT], phy[NT], vp0[NB], va0[NB], vx5[NB];
    float gx[NA], gy[NA], vmu[NA], vxl[NA], vxr[NA];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const double2 v = sph[min(k * T + t, kPhasorN - 1)];
        phx[k] = v.x;
        phy[k] = v.y;
    }
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const int i = min(k * T + t, ND * np - 1);
        const float2 v = sg[i];
        gx[k] = v.x;
        gy[k] = v.y;
        vmu[k] = ev.mu32[i];
        vxl[k] = ev.xL32[i];
        vxr[k] = ev.xR32[i];
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int i = min(k * T + t, np - 1);
        vp0[k] = ev.phi0[i];
        va0[k] = ev.ia0[i];
        vx5[k] = ev.node_x578[i];
    }
    __builtin_amdgcn_sched_barrier(0);  // every load above is issued before the first store
#pragma unroll
    for (int k = 0; k < NT; ++k)
        if (k * T + t < kPhasorN) tab[k * T + t] = double2{phx[k], phy[k]};
#pragma unroll
    for (int k = 0; k < NA; ++k) {
        const int i = k * T + t;
        if (i < ND * np) {
            reinterpret_cast<float2*>(g)[i] = float2{gx[k], gy[k]};
            mu[i] = vmu[k];
            xl[i] = vxl[k];
            xr[i] = vxr[k];
        }
    }
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int i = k * T + t;
        if (i < np) {
            p0[i] = vp0[k];
            a0[i] = va0[k];
            x5[i] = vx5[k];
        }
    }
    __syncthreads();
    ev.phi0 = p0;
    ev.ia0 = a0;
    ev.node_x578 = x5;
    ev.g32 = g;
    ev.mu32 = mu;
    ev.xL32 = xl;
    ev.xR32 = xr;
}
inline size_t staged_nrt_table32_bytes(int nd, int np) { return (size_t)np * (20 * (size_t)nd + 24); }

// LDS bytes of the staged tables.
inline size_t staged_table_bytes(int nd, int np) { return sizeof(double) * (size_t)np * (4 + 3 * (size_t)nd); }

// Jacobian entries the TaylorF2 gradient epilogue reads per chain: the intrinsic block
// (12 rows of 6) and the extrinsic block (9 rows of 4).
constexpr int kJacTf2Int = 12 * 6, kJacTf2 = kJacTf2Int + 36;

// The LDS staging of an 8-chain TaylorF2 workgroup in one memory round trip: every thread
// first issues all of its loads -- the unit-phasor table, the node pairs, the gamma pairs and
// x_L, with NJ > 0 the Jacobian entries of the workgroup's chains (NJ per chain, to sj) and
// with NR > 0 the first NR entries of their records (to sr) -- and only then writes them to
// LDS, followed by one barrier.  A loop that loads and stores
// each element in turn waits one round trip per iteration; the workgroups of a CU run one
// after another, so each of those waits is exposed.  The per-thread counts are bounded by
// the staging limit (npad (4 + 3 ND) doubles <= kStageMaxBytes).  ev's pointers are
// redirected to LDS.
template <int ND, int NJ, int NR = 0>
__device__ inline void stage_tf2_workgroup(EventDev& ev, double2* tab, double* lds, const double* __restrict__ jac,
                                           int64_t chain0, int64_t B, double* sj, const double* __restrict__ recs = nullptr,
                                           double* sr = nullptr) {
    constexpr int T = 64 * kStageChains;
    static_assert(kStageChains * NR <= T, "one record entry per thread");
    constexpr int NPMAX = (int)(kStageMaxBytes / (sizeof(double) * (4 + 3 * ND))) / kNodeTile * kNodeTile;
    constexpr int NT = (kPhasorN + T - 1) / T, NF = (NPMAX + T - 1) / T, NG = (ND * NPMAX + T - 1) / T;
    constexpr int NJT = NJ > 0 ? (kStageChains * NJ + T - 1) / T : 1;
    const int t = threadIdx.x, np = ev.n_nodes_pad;
    const double2* sph = reinterpret_cast<const double2*>(ev.phasor);
    const double2* sfx = reinterpret_cast<const double2*>(ev.node_fx);
    const double2* sil = reinterpret_cast<const double2*>(ev.node_il);
    const double2* sg = reinterpret_cast<const double2*>(ev.g);
    // Loads are unconditional, at indices clamped into the arrays (a clamped element is loaded
    // and not stored), and pairs are held as separate x / y doubles: a load under a branch, or
    // into a vector-typed array, makes the compiler wait for it before the next one.
    double phx[NT], phy[NT], fxx[NF], fxy[NF], ilx[NF], ily[NF], gx[NG], gy[NG], vxl[NG], vj[NJT], vr = 0.0;
#pragma unroll
    for (int k = 0; k < NT; ++k) {
        const double2 v = sph[min(k * T + t, kPhasorN - 1)];
        phx[k] = v.x;
        phy[k] = v.y;
    }
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        const int i = min(k * T + t, np - 1);
        const double2 u = sfx[i], v = sil[i];
        fxx[k] = u.x;
        fxy[k] = u.y;
        ilx[k] = v.x;
        ily[k] = v.y;
    }
#pragma unroll
    for (int k = 0; k < NG; ++k) {
        const int i = min(k * T + t, ND * np - 1);
        const double2 v = sg[i];
        gx[k] = v.x;
        gy[k] = v.y;
        vxl[k] = ev.xL[i];
    }
    if constexpr (NJ > 0) {
#pragma unroll
        for (int k = 0; k < NJT; ++k) {
            const int e = min(k * T + t, kStageChains * NJ - 1), c = e / NJ, j = e - c * NJ;
            const int64_t ch = min(chain0 + c, B - 1);
            vj[k] = jac[ch * kJacStride + (j < kJacTf2Int ? kJacInt + j : kJacExt + (j - kJacTf2Int))];
        }
    }
    if constexpr (NR > 0) {
        const int e = min(t, kStageChains * NR - 1), c = e / NR;
        vr = recs[min(chain0 + c, B - 1) * kRecStride + (e - c * NR)];
    }
    __builtin_amdgcn_sched_barrier(0);  // every load above is issued before the first store
    double* fx = lds;
    double* il = fx + 2 * np;
    double* g = il + 2 * np;
    double* xl = g + 2 * ND * np;
#pragma unroll
    for (int k = 0; k < NT; ++k)
        if (k * T + t < kPhasorN) tab[k * T + t] = double2{phx[k], phy[k]};
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        const int i = k * T + t;
        if (i < np) {
            reinterpret_cast<double2*>(fx)[i] = double2{fxx[k], fxy[k]};
            reinterpret_cast<double2*>(il)[i] = double2{ilx[k], ily[k]};
        }
    }
#pragma unroll
    for (int k = 0; k < NG; ++k) {
        const int i = k * T + t;
        if (i < ND * np) {
            reinterpret_cast<double2*>(g)[i] = double2{gx[k], gy[k]};
            xl[i] = vxl[k];
        }
    }
    if constexpr (NJ > 0) {
#pragma unroll
        for (int k = 0; k < NJT; ++k) {
            const int e = k * T + t, c = e / NJ;
            if (e < kStageChains * NJ && chain0 + c < B) sj[e] = vj[k];
        }
    }
    if constexpr (NR > 0)
        if (t < kStageChains * NR) sr[t] = vr;
    __syncthreads();
    ev.node_fx = fx;
    ev.node_il = il;
    ev.g = g;
    ev.xL = xl;
}

// Chain of wavefront w in workgroup g.  LDS-table kernels: 8-chain workgroups, chain 8 g + w.
// Others: 4-chain workgroups taking half (g / 8) % 2 of the 8-chain block 8 (g / 16) + g % 8,
// which is on the XCD of workgroup g (workgroups are dispatched to the 8 XCDs in turn), as are
// the setup kernels' workgroups that wrote the block's records.  Grids of 16 (g / 16 + 1)
// workgroups cover the blocks of 8 (g / 16 + 1) groups.
template <bool LT>
__device__ inline int64_t chain_of(unsigned g, int w) {
    if constexpr (LT) return (int64_t)g * kStageChains + w;
    const int64_t blk = 8 * (int64_t)(g / 16) + g % 8;
    return blk * 8 + 4 * ((g / 8) % 2) + w;
}
// Workgroups of the 4-chain kernels for B chains (whole groups of 16).
inline unsigned grid4(int64_t B) { return (unsigned)(((B + 7) / 8 + 7) / 8 * 16); }

template <int ND, bool MIXED, int WF, bool LT = false>
__global__ __launch_bounds__(LT ? 64 * kStageChains : 256) void k_loglike_fwd(EventDev ev, const double* __restrict__ recs, int64_t B,
                                                     double* __restrict__ lnl) {
    __shared__ double2 tab[kPhasorN];
    if constexpr (LT && WF == kWfTaylorF2) {
        extern __shared__ double lds_tables[];
        stage_tf2_workgroup<ND, 0>(ev, tab, lds_tables, nullptr, 0, 0, nullptr);
    } else {
        load_phasor_table(ev, tab);
        if constexpr (LT) {
            extern __shared__ double lds_tables[];
            stage_edge_tables<ND>(ev, lds_tables);
        }
    }
    const int lane = threadIdx.x & 63;
    const int64_t chain = chain_of<LT>(blockIdx.x, wave_id());
    if (chain >= B) return;
    const double* rec = recs + chain * kRecStride;
    const double status = rec[kRecStatus];
    if (!(status == 1.0)) {
        if (lane == 0) lnl[chain] = (status == 0.0) ? -__builtin_inf() : __builtin_nan("");
        return;
    }
    ChainVals<ND> cv;
#pragma unroll
    for (int j = 0; j < kTf2Basis; ++j) cv.dc[j] = rec[kRecDc + j];
    const double g_re = rec[kRecG], g_im = rec[kRecG + 1];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const double pr = rec[kRecK + 2 * d], pi = rec[kRecK + 2 * d + 1];
        cv.kre[d] = pr * g_re - pi * g_im;  // K_d = P_d G
        cv.kim[d] = pr * g_im + pi * g_re;
        cv.dtau[d] = rec[kRecTau + d];
    }
    if (WF == kWfNrtv2) {
        double* dst = reinterpret_cast<double*>(&cv.np);
#pragma unroll
        for (int i = 0; i < kNrtParams; ++i) dst[i] = rec[kRecNrt + i];
    }
    double acc;
    if constexpr (WF == kWfNrtv2) {
        if (MIXED && use_mixed<ND>(ev, cv))
            acc = fwd_walk_natural<ND, float>(ev, cv, tab, lane);
        else
            acc = fwd_walk_natural<ND, double>(ev, cv, tab, lane);
    } else {
        if (MIXED && use_mixed<ND>(ev, cv))
            acc = fwd_walk<ND, float>(ev, cv, tab, lane);
        else
            acc = fwd_walk<ND, double>(ev, cv, tab, lane);
    }
    acc = wave_sum(acc);
    if constexpr (WF != kWfNrtv2) acc += tf2_quadratic<ND>(ev, cv);
    if (lane == 0) lnl[chain] = acc;
}

// ---------------------------------------------------------------------------
// Gradient.  d lnL = sum_j Re(conj(Gbar_j) dr_j) with
//   Gbar_j = gamma_j - mu_j r_j + c_j r_{j-1} + c_{j+1} r_{j+1},   z_j = conj(Gbar_j) r_j,
//   c_j = xL_j / 2,  d lnL / d phi_j = 2 pi Im z_j,  d lnL = Re(Z_d dK_d / K_d),  Z_d = sum_j z_dj.
// Each cross term is handled at its later edge: with w = c conj(r_{j-1}) r_j it adds
// w to z_j and conj(w) to z_{j-1} (2 Re w to Z_d, Im w to Im z_j, -Im w to Im z_{j-1}).
// Im z_j = Im(conj(gamma_j) r_j) + cross terms (the mu term is real), and
//   Re Z_d = sum_j [ Re(gamma r*) - mu |r|^2 + 2 (cross) ] = 2 lnL_d - sum_j Re(gamma r*),
// so lnL = (sum_d Re Z_d + sum_dj Re(gamma_dj r_dj*)) / 2 needs one accumulator more
// (IMRPhenomD_NRTidalv2; TaylorF2 accumulates the same sums with K_d factored out, see
// GradAccTf2, and adds the mu part -|K_d|^2 M_d after the walk).
// Per lane: Z_d, T_d = sum_j Im(z_dj) f_j and S_b = sum_j (sum_d Im z_dj) B_b(x_j);
// an edge's basis term is completed one step later, when the cross term to its right
// is known.  Each lane first evaluates the ratio at the edge before its first edge
// (owned by the previous lane), so nothing crosses lanes inside the walk.
// ---------------------------------------------------------------------------
template <int ND, int NA>
struct GradAcc {
    double acc;  // sum_dj Re(gamma_dj r_dj*)
    double zr[ND], zi[ND], ta[ND];
    double sa[NA];  // adjoints of the IMRPhenomD_NRTidalv2 node parameters
};

// TaylorF2 accumulators with K_d factored out, r_dj = K_d u_dj (per lane; reduced after the
// walk):  P_d = sum_j conj(gamma) u (complex),  X_d = sum_j xL Re(u_{j-1} u_j*),
// T_d = sum_j [ f_j Im(K_d conj(gamma_j) u_j) + |K_d|^2 xL Im(u_{j-1}* u_j) (f_j - f_{j-1}) / 2 ],
// S_b = sum_j q_j B_b(x_j) with q_j = sum_d Im z_dj.  Then
//   Z_d / K_d = P_d + conj(K_d) (X_d - M_d),
//   lnL = sum_d [ Re(K_d P_d) + |K_d|^2 (X_d - M_d) / 2 ],
//   d lnL / d tau_d = 2 pi T_d   (tau_d the delay in seconds),
// and K_d = 0 needs no special case.  (One T_d per detector rather than its two parts: fewer
// live registers, measured faster, most of all for the mixed form.)
template <int ND>
struct GradAccTf2 {
    double pr[ND], pi[ND], x[ND], t[ND];
    double sa[kTf2Basis];
};

// UNROLL2: two edges per loop iteration (the LDS-table kernel, which then keeps its loop
// state in registers without copies; measured faster there, not with global tables).
template <int ND, class R, bool UNROLL2 = false>
__device__ inline void grad_walk(const EventDev& ev, const ChainVals<ND>& cv, const double2* tab, int lane,
                                 GradAccTf2<ND>& G) {
    const EdgeTab<R> T = edge_tab(ev, R(0));
    const int npad = ev.n_nodes_pad;
    const int L = ev.L;
    R upr[ND], upi[ND];  // the previous edge's unit phasors
    R kre[ND], kim[ND];
    double k2[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        kre[d] = (R)cv.kre[d];
        kim[d] = (R)cv.kim[d];
        k2[d] = cv.kre[d] * cv.kre[d] + cv.kim[d] * cv.kim[d];
    }
    // halo edge: the last edge of lane - 1 (lane 0 has none; its first edge has xL = 0)
    const unsigned hpos = (unsigned)(lane > 0 ? (L - 1) * 64 + (lane - 1) : npad - 1);
    const Node hn = ld_node(ev, hpos);
    double fp = hn.f, xp = hn.x, ixp = hn.ix, lxp = hn.lx;
    {
        double bas[kTf2Basis];
        tf2_basis(xp, ixp, lxp, bas);
        double ph = -0.0;
#pragma unroll
        for (int b = 0; b < kTf2Basis; ++b) ph = fma(cv.dc[b], bas[b], ph);
#pragma unroll
        for (int d = 0; d < ND; ++d) unit_phasor(fma(fp, cv.dtau[d], ph), tab, upr[d], upi[d]);
    }
    double qprev = 0.0;  // q of the previous edge without its right cross term (halo: not ours)
    auto step = [&](int k) {
        const unsigned pos = (unsigned)(k * 64 + lane);
        const Node n = ld_node(ev, pos);
        const double f = n.f, x = n.x, ix = n.ix, lx = n.lx;
        double bas[kTf2Basis];
        tf2_basis(x, ix, lx, bas);
        double ph = -0.0;
#pragma unroll
        for (int b = 0; b < kTf2Basis; ++b) ph = fma(cv.dc[b], bas[b], ph);
        double qz = -0.0, p2 = -0.0;  // sum_d Im(conj(gamma) r), sum_d 2 Im w
        const double hdf = 0.5 * (f - fp);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            R ur, ui;
            unit_phasor(fma(f, cv.dtau[d], ph), tab, ur, ui);
            const unsigned o = (unsigned)(d * npad) + pos;
            const auto g = ld2(T.g, o);
            const R gre = g.x, gim = g.y, xl = ld(T.xl, o);
            const R pr = gre * ur + gim * ui, pi = gre * ui - gim * ur;  // conj(gamma) u
            G.pr[d] += (double)pr;
            G.pi[d] += (double)pi;
            const R imz = kre[d] * pi + kim[d] * pr;  // Im(conj(gamma) r)
            qz += (double)imz;
            acc_mul(G.x[d], upr[d] * ur + upi[d] * ui, (double)xl);
            const R t = xl * (upr[d] * ui - upi[d] * ur);
            const double kt = k2[d] * (double)t;  // |K_d|^2 xL Im(u_{j-1}* u_j)
            p2 += kt;
            G.t[d] = fma((double)imz, f, fma(kt, hdf, G.t[d]));
            upr[d] = ur;
            upi[d] = ui;
        }
        {   // the previous edge is now complete: it carries q_prev - p, p = p2 / 2
            double bp[kTf2Basis];
            tf2_basis(xp, ixp, lxp, bp);
            const double qp = fma(-0.5, p2, qprev);
#pragma unroll
            for (int b = 0; b < kTf2Basis; ++b) G.sa[b] = fma(qp, bp[b], G.sa[b]);
        }
        qprev = fma(0.5, p2, qz);
        fp = f; xp = x; ixp = ix; lxp = lx;
    };
    if constexpr (UNROLL2) {
#pragma unroll 2
        for (int k = 0; k < L; ++k) step(k);
    } else {
        for (int k = 0; k < L; ++k) step(k);
    }
    double bp[kTf2Basis];
    tf2_basis(xp, ixp, lxp, bp);
#pragma unroll
    for (int b = 0; b < kTf2Basis; ++b) G.sa[b] = fma(qprev, bp[b], G.sa[b]);
}

// IMRPhenomD_NRTidalv2: r_dj = K_d (a_j / a0_j) exp(-2 pi i (Phi_j - Phi0_j + f_j dtau_d)).
// With W_j = sum_d z_dj, the node parameters p receive
//   d lnL / dp = sum_j [ 2 pi Im(W_j) dPhi_j / dp + Re(W_j) / a_j  da_j / dp ],
// accumulated by nrt_node_adjoint.  Natural edge order (see fwd_walk_natural): the
// ratio of the next step is evaluated first, so that both neighbours of every edge of
// the current step are known (previous / next lane, or the carry from the previous
// step / lane 0 of the next step) and W_j is complete when its adjoint runs.  The right
// cross coefficient c_{j+1} = xR_j / 2 is read from the edge's own table.
template <int ND, class R>
__device__ inline void grad_walk_nrt(const EventDev& ev, const ChainVals<ND>& cv, const NrtParams<double>& np,
                                     const double2* tab, int lane, GradAcc<ND, kNrtAdj>& G) {
    const EdgeTab<R> T = edge_tab(ev, R(0));
    const R* xrt = xr_tab(ev, R(0));
    const int npad = ev.n_nodes_pad;
    const int L = ev.L;
    R kre[ND], kim[ND], rcr[ND], rci[ND], rnr[ND], rni[ND], rpr[ND], rpi[ND];
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        kre[d] = (R)cv.kre[d];
        kim[d] = (R)cv.kim[d];
        rpr[d] = rpi[d] = R(0);
    }
    double acur, anext = 0.0;
    NrtShared scur, snext{0.0, 0.0, 0.0};
    nrt_ratio<ND, R>(ev, cv, np, tab, lane, kre, kim, rcr, rci, acur, &scur);
    for (int k = 0; k < L; ++k) {
        if (k + 1 < L) {
            nrt_ratio<ND, R>(ev, cv, np, tab, (k + 1) * 64 + lane, kre, kim, rnr, rni, anext, &snext);
        } else {
#pragma unroll
            for (int d = 0; d < ND; ++d) rnr[d] = rni[d] = R(0);
        }
        const unsigned pos = (unsigned)(k * 64 + lane);
        const Node n = ld_node(ev, pos);
        const double f = n.f;
        double wre = 0.0, wim = 0.0;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const R rre = rcr[d], rim = rci[d];
            const R lre = left_neighbour(rre, rpr[d]), lim = left_neighbour(rim, rpi[d]);
            const R nre = right_neighbour(rre, rnr[d]), nim = right_neighbour(rim, rni[d]);
            const unsigned o = (unsigned)(d * npad) + pos;
            const auto g = ld2(T.g, o);
            const R gre = g.x, gim = g.y, mu = ld(T.mu, o);
            const R cl = R(0.5) * ld(T.xl, o), cr = R(0.5) * ld(xrt, o);
            G.acc += (double)(gre * rre + gim * rim);
            const R gbr = gre - mu * rre + cl * lre + cr * nre;
            const R gbi = gim - mu * rim + cl * lim + cr * nim;
            const double zr = (double)(gbr * rre + gbi * rim), zi = (double)(gbr * rim - gbi * rre);
            G.zr[d] += zr;
            G.zi[d] += zi;
            G.ta[d] = fma(zi, f, G.ta[d]);
            wre += zr;
            wim += zi;
        }
        nrt_node_adjoint(np, f, n.x, n.ix, n.lx, ld(ev.node_x578, pos), scur, (2.0 * kPi) * wim, acur != 0.0 ? wre / acur : 0.0, G.sa);
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            rpr[d] = rcr[d];
            rpi[d] = rci[d];
            rcr[d] = rnr[d];
            rci[d] = rni[d];
        }
        acur = anext;
        scur = snext;
    }
}

// The end of a fused MALA step for one chain (lanes 0..12 hold d lnL'/dtheta_i, all lanes
// active): with the chain's accept record (written by the proposal in the setup kernel),
//   log q(z|z') - log q(z'|z) = sum_i (rq_i - u_i^2),  u_i = dq_i - aq_i d lnL'/dtheta_i,
// the step is accepted when lnL(z) + log u < lnL' + sum_i (rq_i - u_i^2), and then (z, lnL, gz)
// <- (z', lnL', gz') with gz' = f d lnL'/dtheta (f = 1, or -1/sin iota and 1/cos dec).  The
// record is loaded before the walk (lanes 0..15, one row each), so the epilogue, which the
// wavefronts of a generation run at the same time, is two fmas, a 16-lane sum and the stores.
struct MalaState {
    double zp, dq, aq, rq;  // lanes 0..15: slot `lane` of each row
};

__device__ inline MalaState mala_load(const MalaEpi& me, int64_t chain, int lane) {
    MalaState m;
    if (lane < 16) {
        const double* r = me.rec + chain * kMalaRecStride + lane;
        m.zp = r[kMalaRecZp];
        m.dq = r[kMalaRecDq];
        m.aq = r[kMalaRecAq];
        m.rq = r[kMalaRecRq];
    }
    return m;
}

__device__ inline void mala_accept(const MalaEpi& me, const MalaState& m, int64_t chain, int lane, double lnl_new,
                                   double g) {
    const bool c = lane < 13;
    double term = 0.0;
    if (c) {
        const double u = fma(-m.aq, g, m.dq);
        term = fma(-u, u, m.rq);
    }
    term = row0_sum(term);
    const double thr = lane_read(m.rq, kMalaRecThr - kMalaRecRq);
    const double fi = lane_read(m.rq, kMalaRecFIota - kMalaRecRq), fd = lane_read(m.rq, kMalaRecFDec - kMalaRecRq);
    const bool accept = isfinite(lnl_new) && thr < lnl_new + term;
    if (accept && c) {
        const int64_t o = chain * 13 + lane;
        me.z[o] = m.zp;
        me.gz[o] = g * (lane == kMalaIota ? fi : (lane == kMalaDec ? fd : 1.0));
    }
    if (lane == 0) {
        if (accept) me.lnl[chain] = lnl_new;
        me.accepted[chain] = accept ? 1 : 0;
    }
}

// Occupancy target (waves per SIMD): 3 for the TaylorF2 LDS-table walk (unrolled by two, one
// 8-wave workgroup per CU; two workgroups at 128 registers measured slower) and the mixed
// walk (which spills at 4); 2 for the TaylorF2 FP64 global-table walk (170 registers: faster
// than 3 with spills or 4 with more) and for NRTidalv2, whose 26 adjoint accumulators and
// per-edge model would otherwise spill.
template <int ND, bool MIXED, int WF, bool LT = false, bool MALA = false>
__global__ __launch_bounds__(LT ? 64 * kStageChains : 256) __attribute__((amdgpu_waves_per_eu((WF == kWfNrtv2 || !(LT || MIXED)) ? 2 : 3))) void k_loglike_grad(
    EventDev ev, const double* __restrict__ recs, const double* __restrict__ jac, int64_t B,
    double* __restrict__ lnl, double* __restrict__ grad, MalaEpi me) {
    __shared__ double2 tab[kPhasorN];
    // TaylorF2 with LDS tables: the chains' Jacobian entries are staged too (sj), so that the
    // epilogue reads them from LDS rather than waiting a memory round trip after the walk.
    // and so are the chains' record entries [0, kRecDl] (sr), read back into scalar registers.
    constexpr bool JL = LT && WF == kWfTaylorF2;
    constexpr int NR = JL ? kRecDl + 1 : 1;
    double* sj = nullptr;
    double rv[NR];
    if constexpr (JL) {
        extern __shared__ double lds_tables[];
        sj = lds_tables + (size_t)ev.n_nodes_pad * (4 + 3 * ND);  // after the staged tables
        double* sr = sj + kStageChains * kJacTf2;
        stage_tf2_workgroup<ND, kJacTf2, NR>(ev, tab, lds_tables, jac, (int64_t)blockIdx.x * kStageChains, B, sj,
                                             recs, sr);
        double tmp[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) tmp[i] = sr[wave_id() * NR + i];
        __builtin_amdgcn_sched_barrier(0);  // all LDS reads in flight before the first use
#pragma unroll
        for (int i = 0; i < NR; ++i) rv[i] = uniform(tmp[i]);
    } else if constexpr (LT) {
        extern __shared__ double lds_tables[];
        if constexpr (WF == kWfNrtv2 && MIXED)
            stage_nrt_tables32<ND>(ev, tab, lds_tables);
        else
            stage_nrt_tables<ND>(ev, tab, lds_tables);
    } else {
        load_phasor_table(ev, tab);
    }
    const int lane = threadIdx.x & 63;
    const int64_t chain = chain_of<LT>(blockIdx.x, wave_id());
    if (chain >= B) return;
    MalaState ms;
    if constexpr (MALA) ms = mala_load(me, chain, lane);  // in flight during the walk
    const double* rec = recs + chain * kRecStride;
    auto rd = [&](int i) { return JL ? rv[i < NR ? i : 0] : rec[i]; };  // record entries up to kRecDl
    const double status = rd(kRecStatus);
    if (!(status == 1.0)) {
        if constexpr (MALA) {
            if (lane == 0) me.accepted[chain] = 0;  // a proposal outside the prior box, or not physical
        } else {
            if (lane == 0) lnl[chain] = (status == 0.0) ? -__builtin_inf() : __builtin_nan("");
            if (lane < 13) grad[chain * 13 + lane] = (status == 0.0) ? 0.0 : __builtin_nan("");
        }
        return;
    }
    // IMRPhenomD_NRTidalv2: the chain's 29 node parameters are read by the walk from LDS
    // (uniform-address loads) rather than held in scalar registers, which would overflow
    // into per-step spill reloads next to the table bases, K_d and the delays.
    __shared__ NrtParams<double> snp[LT ? kStageChains : 4];
    if constexpr (WF == kWfNrtv2) {
        if (lane < kNrtParams) reinterpret_cast<double*>(&snp[wave_id()])[lane] = rec[kRecNrt + lane];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    constexpr int NA = WF == kWfNrtv2 ? kNrtAdj : kTf2Basis;
    ChainVals<ND> cv;
#pragma unroll
    for (int j = 0; j < kTf2Basis; ++j) cv.dc[j] = rd(kRecDc + j);
    if (WF == kWfNrtv2) {
        double* dst = reinterpret_cast<double*>(&cv.np);
#pragma unroll
        for (int i = 0; i < kNrtParams; ++i) dst[i] = rec[kRecNrt + i];
    }
    const double g_re = rd(kRecG), g_im = rd(kRecG + 1);
    bool zero_k = false;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
        const double pr = rd(kRecK + 2 * d), pi = rd(kRecK + 2 * d + 1);
        cv.kre[d] = pr * g_re - pi * g_im;  // K_d = P_d G
        cv.kim[d] = pr * g_im + pi * g_re;
        cv.dtau[d] = rd(kRecTau + d);
        zero_k = zero_k || !(cv.kre[d] * cv.kre[d] + cv.kim[d] * cv.kim[d] > 1e-280);
    }
    // Z'_d = Z_d / K_d is the gradient with respect to K_d.
    double acc, A[NA], ZR[ND], ZI[ND], Tt[ND];
    if constexpr (WF == kWfNrtv2) {
        GradAcc<ND, NA> G;
        G.acc = 0.0;
#pragma unroll
        for (int d = 0; d < ND; ++d) G.zr[d] = G.zi[d] = G.ta[d] = 0.0;
#pragma unroll
        for (int b = 0; b < NA; ++b) G.sa[b] = 0.0;
        if (MIXED && use_mixed<ND>(ev, cv))
            grad_walk_nrt<ND, float>(ev, cv, snp[wave_id()], tab, lane, G);
        else
            grad_walk_nrt<ND, double>(ev, cv, snp[wave_id()], tab, lane, G);
        // Wave reductions of all accumulators at once.
        constexpr int NV = (1 + NA + 3 * ND + 3) / 4 * 4;
        double part[NV], tot[NV];
        part[0] = G.acc;
#pragma unroll
        for (int b = 0; b < NA; ++b) part[1 + b] = G.sa[b];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            part[1 + NA + d] = G.zr[d];
            part[1 + NA + ND + d] = G.zi[d];
            part[1 + NA + 2 * ND + d] = G.ta[d];
        }
#pragma unroll
        for (int i = 1 + NA + 3 * ND; i < NV; ++i) part[i] = 0.0;
        wave_sum_n<NV>(part, tot);
        acc = tot[0];
#pragma unroll
        for (int b = 0; b < NA; ++b) A[b] = tot[1 + b];  // the node adjoints include 2 pi
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const double k2 = cv.kre[d] * cv.kre[d] + cv.kim[d] * cv.kim[d];
            const double zre = tot[1 + NA + d], zim = tot[1 + NA + ND + d];
            acc += zre;
            const double ik2 = 1.0 / k2;
            ZR[d] = (zre * cv.kre[d] + zim * cv.kim[d]) * ik2;
            ZI[d] = (zim * cv.kre[d] - zre * cv.kim[d]) * ik2;
            Tt[d] = 2.0 * kPi * tot[1 + NA + 2 * ND + d];
        }
        acc *= 0.5;  // lnL = (sum_d Re Z_d + sum Re(gamma r*)) / 2
        if (zero_k) {
            // A detector with K_d = 0 has r = 0 everywhere: d lnL / dK_d = sum_j conj(gamma_j) u_j.
            const int npad = ev.n_nodes_pad;
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                if (cv.kre[d] * cv.kre[d] + cv.kim[d] * cv.kim[d] > 1e-280) continue;
                double sr = 0.0, si = 0.0;
                for (int k = 0; k < ev.L; ++k) {
                    const unsigned pos = (unsigned)(k * 64 + lane);
                    const Node n = ld_node(ev, pos);
                    double ph, ar;
                    edge_phase<ND, WF>(ev, cv, pos, n, ph, ar);
                    double ur, ui;
                    expm2pi_rev(fma(n.f, cv.dtau[d], ph) * (1.0 / kPhasorN), ur, ui);
                    ur *= ar;
                    ui *= ar;
                    const double2 g = ld2(ev.g, (unsigned)(d * npad) + pos);
                    sr += g.x * ur + g.y * ui;
                    si += g.x * ui - g.y * ur;
                }
                ZR[d] = wave_sum(sr);
                ZI[d] = wave_sum(si);
            }
        }
    } else {
        GradAccTf2<ND> G;
#pragma unroll
        for (int d = 0; d < ND; ++d) G.pr[d] = G.pi[d] = G.x[d] = G.t[d] = 0.0;
#pragma unroll
        for (int b = 0; b < kTf2Basis; ++b) G.sa[b] = 0.0;
        if (MIXED && use_mixed<ND>(ev, cv))
            grad_walk<ND, float>(ev, cv, tab, lane, G);
        else
            grad_walk<ND, double, LT>(ev, cv, tab, lane, G);
        constexpr int NV = (kTf2Basis + 4 * ND + 3) / 4 * 4;
        double part[NV], tot[NV];
#pragma unroll
        for (int b = 0; b < kTf2Basis; ++b) part[b] = G.sa[b];
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            part[kTf2Basis + d] = G.pr[d];
            part[kTf2Basis + ND + d] = G.pi[d];
            part[kTf2Basis + 2 * ND + d] = G.x[d];
            part[kTf2Basis + 3 * ND + d] = G.t[d];
        }
#pragma unroll
        for (int i = kTf2Basis + 4 * ND; i < NV; ++i) part[i] = 0.0;
        wave_sum_n<NV>(part, tot);
#pragma unroll
        for (int b = 0; b < NA; ++b) A[b] = (2.0 * kPi) * tot[b];
        acc = 0.0;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
            const double kr = cv.kre[d], ki = cv.kim[d], k2 = kr * kr + ki * ki;
            const double pr = tot[kTf2Basis + d], pi = tot[kTf2Basis + ND + d];
            const double xm = tot[kTf2Basis + 2 * ND + d] - ev.mu_sum[d];
            acc = fma(kr, pr, fma(-ki, pi, fma(0.5 * k2, xm, acc)));
            ZR[d] = fma(kr, xm, pr);
            ZI[d] = fma(-ki, xm, pi);
            Tt[d] = (2.0 * kPi) * tot[kTf2Basis + 3 * ND + d];
        }
    }
    // Chain rule through the setup: d lnL = sum_b A_b d dc_b + sum_d Re(Z'_d dK_d) + sum_d T_d d dtau_d,
    //   intrinsic i:  dK_d = K_d (d ln amp - 2 pi i d dc_const)
    //   dL: dK_d = -K_d / dL;  phic: dK_d = 2i K_d;  tc: d dtau_d = 1
    //   angles a:     dK_d = G dP_d,  d dtau_d = d dt_d
    double g = 0.0;
    if (lane < 13) {
        const double* J = jac + chain * kJacStride;
        const double* Jl = JL ? sj + wave_id() * kJacTf2 : nullptr;  // staged: [intrinsic | extrinsic]
        auto jint = [&](int i) { return JL ? Jl[i - kJacInt] : J[i]; };
        auto jext = [&](int i) { return JL ? Jl[kJacTf2Int + (i - kJacExt)] : J[i]; };
        if (lane < 6 && WF == kWfNrtv2) {
#pragma unroll
            for (int b = 0; b < NA; ++b) g = fma(A[b], J[kJacInt + b * 6 + lane], g);
            const double dre = J[kJacInt + kJacAmpNrt * 6 + lane];
#pragma unroll
            for (int d = 0; d < ND; ++d) g = fma(ZR[d] * cv.kre[d] - ZI[d] * cv.kim[d], dre, g);
        } else if (lane < 6) {
#pragma unroll
            for (int b = 0; b < NA; ++b) g = fma(A[b], jint(kJacInt + b * 6 + lane), g);
            const double dre = jint(kJacInt + kJacAmpTf2 * 6 + lane);
            const double dim = -2.0 * kPi * jint(kJacInt + 10 * 6 + lane);
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                const double wr = ZR[d] * cv.kre[d] - ZI[d] * cv.kim[d], wi = ZR[d] * cv.kim[d] + ZI[d] * cv.kre[d];
                g += wr * dre - wi * dim;
            }
        } else if (lane == 6 || lane == 8) {
            double sr = 0.0, si = 0.0;  // sum_d Z'_d K_d
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                sr += ZR[d] * cv.kre[d] - ZI[d] * cv.kim[d];
                si += ZR[d] * cv.kim[d] + ZI[d] * cv.kre[d];
            }
            g = (lane == 6) ? -sr / rd(kRecDl) : -2.0 * si;
        } else if (lane == 7) {
#pragma unroll
            for (int d = 0; d < ND; ++d) g += Tt[d];
        } else {
            const int a = lane - 9;
#pragma unroll
            for (int d = 0; d < ND; ++d) {
                const double pr = jext(kJacExt + (d * 3 + 0) * 4 + a), pi = jext(kJacExt + (d * 3 + 1) * 4 + a);
                const double kr = g_re * pr - g_im * pi, ki = g_re * pi + g_im * pr;  // dK_d
                g += ZR[d] * kr - ZI[d] * ki + Tt[d] * jext(kJacExt + (d * 3 + 2) * 4 + a);
            }
        }
    }
    if constexpr (MALA) {
        mala_accept(me, ms, chain, lane, acc, g);
    } else {
        if (lane == 0) lnl[chain] = acc;
        if (lane < 13) grad[chain * 13 + lane] = g;
    }
}

// ---------------------------------------------------------------------------
// Launch wrappers: 4 chains (wavefronts) per 256-thread workgroup.
// ---------------------------------------------------------------------------
template <int ND>
static void fwd_nd(const EventDev& ev, const double* rec, int64_t B, int mixed, double* lnl, hipStream_t s,
                   KTime kt) {
    const unsigned grid = grid4(B);
    if (ev.waveform == kWfNrtv2) {
        if (mixed)
            launch_k(k_loglike_fwd<ND, true, kWfNrtv2>, dim3(grid), dim3(256), s, kt, ev, rec, B, lnl);
        else
            launch_k(k_loglike_fwd<ND, false, kWfNrtv2>, dim3(grid), dim3(256), s, kt, ev, rec, B, lnl);
    } else {
        const size_t lb = staged_table_bytes(ND, ev.n_nodes_pad);
        if (mixed)
            launch_k(k_loglike_fwd<ND, true, kWfTaylorF2>, dim3(grid), dim3(256), s, kt, ev, rec, B, lnl);
        else if (lb <= kStageMaxBytes)
            launch_k_lds(k_loglike_fwd<ND, false, kWfTaylorF2, true>,
                         dim3((unsigned)((B + kStageChains - 1) / kStageChains)), dim3(64 * kStageChains), lb, s, kt,
                         ev, rec, B, lnl);
        else
            launch_k(k_loglike_fwd<ND, false, kWfTaylorF2>, dim3(grid), dim3(256), s, kt, ev, rec, B, lnl);
    }
}

hipError_t launch_loglike(const EventDev& ev, const double* rec, int64_t B, int mixed, double* lnl, hipStream_t s,
                          KTime kt) {
    switch (ev.n_det) {
        case 1: fwd_nd<1>(ev, rec, B, mixed, lnl, s, kt); break;
        case 2: fwd_nd<2>(ev, rec, B, mixed, lnl, s, kt); break;
        default: fwd_nd<3>(ev, rec, B, mixed, lnl, s, kt); break;
    }
    return hipGetLastError();
}

template <int ND, bool MALA>
static void grad_nd(const EventDev& ev, const double* rec, const double* jac, int64_t B, int mixed, double* lnl,
                    double* grad, hipStream_t s, KTime kt, const MalaEpi& me) {
    const unsigned grid = grid4(B);
    const unsigned grid_lt = (unsigned)((B + kStageChains - 1) / kStageChains);
    const dim3 blk(256), blk_lt(64 * kStageChains);
    if (ev.waveform == kWfNrtv2) {
        const size_t lb = staged_nrt_table_bytes(ND, ev.n_nodes_pad);
        const size_t lb32 = staged_nrt_table32_bytes(ND, ev.n_nodes_pad);
        if (mixed && lb32 <= kNrtStageMaxBytes)
            launch_k_lds(k_loglike_grad<ND, true, kWfNrtv2, true, MALA>, dim3(grid_lt), blk_lt, lb32, s, kt, ev, rec,
                         jac, B, lnl, grad, me);
        else if (mixed)
            launch_k(k_loglike_grad<ND, true, kWfNrtv2, false, MALA>, dim3(grid), blk, s, kt, ev, rec, jac, B, lnl,
                     grad, me);
        else if (lb <= kNrtStageMaxBytes)
            launch_k_lds(k_loglike_grad<ND, false, kWfNrtv2, true, MALA>, dim3(grid_lt), blk_lt, lb, s, kt, ev, rec,
                         jac, B, lnl, grad, me);
        else
            launch_k(k_loglike_grad<ND, false, kWfNrtv2, false, MALA>, dim3(grid), blk, s, kt, ev, rec, jac, B, lnl,
                     grad, me);
    } else {
        const size_t lb = staged_table_bytes(ND, ev.n_nodes_pad);
        if (mixed)
            launch_k(k_loglike_grad<ND, true, kWfTaylorF2, false, MALA>, dim3(grid), blk, s, kt, ev, rec, jac, B, lnl,
                     grad, me);
        else if (lb <= kStageMaxBytes)
            launch_k_lds(k_loglike_grad<ND, false, kWfTaylorF2, true, MALA>, dim3(grid_lt), blk_lt,
                         lb + sizeof(double) * kStageChains * (kJacTf2 + kRecDl + 1), s, kt, ev, rec, jac, B, lnl,
                         grad, me);
        else
            launch_k(k_loglike_grad<ND, false, kWfTaylorF2, false, MALA>, dim3(grid), blk, s, kt, ev, rec, jac, B,
                     lnl, grad, me);
    }
}

hipError_t launch_loglike_grad(const EventDev& ev, const double* rec, const double* jac, int64_t B, int mixed,
                               double* lnl, double* grad, hipStream_t s, KTime kt, const MalaEpi* mala) {
    const MalaEpi none{};
    if (mala) {
        switch (ev.n_det) {
            case 1: grad_nd<1, true>(ev, rec, jac, B, mixed, lnl, grad, s, kt, *mala); break;
            case 2: grad_nd<2, true>(ev, rec, jac, B, mixed, lnl, grad, s, kt, *mala); break;
            default: grad_nd<3, true>(ev, rec, jac, B, mixed, lnl, grad, s, kt, *mala); break;
        }
    } else {
        switch (ev.n_det) {
            case 1: grad_nd<1, false>(ev, rec, jac, B, mixed, lnl, grad, s, kt, none); break;
            case 2: grad_nd<2, false>(ev, rec, jac, B, mixed, lnl, grad, s, kt, none); break;
            default: grad_nd<3, false>(ev, rec, jac, B, mixed, lnl, grad, s, kt, none); break;
        }
    }
    return hipGetLastError();
}

}  // namespace rbl
