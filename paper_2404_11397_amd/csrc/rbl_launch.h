// Kernel argument blocks and launch wrappers (internal to the library).
#pragma once
#include <hip/hip_ext.h>
#include "rbl_internal.h"

namespace rbl {

struct Theta13 {
    double v[13];
};

// The summary pass: one workgroup per bin of kSumThreads* threads, each taking kSumPpt* grid
// points per pass (TaylorF2 / IMRPhenomD_NRTidalv2).
constexpr int kSumThreadsTf2 = 256;
constexpr int kSumPptTf2 = 4;
constexpr int kSumThreadsNrt = 256;
constexpr int kSumPptNrt = 2;

struct SummaryArgs {
    const int64_t* edges;  // [n_bins + 1] grid indices of the bin edges
    const int32_t* order;  // [n_bins] bin of each workgroup
    double f_low, delta_f;
    int64_t n_freq;
    int32_t n_det, n_bins;
    const double* data;    // [n_det][n_freq][2]
    const double* psd;     // [n_det][n_freq]
    double* summary;       // [n_det][n_bins][7]
    const double* phasor;  // [kPhasorN][2] unit-phasor table
    RefConsts ref;
    int32_t ref_taper;
};

struct NodeArgs {
    int32_t n_nodes, n_nodes_pad, L, n_det, keep_b2, ref_taper;
    int32_t centre;  // nodes are the edges and the bin centres interleaved (RBL_CENTRE_NODES)
    RefConsts ref;
    double *phi0, *ia0;
    float* ia0_32;
    double* node_x578;
    int32_t* bad_ref;  // set to 1 if the reference amplitude is not positive and finite at an edge
    const int64_t* edges;
    double f_low, delta_f;
    const double* summary;  // [n_det][n_bins][7]
    double *node_fx, *node_il;  // [n_nodes_pad][2]
    double *g, *mu, *xL, *xR;  // g: [n_det][n_nodes_pad][2]
    float *g32, *mu32, *xL32, *xR32;
    double* scales;
    double* mu_sum;
};

struct FullArgs {
    const double* recs;
    RefConsts ref;
    int32_t n_det;
    int64_t n_freq;
    double f_low, delta_f;
    const double* data;
    const double* psd;
    const double* phasor;  // [kPhasorN][2] unit-phasor table
    double* lnl;
};

// Full-band likelihood: chains are taken in groups of kFullGroup* that share every grid
// point's loads and chain-independent waveform work; the grid is cut into tiles whose
// per-chain partial sums are added in tile order.
constexpr int kFullStride = 56;     // doubles of per-chain constants
constexpr int kFullGroupTf2 = 8;    // chains per group (TaylorF2)
constexpr int kFullGroupNrt = 4;    // chains per group (IMRPhenomD_NRTidalv2)
struct FullPlan {
    int64_t chains_per_group, n_groups, tile_points, n_tiles;
};
FullPlan full_plan(int64_t n_freq, int64_t B, int32_t waveform);
struct FullTileArgs {
    const double* consts;  // [B][kFullStride]
    double* partials;      // [B][n_tiles]
    const double* phasor;
    const double* data;    // [n_det][n_freq][2]
    const double* psd;     // [n_det][n_freq]
    int64_t B, n_freq;
    double f_low, delta_f;
    int64_t tile_points, n_tiles, n_groups;
};

// Optional start / stop events recorded by the runtime at the kernel's own start and end
// (benchmark timing); both null = a plain launch.
struct KTime {
    hipEvent_t start = nullptr, stop = nullptr;
};
template <typename F, typename... Args>
inline void launch_k(F kernel, dim3 grid, dim3 block, hipStream_t s, KTime kt, Args... args) {
    if (kt.start || kt.stop)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s, kt.start, kt.stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}
// The same with dynamic LDS bytes.
template <typename F, typename... Args>
inline void launch_k_lds(F kernel, dim3 grid, dim3 block, size_t lds_bytes, hipStream_t s, KTime kt, Args... args) {
    if (kt.start || kt.stop)
        hipExtLaunchKernelGGL(kernel, grid, block, lds_bytes, s, kt.start, kt.stop, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, lds_bytes, s, args...);
}

// MALA step fused into the gradient kernels (Sec. II D): the proposal
//   z' = z + (s/2) gz + sqrt(s) xi,  theta' = theta(z') (iota = arccos z_9, dec = arcsin z_12),
// a NaN row outside the prior box, made by the gradient setup kernel; the Metropolis
// decision on log u < lnL' - lnL + log q(z|z') - log q(z'|z) and the in-place update of
// (z, lnL, gz), made by the gradient kernel's epilogue.
// The per-chain accept record of a MALA step, written by the proposal (setup kernel) and read
// by the accept epilogue (gradient kernel): four rows of 16 doubles, z', dq, aq and rq of each
// of the 13 components (lane-contiguous for the epilogue's loads), with lnL(z) + log u and the
// factors from d lnL/dtheta to d lnL/dz of iota and dec in the spare slots of the rq row.
constexpr int kMalaIota = 9, kMalaDec = 12;
constexpr int kMalaRecZp = 0, kMalaRecDq = 16, kMalaRecAq = 32, kMalaRecRq = 48;
constexpr int kMalaRecThr = kMalaRecRq + 13, kMalaRecFIota = kMalaRecRq + 14, kMalaRecFDec = kMalaRecRq + 15;
constexpr int kMalaRecStride = 64;

struct MalaProp {
    const double *z, *gz, *xi;  // [B][13]
    const double *lnl, *logu;   // [B]
    double* rec;                // [B][kMalaRecStride] accept records
    double s[13], sq[13], lo[13], hi[13];
    double k[13], hk[13];       // 1/sqrt(2 s) and (s/2)/sqrt(2 s)
};
struct MalaEpi {
    const double* rec;     // [B][kMalaRecStride]
    double *z, *gz, *lnl;  // updated in place where accepted
    int32_t* accepted;
};

hipError_t launch_ref_setup(const double* theta_host, const Network& net, int32_t waveform, RefConsts* out_dev,
                            hipStream_t s);
// prop (gradient setup only): take theta from the MALA proposal instead of `theta`.
hipError_t launch_chain_setup(const double* theta, int64_t B, const Network& net, const RefConsts& ref,
                              double* rec, double* jac, hipStream_t s, KTime kt = {}, const MalaProp* prop = nullptr);
hipError_t launch_summary(const SummaryArgs& a, hipStream_t s, KTime kt = {});
hipError_t launch_node_tables(const NodeArgs& a, hipStream_t s);
hipError_t launch_loglike(const EventDev& ev, const double* rec, int64_t B, int mixed, double* lnl, hipStream_t s,
                          KTime kt = {});
// mala: finish a MALA step in the epilogue instead of writing lnl and grad.
hipError_t launch_loglike_grad(const EventDev& ev, const double* rec, const double* jac, int64_t B, int mixed,
                               double* lnl, double* grad, hipStream_t s, KTime kt = {}, const MalaEpi* mala = nullptr);
// consts: B * kFullStride doubles; partials: B * n_tiles doubles (full_plan).
hipError_t launch_loglike_full(const FullArgs& a, int64_t B, double* consts, double* partials, hipStream_t s,
                               KTime kt = {});
// Bin edges on the device by the post-Newtonian phase-bound ansatz; phi: n doubles of scratch.
hipError_t launch_bin_edges(double f_low, double delta_f, int64_t n, int32_t n_bins, double* phi, int64_t* edges,
                            hipStream_t s);
hipError_t launch_strain(const RefConsts* cst_dev, int32_t waveform, int32_t taper, int32_t n_det, double f_low,
                         double delta_f, int64_t n_freq, double* out, hipStream_t s);

}  // namespace rbl
