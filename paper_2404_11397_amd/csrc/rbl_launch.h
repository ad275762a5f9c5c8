// Kernel argument blocks and launch wrappers (internal to the library).
#pragma once
#include <hip/hip_ext.h>
#include "rbl_internal.h"

namespace rbl {

struct Theta13 {
    double v[13];
};

// One work item of the summary pass: a run of grid points inside one bin, with the bin
// centre precomputed (one load gives a wavefront everything it needs before its data).
struct SumItem {
    int64_t start;
    int32_t count, bin;
    double fm;
};

struct SummaryArgs {
    int64_t n_items;
    const SumItem* items;
    double f_low, delta_f;
    int64_t n_freq;
    int32_t n_det, n_bins;
    const double* data;  // [n_det][n_freq][2]
    const double* psd;   // [n_det][n_freq]
    double* partials;    // [n_items][n_det][7]
    const double* phasor;  // [kPhasorN][2] unit-phasor table
    RefConsts ref;
    int32_t ref_taper;
};

struct NodeArgs {
    int32_t n_nodes, n_nodes_pad, L, n_det, keep_b2, ref_taper;
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
    double* lnl;
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

hipError_t launch_ref_setup(const double* theta_host, const Network& net, int32_t waveform, RefConsts* out_dev,
                            hipStream_t s);
hipError_t launch_chain_setup(const double* theta, int64_t B, const Network& net, const RefConsts& ref,
                              double* rec, double* jac, hipStream_t s, KTime kt = {});
// kt_items / kt_reduce: timing of the per-item kernel and of the reduction.
hipError_t launch_summary(const SummaryArgs& a, const int64_t* bin_first_item, double* summary, hipStream_t s,
                          KTime kt_items = {}, KTime kt_reduce = {});
hipError_t launch_node_tables(const NodeArgs& a, hipStream_t s);
hipError_t launch_loglike(const EventDev& ev, const double* rec, int64_t B, int mixed, double* lnl, hipStream_t s,
                          KTime kt = {});
hipError_t launch_loglike_grad(const EventDev& ev, const double* rec, const double* jac, int64_t B, int mixed,
                               double* lnl, double* grad, hipStream_t s, KTime kt = {});
hipError_t launch_loglike_full(const FullArgs& a, int64_t B, hipStream_t s, KTime kt = {});
hipError_t launch_strain(const RefConsts* cst_dev, int32_t waveform, int32_t taper, int32_t n_det, double f_low,
                         double delta_f, int64_t n_freq, double* out, hipStream_t s);

}  // namespace rbl
