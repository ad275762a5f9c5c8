// Metropolis-adjusted Langevin (MALA) local step on the device (the gradient-based local
// sampler of Sec. II D), over Tab. II's uniform priors.
//
// A chain's state is z (13): (Mc, q, chi1, chi2, Lambda1, Lambda2, dL, tc, phic, cos iota,
// psi, ra, sin delta) -- the coordinates in which the priors are uniform -- with its lnL and
// g = d lnL / dz.  One step is two launches of the gradient path: the gradient setup kernel
// makes the proposal z' = z + (s/2) g + sqrt(s) xi and theta(z') (a NaN row outside the prior
// box, which the likelihood kernel then skips), and the gradient kernel's epilogue accepts
// when
//   log u < lnL' - lnL + log q(z | z') - log q(z' | z),
//   log q(b | a) = -sum_i (b_i - a_i - s_i g_i(a) / 2)^2 / (2 s_i),
// updating (z, lnL, g) in place.  xi and log u are inputs.
#include "rbl_host.h"

using namespace rbl;

namespace {

constexpr int kIota = 9, kDec = 12;

struct MalaArgs {
    double s[13], sq[13], lo[13], hi[13];  // step (variance), its square root, prior box
};

// theta(z): iota = arccos(cos iota), dec = arcsin(sin dec); the rest unchanged.
__device__ inline void z_to_theta(const double* z, double* th) {
#pragma unroll
    for (int i = 0; i < 13; ++i) th[i] = z[i];
    th[kIota] = acos(fmin(fmax(z[kIota], -1.0), 1.0));
    th[kDec] = asin(fmin(fmax(z[kDec], -1.0), 1.0));
}

// d lnL / dz from d lnL / dtheta: d/dcos(iota) = -(d/diota) / sin(iota), d/dsin(dec) = (d/ddec) / cos(dec).
__device__ inline void grad_to_z(const double* th, const double* g, double* gz) {
#pragma unroll
    for (int i = 0; i < 13; ++i) gz[i] = g[i];
    gz[kIota] = -g[kIota] / sin(th[kIota]);
    gz[kDec] = g[kDec] / cos(th[kDec]);
}

__global__ void k_mala_theta(const double* __restrict__ z, int64_t B, double* __restrict__ theta) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double zz[13], th[13];
    for (int i = 0; i < 13; ++i) zz[i] = z[b * 13 + i];
    z_to_theta(zz, th);
    for (int i = 0; i < 13; ++i) theta[b * 13 + i] = th[i];
}

__global__ void k_mala_gradz(const double* __restrict__ theta, const double* __restrict__ g, int64_t B,
                             double* __restrict__ gz) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double th[13], gg[13], out[13];
    for (int i = 0; i < 13; ++i) {
        th[i] = theta[b * 13 + i];
        gg[i] = g[b * 13 + i];
    }
    grad_to_z(th, gg, out);
    for (int i = 0; i < 13; ++i) gz[b * 13 + i] = out[i];
}

// Workspace: theta(z) and d lnL/dtheta (initialisation), the accept records (steps), then the
// likelihood workspace (records and Jacobians).
struct MalaWs {
    double *thp, *gthp;  // [B][13]
    double* mrec;        // [B][kMalaRecStride]
    void* lws;
};

MalaWs carve(void* ws, int64_t B) {
    char* p = (char*)ws;
    MalaWs w;
    const int64_t row = align_up(B * 13 * (int64_t)sizeof(double));
    w.thp = (double*)p;
    w.gthp = (double*)(p + row);
    w.mrec = (double*)(p + 2 * row);
    w.lws = p + 2 * row + align_up(B * kMalaRecStride * (int64_t)sizeof(double));
    return w;
}

int check_mala(const char* who, const rbl_event* ev, const void* z, int64_t B, int32_t precision, const void* lnl,
               const void* gz, const void* ws) {
    if (!ev || !z || !lnl || !gz || !ws) return fail(RBL_EINVAL, std::string(who) + ": null argument");
    if (B < 0 || B > ((int64_t)1 << 31)) return fail(RBL_EINVAL, std::string(who) + ": B out of range");
    if (precision != RBL_FP64 && precision != RBL_MIXED) return fail(RBL_EINVAL, std::string(who) + ": unknown precision");
    if (((uintptr_t)ws) % kAlign) return fail(RBL_EINVAL, std::string(who) + ": workspace not 256-byte aligned");
    return RBL_OK;
}

}  // namespace

extern "C" int64_t rbl_mala_workspace_bytes(const rbl_event* ev, int64_t B) {
    if (!ev || B < 0) return 0;
    return 2 * align_up(B * 13 * (int64_t)sizeof(double)) + align_up(B * kMalaRecStride * (int64_t)sizeof(double)) +
           workspace_bytes(B, true);
}

extern "C" int rbl_mala_init(const rbl_event* ev, const double* z_dev, int64_t B, int32_t precision, double* lnl_dev,
                             double* gz_dev, void* workspace, void* hip_stream) {
    int rc = check_mala("rbl_mala_init", ev, z_dev, B, precision, lnl_dev, gz_dev, workspace);
    if (rc || B == 0) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    MalaWs w = carve(workspace, B);
    const unsigned grid = (unsigned)((B + 63) / 64);
    hipLaunchKernelGGL(k_mala_theta, dim3(grid), dim3(64), 0, s, z_dev, B, w.thp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "rbl_mala_init: launch");
    rc = rbl_loglike_grad(ev, w.thp, B, precision, lnl_dev, w.gthp, w.lws, hip_stream);
    if (rc) return rc;
    hipLaunchKernelGGL(k_mala_gradz, dim3(grid), dim3(64), 0, s, w.thp, w.gthp, B, gz_dev);
    e = hipGetLastError();
    return e == hipSuccess ? RBL_OK : hip_fail(e, "rbl_mala_init: launch");
}

extern "C" int rbl_mala_step(const rbl_event* ev, double* z_dev, double* lnl_dev, double* gz_dev, int64_t B,
                             int32_t precision, const double* step, const double* lo, const double* hi,
                             const double* xi_dev, const double* logu_dev, int32_t* accepted_dev, void* workspace,
                             void* hip_stream) {
    int rc = check_mala("rbl_mala_step", ev, z_dev, B, precision, lnl_dev, gz_dev, workspace);
    if (rc) return rc;
    if (!step || !lo || !hi) return fail(RBL_EINVAL, "rbl_mala_step: null step or prior box");
    MalaArgs m{};
    for (int i = 0; i < 13; ++i) {
        if (!(step[i] > 0.0) || !std::isfinite(step[i])) return fail(RBL_EINVAL, "rbl_mala_step: step must be > 0");
        if (!(lo[i] < hi[i])) return fail(RBL_EINVAL, "rbl_mala_step: prior box needs lo < hi");
        m.s[i] = step[i];
        m.sq[i] = std::sqrt(step[i]);
        m.lo[i] = lo[i];
        m.hi[i] = hi[i];
    }
    if (B == 0) return RBL_OK;
    if (!xi_dev || !logu_dev || !accepted_dev) return fail(RBL_EINVAL, "rbl_mala_step: null random numbers or output");
    hipStream_t s = (hipStream_t)hip_stream;
    MalaWs w = carve(workspace, B);
    if (fault_take(RBL_FAULT_LAUNCH)) return hip_fail(hipErrorLaunchFailure, "rbl_mala_step: injected");
    // Two launches: the gradient setup kernel makes the proposal, the gradient kernel's
    // epilogue takes the Metropolis decision and updates (z, lnL, gz) in place.
    MalaProp mp{};
    mp.z = z_dev;
    mp.gz = gz_dev;
    mp.xi = xi_dev;
    mp.lnl = lnl_dev;
    mp.logu = logu_dev;
    mp.rec = w.mrec;
    MalaEpi me{};
    me.rec = w.mrec;
    me.z = z_dev;
    me.gz = gz_dev;
    me.lnl = lnl_dev;
    me.accepted = accepted_dev;
    for (int i = 0; i < 13; ++i) {
        mp.s[i] = m.s[i];
        mp.sq[i] = m.sq[i];
        mp.lo[i] = m.lo[i];
        mp.hi[i] = m.hi[i];
        mp.k[i] = 1.0 / std::sqrt(2.0 * m.s[i]);
        mp.hk[i] = 0.5 * m.s[i] * mp.k[i];
    }
    double* rec = (double*)w.lws;
    double* jac = (double*)((char*)w.lws + align_up(B * kRecStride * (int64_t)sizeof(double)));
    CallTimer tm;
    hipError_t e = launch_chain_setup(nullptr, B, ev->net, ev->ref, rec, jac, s, tm.setup(), &mp);
    if (e != hipSuccess) return hip_fail(e, "rbl_mala_step: setup launch");
    e = launch_loglike_grad(ev->dev, rec, jac, B, precision == RBL_MIXED, nullptr, nullptr, s, tm.main(), &me);
    tm.done();
    return e == hipSuccess ? RBL_OK : hip_fail(e, "rbl_mala_step: launch");
}
