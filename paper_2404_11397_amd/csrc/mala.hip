// Metropolis-adjusted Langevin (MALA) local step on the device (the gradient-based local
// sampler of Sec. II D), over Tab. II's uniform priors.
//
// A chain's state is z (13): (Mc, q, chi1, chi2, Lambda1, Lambda2, dL, tc, phic, cos iota,
// psi, ra, sin delta) -- the coordinates in which the priors are uniform -- with its lnL and
// g = d lnL / dz.  One step: propose z' = z + (s/2) g + sqrt(s) xi (k_mala_propose), evaluate
// lnL and its gradient at theta(z') with the likelihood kernels, then accept when
//   log u < lnL' - lnL + log q(z | z') - log q(z' | z),
//   log q(b | a) = -sum_i (b_i - a_i - s_i g_i(a) / 2)^2 / (2 s_i),
// and z' lies inside the prior box (k_mala_accept).  xi and log u are inputs.
#include "rbl_host.h"

using namespace rbl;

namespace {

constexpr int kIota = 9, kDec = 12;

struct MalaArgs {
    double s[13], sq[13], lo[13], hi[13];  // step (variance), its square root, prior box
};

__device__ inline bool inside_box(const double* z, const MalaArgs& m) {
    bool in = true;
#pragma unroll
    for (int i = 0; i < 13; ++i) in = in && (z[i] >= m.lo[i]) && (z[i] <= m.hi[i]);
    return in;
}

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

// z' = z + (s/2) g + sqrt(s) xi; theta(z'), or a NaN row when z' leaves the prior box
// (the likelihood kernels then skip the chain).
__global__ void k_mala_propose(const double* __restrict__ z, const double* __restrict__ gz,
                               const double* __restrict__ xi, int64_t B, MalaArgs m, double* __restrict__ zp,
                               double* __restrict__ thp) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double q[13], th[13];
    for (int i = 0; i < 13; ++i) q[i] = z[b * 13 + i] + 0.5 * m.s[i] * gz[b * 13 + i] + m.sq[i] * xi[b * 13 + i];
    for (int i = 0; i < 13; ++i) zp[b * 13 + i] = q[i];
    if (inside_box(q, m)) {
        z_to_theta(q, th);
    } else {
        for (int i = 0; i < 13; ++i) th[i] = __builtin_nan("");
    }
    for (int i = 0; i < 13; ++i) thp[b * 13 + i] = th[i];
}

__global__ void k_mala_accept(double* __restrict__ z, double* __restrict__ lnl, double* __restrict__ gz,
                              const double* __restrict__ zp, const double* __restrict__ thp,
                              const double* __restrict__ lnlp, const double* __restrict__ gthp,
                              const double* __restrict__ logu, int64_t B, MalaArgs m, int32_t* __restrict__ accepted) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double a[13], q[13], ga[13], gq[13], th[13], gt[13];
    for (int i = 0; i < 13; ++i) {
        a[i] = z[b * 13 + i];
        q[i] = zp[b * 13 + i];
        ga[i] = gz[b * 13 + i];
        th[i] = thp[b * 13 + i];
        gt[i] = gthp[b * 13 + i];
    }
    const double lp = lnlp[b];
    bool ok = inside_box(q, m) && isfinite(lp);
    int32_t acc = 0;
    if (ok) {
        grad_to_z(th, gt, gq);
        double lq_back = 0.0, lq_fwd = 0.0;  // log q(z | z'), log q(z' | z)
        for (int i = 0; i < 13; ++i) {
            const double rb = a[i] - q[i] - 0.5 * m.s[i] * gq[i];
            const double rf = q[i] - a[i] - 0.5 * m.s[i] * ga[i];
            lq_back -= rb * rb / (2.0 * m.s[i]);
            lq_fwd -= rf * rf / (2.0 * m.s[i]);
        }
        const double log_alpha = lp - lnl[b] + lq_back - lq_fwd;
        if (logu[b] < log_alpha) {
            acc = 1;
            for (int i = 0; i < 13; ++i) {
                z[b * 13 + i] = q[i];
                gz[b * 13 + i] = gq[i];
            }
            lnl[b] = lp;
        }
    }
    accepted[b] = acc;
}

struct MalaWs {
    double *thp, *zp, *lnlp, *gthp;
    void* lws;
};

MalaWs carve(void* ws, int64_t B) {
    char* p = (char*)ws;
    MalaWs w;
    const int64_t row = align_up(B * 13 * (int64_t)sizeof(double));
    w.thp = (double*)p;
    w.zp = (double*)(p + row);
    w.gthp = (double*)(p + 2 * row);
    w.lnlp = (double*)(p + 3 * row);
    w.lws = p + 3 * row + align_up(B * (int64_t)sizeof(double));
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
    return 3 * align_up(B * 13 * (int64_t)sizeof(double)) + align_up(B * (int64_t)sizeof(double)) +
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
    const unsigned grid = (unsigned)((B + 63) / 64);
    hipLaunchKernelGGL(k_mala_propose, dim3(grid), dim3(64), 0, s, z_dev, gz_dev, xi_dev, B, m, w.zp, w.thp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "rbl_mala_step: launch");
    rc = rbl_loglike_grad(ev, w.thp, B, precision, w.lnlp, w.gthp, w.lws, hip_stream);
    if (rc) return rc;
    hipLaunchKernelGGL(k_mala_accept, dim3(grid), dim3(64), 0, s, z_dev, lnl_dev, gz_dev, w.zp, w.thp, w.lnlp, w.gthp,
                       logu_dev, B, m, accepted_dev);
    e = hipGetLastError();
    return e == hipSuccess ? RBL_OK : hip_fail(e, "rbl_mala_step: launch");
}
