// lnL and gradient without any allocation: rbl_loglike_grad_noalloc.
//
// The per-chain records and Jacobians that rbl_loglike_grad keeps in the caller's workspace
// live here in one file-scope device array, `scratch`, sized for kNoAllocMaxChains chains.
// Each GPU holds its own copy of the array (from module load until the process ends).  The
// host never passes the array's name to a kernel: on the first call on a device, with that
// device current, hipGetSymbolAddress gives the array's device address, which is kept per
// device and passed to the kernels in place of the workspace.  Nothing in the array needs to
// start at zero: the setup kernel writes every value the likelihood kernel reads.
#include <mutex>

#include "rbl_host.h"

using namespace rbl;

constexpr int64_t kNoAllocMaxChains = RBL_NOALLOC_MAX_CHAINS;
constexpr int64_t kScratchBytes = (kNoAllocMaxChains * kRecStride * 8 + kAlign - 1) / kAlign * kAlign +
                                  (kNoAllocMaxChains * kJacStride * 8 + kAlign - 1) / kAlign * kAlign;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// The device address of this device's copy of `scratch` (looked up once per device).
int scratch_address(int dev, void** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "rbl_loglike_grad_noalloc: hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p) % kAlign) return fail(RBL_EDEVICE, "rbl_loglike_grad_noalloc: scratch misaligned");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return RBL_OK;
}

}  // namespace

extern "C" int rbl_loglike_grad_noalloc(const rbl_event* ev, const double* theta_dev, int64_t B, int32_t precision,
                                        double* lnl_dev, double* grad_dev, void* hip_stream) {
    if (!ev) return fail(RBL_EINVAL, "rbl_loglike_grad_noalloc: null event");
    if (B < 0) return fail(RBL_EINVAL, "rbl_loglike_grad_noalloc: B < 0");
    if (B == 0) return RBL_OK;
    if (B > kNoAllocMaxChains)
        return fail(RBL_EINVAL, "rbl_loglike_grad_noalloc: B = " + std::to_string(B) + " exceeds the " +
                                    std::to_string(kNoAllocMaxChains) + " chains of the static scratch");
    if (!theta_dev || !lnl_dev || !grad_dev) return fail(RBL_EINVAL, "rbl_loglike_grad_noalloc: null theta or output");
    if (precision != RBL_FP64 && precision != RBL_MIXED)
        return fail(RBL_EINVAL, "rbl_loglike_grad_noalloc: unknown precision");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "rbl_loglike_grad_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(RBL_EDEVICE, "rbl_loglike_grad_noalloc: device index out of range");
    if (dev != ev->device)
        return fail(RBL_EINVAL, "rbl_loglike_grad_noalloc: the current device is not the event's device");
    void* base = nullptr;
    int rc = scratch_address(dev, &base);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    double* rec = (double*)base;
    double* jac = (double*)((char*)base + align_up(B * kRecStride * (int64_t)sizeof(double)));
    e = launch_chain_setup(theta_dev, B, ev->net, ev->ref, rec, jac, s);
    if (e != hipSuccess) return hip_fail(e, "rbl_loglike_grad_noalloc: setup launch");
    e = launch_loglike_grad(ev->dev, rec, jac, B, precision == RBL_MIXED, lnl_dev, grad_dev, s);
    if (e != hipSuccess) return hip_fail(e, "rbl_loglike_grad_noalloc: launch");
    return RBL_OK;
}
