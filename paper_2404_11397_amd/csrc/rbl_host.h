// Host-side state shared by the C-ABI translation units (events, errors, helpers).
#pragma once
#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/rbl.h"
#include "rbl_launch.h"

namespace rbl {

// Thread-local error text for rbl_last_error; both return the code they are given
// (hip_fail: RBL_EDEVICE).
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

// Failure injection (rbl_debug_inject_fault): true when this allocation / launch must fail.
bool fault_take(int kind);

// Kernel timing of a call while rbl_profile_enable is on (every n-th call): runtime start/stop
// events around its setup and main kernels, collected by rbl_profile_read.
struct CallTimer {
    std::array<hipEvent_t, 4> ev{{nullptr, nullptr, nullptr, nullptr}};
    bool active = false;
    CallTimer();
    KTime setup() const { return active ? KTime{ev[0], ev[1]} : KTime{}; }
    KTime main() const { return active ? KTime{ev[2], ev[3]} : KTime{}; }
    void done();
};

constexpr int64_t kAlign = 256;
inline int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Device allocations of one owner, released together.
struct DevList {
    std::vector<void*> ptrs;
    hipError_t alloc(void** p, size_t bytes) {
        if (fault_take(RBL_FAULT_ALLOC)) return hipErrorOutOfMemory;
        hipError_t e = hipMalloc(p, bytes ? bytes : 1);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
    void release() {
        for (void* p : ptrs) (void)hipFree(p);
        ptrs.clear();
    }
};

// Workspace bytes of B chains (records, plus the Jacobians for the gradient).
inline int64_t workspace_bytes(int64_t B, bool with_grad) {
    int64_t bytes = align_up(B * kRecStride * (int64_t)sizeof(double));
    if (with_grad) bytes += align_up(B * kJacStride * (int64_t)sizeof(double));
    return bytes;
}
// Workspace bytes of the full-band likelihood: records, chain constants, tile partials.
inline int64_t full_workspace_bytes(int64_t n_freq, int64_t B, int32_t waveform) {
    const FullPlan p = full_plan(n_freq, B, waveform);
    return align_up(B * kRecStride * (int64_t)sizeof(double)) + align_up(B * kFullStride * (int64_t)sizeof(double)) +
           align_up(p.n_tiles * B * (int64_t)sizeof(double));
}

}  // namespace rbl

// A resident event: immutable after rbl_event_create.
struct rbl_event {
    int32_t n_det = 0, n_bins = 0, n_nodes = 0, n_nodes_pad = 0, waveform = 0;
    int32_t device = -1;  // the device current at rbl_event_create (holds the event's buffers)
    uint32_t flags = 0;
    int64_t n_freq = 0;
    double f_low = 0, delta_f = 0, gmst = 0;
    rbl::Network net{};
    rbl::RefConsts ref{};
    rbl::EventDev dev{};
    double* d_summary = nullptr;
    double* d_data = nullptr;  // only with RBL_KEEP_GRID
    double* d_psd = nullptr;
    int64_t footprint = 0;
    std::vector<int64_t> edges;  // the bin edges (grid indices), given or placed on the device
    rbl::DevList mem;
};
