// Host side of the C-ABI: validation, resident event state, kernel launches.
#include <algorithm>
#include <numeric>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rbl_host.h"

using namespace rbl;

namespace rbl {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return RBL_EDEVICE;
}

std::atomic<int> g_fault[2];

bool fault_take(int kind) {
    int c = g_fault[kind].load();
    while (c > 1)
        if (g_fault[kind].compare_exchange_weak(c, c - 1)) return false;
    return c == 1;  // armed: fails until cleared
}

}  // namespace rbl

extern "C" int rbl_debug_inject_fault(int32_t kind, int32_t count) {
    if (kind != RBL_FAULT_ALLOC && kind != RBL_FAULT_LAUNCH) return fail(RBL_EINVAL, "rbl_debug_inject_fault: unknown kind");
    if (count < 0) return fail(RBL_EINVAL, "rbl_debug_inject_fault: count < 0");
    g_fault[kind].store(count);
    return RBL_OK;
}

namespace {


bool theta_in_domain(const double* t) {
    for (int i = 0; i < 13; ++i)
        if (!std::isfinite(t[i])) return false;
    return t[0] > 0.0 && t[1] > 0.0 && t[6] > 0.0 && std::fabs(t[2]) < 1.0 && std::fabs(t[3]) < 1.0 &&
           t[4] >= 0.0 && t[5] >= 0.0;
}

// Benchmark timing: the runtime records start / stop events at the setup kernel's and the
// main kernel's own start and end (hipExtLaunchKernel), so the times are kernel durations.
struct ProfState {
    int32_t every = 0;   // 0: off; n: time every n-th call
    int64_t calls = 0;   // calls seen while on
    bool on = false;
    std::vector<hipEvent_t> free_events;
    std::vector<std::array<hipEvent_t, 4>> pending;  // setup start, setup stop, main start, main stop
    double summary_ms = 0.0;                          // summary-pass kernels of rbl_event_create
    int64_t summary_n = 0;
    hipEvent_t get() {
        if (!free_events.empty()) {
            hipEvent_t e = free_events.back();
            free_events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};
ProfState g_prof;

}  // namespace

CallTimer::CallTimer() {
    if (!g_prof.on || (g_prof.calls++ % g_prof.every) != 0) return;
    for (auto& e : ev) e = g_prof.get();
    active = ev[0] && ev[1] && ev[2] && ev[3];
}

void CallTimer::done() {
    if (active) g_prof.pending.push_back(ev);
}

extern "C" int rbl_profile_enable(int32_t every) {
    if (every < 0) return fail(RBL_EINVAL, "rbl_profile_enable: every must be >= 0");
    g_prof.on = every != 0;
    g_prof.every = every;
    g_prof.calls = 0;
    return RBL_OK;
}

extern "C" int rbl_profile_read_summary(double* ms, int64_t* events) {
    if (ms) *ms = g_prof.summary_ms;
    if (events) *events = g_prof.summary_n;
    g_prof.summary_ms = 0.0;
    g_prof.summary_n = 0;
    return RBL_OK;
}

extern "C" int rbl_profile_read(double* main_ms, double* setup_ms, int64_t* calls) {
    double m = 0.0, st = 0.0;
    int64_t n = 0;
    for (auto& t : g_prof.pending) {
        hipError_t e = hipEventSynchronize(t[3]);
        if (e != hipSuccess) return hip_fail(e, "rbl_profile_read");
        float a = 0.f, b = 0.f;
        (void)hipEventElapsedTime(&a, t[0], t[1]);
        (void)hipEventElapsedTime(&b, t[2], t[3]);
        st += a;
        m += b;
        ++n;
        for (auto e2 : t) g_prof.free_events.push_back(e2);
    }
    g_prof.pending.clear();
    if (main_ms) *main_ms = m;
    if (setup_ms) *setup_ms = st;
    if (calls) *calls = n;
    return RBL_OK;
}

extern "C" const char* rbl_last_error(void) { return g_err.c_str(); }

extern "C" int rbl_bin_edges(double f_low, double delta_f, int64_t n_freq, int32_t n_bins, int64_t* edges_out) {
    if (!edges_out) return fail(RBL_EINVAL, "rbl_bin_edges: null output");
    if (!(f_low > 0.0) || !(delta_f > 0.0) || n_freq < 2) return fail(RBL_EINVAL, "rbl_bin_edges: bad grid");
    if (n_bins < 1 || n_bins > n_freq - 1) return fail(RBL_EINVAL, "rbl_bin_edges: need 1 <= n_bins <= n_freq-1");
    static const double g[5] = {-5.0 / 3.0, -2.0 / 3.0, 1.0, 5.0 / 3.0, 7.0 / 3.0};
    const double f_high = f_low + (double)(n_freq - 1) * delta_f;
    std::vector<double> phi((size_t)n_freq);
    for (int64_t k = 0; k < n_freq; ++k) {
        const double f = f_low + (double)k * delta_f;
        double s = 0.0;
        for (double gg : g) {
            const double fs = gg < 0.0 ? f_low : f_high;
            s += (gg < 0.0 ? -1.0 : 1.0) * std::pow(f / fs, gg);
        }
        phi[(size_t)k] = s;
    }
    const double p0 = phi.front(), p1 = phi.back();
    for (int32_t i = 0; i <= n_bins; ++i) {
        const double tgt = p0 + (p1 - p0) * (double)i / (double)n_bins;
        // first index with phi >= tgt, clipped to [1, n-1]; pick the nearer neighbour
        int64_t pos = std::lower_bound(phi.begin(), phi.end(), tgt) - phi.begin();
        pos = std::min<int64_t>(std::max<int64_t>(pos, 1), n_freq - 1);
        edges_out[i] = (tgt - phi[(size_t)pos - 1] <= phi[(size_t)pos] - tgt) ? pos - 1 : pos;
    }
    edges_out[0] = 0;
    edges_out[n_bins] = n_freq - 1;
    for (int32_t i = 1; i <= n_bins; ++i) edges_out[i] = std::max(edges_out[i], edges_out[i - 1] + 1);
    edges_out[n_bins] = n_freq - 1;
    for (int32_t i = n_bins - 1; i >= 0; --i) edges_out[i] = std::min(edges_out[i], edges_out[i + 1] - 1);
    return RBL_OK;
}

static int validate_desc(const rbl_event_desc* d) {
    if (!d) return fail(RBL_EINVAL, "rbl_event_create: null descriptor");
    if (d->n_det < 1 || d->n_det > kMaxDet) return fail(RBL_EINVAL, "rbl_event_create: n_det must be 1..3");
    if (d->waveform != RBL_TAYLORF2 && d->waveform != RBL_PHENOMD_NRTV2)
        return fail(RBL_EINVAL, "rbl_event_create: unknown waveform");
    if (d->n_freq < 2) return fail(RBL_EINVAL, "rbl_event_create: n_freq must be >= 2");
    if (!(d->f_low > 0.0) || !std::isfinite(d->f_low)) return fail(RBL_EINVAL, "rbl_event_create: f_low must be > 0");
    if (!(d->delta_f > 0.0) || !std::isfinite(d->delta_f)) return fail(RBL_EINVAL, "rbl_event_create: delta_f must be > 0");
    if (!std::isfinite(d->gmst)) return fail(RBL_EINVAL, "rbl_event_create: gmst not finite");
    if (!d->data || !d->psd || !d->det_tensor || !d->det_vertex || !d->theta_ref)
        return fail(RBL_EINVAL, "rbl_event_create: null pointer in descriptor");
    if (d->n_bins < 1 || (int64_t)d->n_bins > d->n_freq - 1)
        return fail(RBL_EEDGES, "rbl_event_create: need 1 <= n_bins <= n_freq - 1");
    if (d->edges) {  // NULL: placed on the device
        if (d->edges[0] != 0 || d->edges[d->n_bins] != d->n_freq - 1)
            return fail(RBL_EEDGES, "rbl_event_create: first edge must be 0 and last n_freq - 1");
        for (int32_t i = 0; i < d->n_bins; ++i)
            if (!(d->edges[i + 1] > d->edges[i]))
                return fail(RBL_EEDGES, "rbl_event_create: edges not strictly increasing");
    }
    for (int i = 0; i < 9 * d->n_det; ++i)
        if (!std::isfinite(d->det_tensor[i])) return fail(RBL_EINVAL, "rbl_event_create: detector tensor not finite");
    for (int i = 0; i < 3 * d->n_det; ++i)
        if (!std::isfinite(d->det_vertex[i])) return fail(RBL_EINVAL, "rbl_event_create: detector vertex not finite");
    if (!theta_in_domain(d->theta_ref)) return fail(RBL_EINVAL, "rbl_event_create: theta_ref outside the physical domain");
    if ((d->flags & RBL_CENTRE_NODES) && (d->flags & RBL_KEEP_B2))
        return fail(RBL_EUNSUPPORTED, "rbl_event_create: RBL_KEEP_B2 is not offered with RBL_CENTRE_NODES");
    return RBL_OK;
}

extern "C" int rbl_event_create(const rbl_event_desc* desc, void* hip_stream, rbl_event** out) {
    if (!out) return fail(RBL_EINVAL, "rbl_event_create: null output");
    *out = nullptr;
    int rc = validate_desc(desc);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    const int nd = desc->n_det;
    const int64_t n = desc->n_freq;
    const int nb = desc->n_bins;
    const bool on_dev = (desc->flags & RBL_INPUT_ON_DEVICE) != 0;

    // PSD check (host copy if the input is on the device).
    {
        std::vector<double> tmp;
        const double* psd = desc->psd;
        if (on_dev) {
            tmp.resize((size_t)(nd * n));
            hipError_t e = hipMemcpy(tmp.data(), desc->psd, sizeof(double) * nd * n, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "rbl_event_create: reading psd");
            psd = tmp.data();
        }
        for (int64_t i = 0; i < nd * n; ++i)
            if (!(psd[i] > 0.0) || !std::isfinite(psd[i])) return fail(RBL_EPSD, "rbl_event_create: psd must be > 0 and finite");
    }

    rbl_event* ev = new rbl_event();
    ev->n_det = nd;
    ev->n_bins = nb;
    const bool centre = (desc->flags & RBL_CENTRE_NODES) != 0;
    ev->n_nodes = centre ? 2 * nb + 1 : nb + 1;  // bin edges, or edges and bin centres interleaved
    ev->n_nodes_pad = (int32_t)((ev->n_nodes + kNodeTile - 1) / kNodeTile * kNodeTile);  // 64 L
    ev->waveform = desc->waveform;
    ev->flags = desc->flags;
    ev->n_freq = n;
    ev->f_low = desc->f_low;
    ev->delta_f = desc->delta_f;
    ev->gmst = desc->gmst;
    ev->net.n_det = nd;
    ev->net.gmst = desc->gmst;
    for (int d = 0; d < nd; ++d) {
        for (int i = 0; i < 9; ++i) ev->net.D[d][i] = desc->det_tensor[9 * d + i];
        for (int i = 0; i < 3; ++i) ev->net.r[d][i] = desc->det_vertex[3 * d + i];
    }
    DevList tmp;  // temporaries of the build
    auto cleanup = [&](int code) {
        tmp.release();
        ev->mem.release();
        delete ev;
        return code;
    };
    hipError_t e;
    // Inputs on the device.
    double *d_data = nullptr, *d_psd = nullptr;
    DevList& grid_owner = (desc->flags & RBL_KEEP_GRID) ? ev->mem : tmp;
    if ((e = grid_owner.alloc((void**)&d_data, sizeof(double) * 2 * nd * n)) != hipSuccess)
        return cleanup(fail(RBL_ENOMEM, "rbl_event_create: device allocation (data)"));
    if ((e = grid_owner.alloc((void**)&d_psd, sizeof(double) * nd * n)) != hipSuccess)
        return cleanup(fail(RBL_ENOMEM, "rbl_event_create: device allocation (psd)"));
    const hipMemcpyKind kind = on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if ((e = hipMemcpyAsync(d_data, desc->data, sizeof(double) * 2 * nd * n, kind, s)) != hipSuccess)
        return cleanup(hip_fail(e, "rbl_event_create: copy data"));
    if ((e = hipMemcpyAsync(d_psd, desc->psd, sizeof(double) * nd * n, kind, s)) != hipSuccess)
        return cleanup(hip_fail(e, "rbl_event_create: copy psd"));
    if (desc->flags & RBL_KEEP_GRID) {
        ev->d_data = d_data;
        ev->d_psd = d_psd;
    }

    // Reference constants.
    RefConsts* d_ref = nullptr;
    if ((e = tmp.alloc((void**)&d_ref, sizeof(RefConsts))) != hipSuccess)
        return cleanup(fail(RBL_ENOMEM, "rbl_event_create: device allocation (ref)"));
    if ((e = launch_ref_setup(desc->theta_ref, ev->net, desc->waveform, d_ref, s)) != hipSuccess)
        return cleanup(hip_fail(e, "rbl_event_create: reference setup"));
    if ((e = hipMemcpyAsync(&ev->ref, d_ref, sizeof(RefConsts), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return cleanup(hip_fail(e, "rbl_event_create: copy reference"));
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return cleanup(hip_fail(e, "rbl_event_create: reference setup"));
    if (ev->ref.status != 1) return cleanup(fail(RBL_EINVAL, "rbl_event_create: theta_ref outside the physical domain"));
    for (int d = 0; d < nd; ++d) {
        const double a = ev->ref.invC0_re[d], b = ev->ref.invC0_im[d];
        if (!std::isfinite(a) || !std::isfinite(b) || !std::isfinite(ev->ref.h0fac_re[d]) || !std::isfinite(ev->ref.h0fac_im[d]) ||
            (ev->ref.h0fac_re[d] == 0.0 && ev->ref.h0fac_im[d] == 0.0))
            return cleanup(fail(RBL_EREF, "rbl_event_create: reference strain vanishes in detector " + std::to_string(d)));
    }

    // Bin edges: given, or placed on the device by the post-Newtonian phase-bound ansatz.
    if (desc->edges) {
        ev->edges.assign(desc->edges, desc->edges + nb + 1);
    } else {
        double* d_phi = nullptr;
        int64_t* d_pe = nullptr;
        if (tmp.alloc((void**)&d_phi, sizeof(double) * n) != hipSuccess ||
            tmp.alloc((void**)&d_pe, sizeof(int64_t) * (nb + 1)) != hipSuccess)
            return cleanup(fail(RBL_ENOMEM, "rbl_event_create: device allocation (bin placement)"));
        ev->edges.resize((size_t)nb + 1);
        if ((e = launch_bin_edges(ev->f_low, ev->delta_f, n, nb, d_phi, d_pe, s)) != hipSuccess ||
            (e = hipMemcpyAsync(ev->edges.data(), d_pe, sizeof(int64_t) * (nb + 1), hipMemcpyDeviceToHost, s)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return cleanup(hip_fail(e, "rbl_event_create: bin placement"));
    }
    const int64_t* edges = ev->edges.data();

    int64_t* d_edges = nullptr;
    if (tmp.alloc((void**)&d_edges, sizeof(int64_t) * (nb + 1)) != hipSuccess)
        return cleanup(fail(RBL_ENOMEM, "rbl_event_create: device allocation (edges)"));
    if ((e = hipMemcpyAsync(d_edges, edges, sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice, s)) != hipSuccess)
        return cleanup(hip_fail(e, "rbl_event_create: copy edges"));

    // Resident tables.
    const int64_t np = ev->n_nodes_pad;
    if (ev->mem.alloc((void**)&ev->d_summary, sizeof(double) * nd * nb * 7) != hipSuccess)
        return cleanup(fail(RBL_ENOMEM, "rbl_event_create: device allocation (summary)"));
    double* node_block = nullptr;
    // FP64 tables, scales, FP32 tables (2 nd np floats), reference phase / amplitude (2 np), FP32 amplitude
    // tables: 4 edge columns and 5 per-detector columns (FP64), the scales, 5 per-detector
    // FP32 columns, phi0 and 1/a0 (FP64), 1/a0 (FP32), x^5.78 (FP64), the phasor table, the
    // per-detector sums of mu; np is a multiple of 64
    const int64_t node_doubles =
        np * (4 + 5 * nd) + 2 * kMaxDet + np * 5 * nd / 2 + 2 * np + np / 2 + np + 2 * kPhasorN + kMaxDet;
    if (ev->mem.alloc((void**)&node_block, sizeof(double) * node_doubles) != hipSuccess)
        return cleanup(fail(RBL_ENOMEM, "rbl_event_create: device allocation (node tables)"));
    // the phasor table (used by the summary pass and the likelihood kernels) sits after the
    // other node-block tables: cos and sin of 2 pi k / kPhasorN, evaluated in extended
    // precision and rounded once
    double* d_phasor = node_block + node_doubles - 2 * kPhasorN - kMaxDet;
    std::vector<double> phasor(2 * kPhasorN);
    for (int k = 0; k < kPhasorN; ++k) {
        const long double a = 2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)kPhasorN;
        phasor[2 * k] = (double)std::cos(a);
        phasor[2 * k + 1] = (double)std::sin(a);
    }
    if ((e = hipMemcpyAsync(d_phasor, phasor.data(), sizeof(double) * 2 * kPhasorN, hipMemcpyHostToDevice, s)) !=
        hipSuccess)
        return cleanup(hip_fail(e, "rbl_event_create: copy phasor table"));

    // Workgroup order of the summary pass: bins by decreasing size, every other group of
    // n_cu workgroups reversed (breadth-first dispatch puts workgroups w and w + n_cu on one
    // CU, so a large bin shares its CU with a small one).
    int n_cu = 256;
    {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            n_cu = v;
    }
    std::vector<int32_t> order((size_t)nb);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return edges[x + 1] - edges[x] > edges[y + 1] - edges[y];
    });
    for (int64_t g0 = n_cu; g0 < nb; g0 += 2 * (int64_t)n_cu)
        std::reverse(order.begin() + g0, order.begin() + std::min<int64_t>(g0 + n_cu, nb));
    int32_t* d_order = nullptr;
    if (tmp.alloc((void**)&d_order, sizeof(int32_t) * nb) != hipSuccess)
        return cleanup(fail(RBL_ENOMEM, "rbl_event_create: device allocation (bin order)"));
    if ((e = hipMemcpyAsync(d_order, order.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, s)) != hipSuccess)
        return cleanup(hip_fail(e, "rbl_event_create: copy bin order"));

    SummaryArgs sa{};
    sa.edges = d_edges;
    sa.order = d_order;
    sa.f_low = ev->f_low;
    sa.delta_f = ev->delta_f;
    sa.n_freq = n;
    sa.n_det = nd;
    sa.n_bins = nb;
    sa.data = d_data;
    sa.psd = d_psd;
    sa.summary = ev->d_summary;
    sa.phasor = d_phasor;
    sa.ref = ev->ref;
    sa.ref_taper = (desc->flags & RBL_REF_TAPER) ? 1 : 0;
    // benchmark timing: the summary kernel's own duration
    std::array<hipEvent_t, 2> te{{nullptr, nullptr}};
    if (g_prof.on)
        for (auto& t : te) t = g_prof.get();
    const bool timed = te[0] && te[1];
    if ((e = launch_summary(sa, s, timed ? KTime{te[0], te[1]} : KTime{})) != hipSuccess)
        return cleanup(hip_fail(e, "rbl_event_create: summary pass"));
    if (timed && hipEventSynchronize(te[1]) == hipSuccess) {
        float m1 = 0.f;
        if (hipEventElapsedTime(&m1, te[0], te[1]) == hipSuccess) {
            g_prof.summary_ms += m1;
            g_prof.summary_n += 1;
        }
    }
    for (auto t : te)
        if (t) g_prof.free_events.push_back(t);

    NodeArgs na{};
    na.n_nodes = ev->n_nodes;
    na.n_nodes_pad = (int32_t)np;
    na.L = (int32_t)(np / kNodeTile);
    na.n_det = nd;
    na.keep_b2 = (desc->flags & RBL_KEEP_B2) ? 1 : 0;
    na.centre = centre ? 1 : 0;
    na.edges = d_edges;
    na.f_low = ev->f_low;
    na.delta_f = ev->delta_f;
    na.summary = ev->d_summary;
    na.node_fx = node_block;
    na.node_il = node_block + 2 * np;
    na.g = node_block + 4 * np;
    na.mu = na.g + 2 * nd * np;
    na.xL = na.mu + nd * np;
    na.xR = na.xL + nd * np;
    na.scales = na.xR + nd * np;
    na.g32 = (float*)(na.scales + 2 * kMaxDet);
    na.mu32 = na.g32 + 2 * nd * np;
    na.xL32 = na.mu32 + nd * np;
    na.xR32 = na.xL32 + nd * np;
    na.phi0 = na.scales + 2 * kMaxDet + np * 5 * nd / 2;  // after the FP32 tables (5 nd np floats)
    na.ia0 = na.phi0 + np;
    na.ia0_32 = (float*)(na.ia0 + np);
    na.node_x578 = na.ia0 + np + np / 2;
    na.mu_sum = d_phasor + 2 * kPhasorN;
    na.ref = ev->ref;
    na.ref_taper = (desc->flags & RBL_REF_TAPER) ? 1 : 0;
    int32_t* d_bad = nullptr;
    if (tmp.alloc((void**)&d_bad, sizeof(int32_t)) != hipSuccess)
        return cleanup(fail(RBL_ENOMEM, "rbl_event_create: device allocation (flag)"));
    if ((e = hipMemsetAsync(d_bad, 0, sizeof(int32_t), s)) != hipSuccess)
        return cleanup(hip_fail(e, "rbl_event_create: clear flag"));
    na.bad_ref = d_bad;
    if ((e = launch_node_tables(na, s)) != hipSuccess) return cleanup(hip_fail(e, "rbl_event_create: node tables"));
    int32_t bad = 0;
    if ((e = hipMemcpyAsync(&bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return cleanup(hip_fail(e, "rbl_event_create: read flag"));
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return cleanup(hip_fail(e, "rbl_event_create: build"));
    if (bad) return cleanup(fail(RBL_EREF, "rbl_event_create: reference amplitude not positive at a bin edge"));
    tmp.release();

    EventDev& dv = ev->dev;
    dv.n_det = nd;
    dv.n_bins = nb;
    dv.n_nodes = ev->n_nodes;
    dv.n_nodes_pad = (int32_t)np;
    dv.L = (int32_t)(np / kNodeTile);
    dv.n_freq = n;
    dv.f_low = ev->f_low;
    dv.delta_f = ev->delta_f;
    dv.node_fx = na.node_fx;
    dv.node_il = na.node_il;
    dv.g = na.g;
    dv.mu = na.mu;
    dv.xL = na.xL;
    dv.xR = na.xR;
    dv.g32 = na.g32;
    dv.mu32 = na.mu32;
    dv.xL32 = na.xL32;
    dv.xR32 = na.xR32;
    dv.scales = na.scales;
    dv.waveform = desc->waveform;
    dv.phi0 = na.phi0;
    dv.ia0 = na.ia0;
    dv.ia0_32 = na.ia0_32;
    dv.node_x578 = na.node_x578;
    dv.phasor = d_phasor;
    dv.mu_sum = na.mu_sum;
    ev->footprint = (int64_t)sizeof(double) * (nd * nb * 7 + node_doubles) +
                    ((desc->flags & RBL_KEEP_GRID) ? (int64_t)sizeof(double) * 3 * nd * n : 0);
    if (hipGetDevice(&ev->device) != hipSuccess) ev->device = -1;
    *out = ev;
    return RBL_OK;
}

extern "C" void rbl_event_free(rbl_event* ev) {
    if (!ev) return;
    ev->mem.release();
    delete ev;
}

extern "C" int64_t rbl_workspace_bytes(const rbl_event* ev, int64_t B, int32_t with_grad) {
    if (!ev || B < 0) return 0;
    const int64_t w = workspace_bytes(B, with_grad != 0);
    if (!(ev->flags & RBL_KEEP_GRID)) return w;
    const int64_t wf = full_workspace_bytes(ev->n_freq, B, ev->waveform);
    return wf > w ? wf : w;
}

extern "C" int64_t rbl_event_footprint_bytes(const rbl_event* ev) { return ev ? ev->footprint : 0; }

static int check_call(const char* who, const rbl_event* ev, const double* theta, int64_t B, int32_t precision,
                      const void* lnl, const void* ws) {
    if (!ev) return fail(RBL_EINVAL, std::string(who) + ": null event");
    if (B < 0) return fail(RBL_EINVAL, std::string(who) + ": B < 0");
    if (B == 0) return RBL_OK;
    if (!theta || !lnl) return fail(RBL_EINVAL, std::string(who) + ": null theta or output");
    if (!ws) return fail(RBL_EINVAL, std::string(who) + ": null workspace");
    if (((uintptr_t)ws) % kAlign) return fail(RBL_EINVAL, std::string(who) + ": workspace not 256-byte aligned");
    if (precision != RBL_FP64 && precision != RBL_MIXED) return fail(RBL_EINVAL, std::string(who) + ": unknown precision");
    if (B > (int64_t)1 << 31) return fail(RBL_EINVAL, std::string(who) + ": B too large");
    if (fault_take(RBL_FAULT_LAUNCH)) return hip_fail(hipErrorLaunchFailure, (std::string(who) + ": injected").c_str());
    return RBL_OK;
}

extern "C" int rbl_loglike(const rbl_event* ev, const double* theta_dev, int64_t B, int32_t precision,
                           double* lnl_dev, void* workspace, void* hip_stream) {
    int rc = check_call("rbl_loglike", ev, theta_dev, B, precision, lnl_dev, workspace);
    if (rc || B == 0) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    double* rec = (double*)workspace;
    CallTimer tm;
    hipError_t e = launch_chain_setup(theta_dev, B, ev->net, ev->ref, rec, nullptr, s, tm.setup());
    if (e != hipSuccess) return hip_fail(e, "rbl_loglike: setup launch");
    e = launch_loglike(ev->dev, rec, B, precision == RBL_MIXED, lnl_dev, s, tm.main());
    if (e != hipSuccess) return hip_fail(e, "rbl_loglike: launch");
    tm.done();
    return RBL_OK;
}

extern "C" int rbl_loglike_grad(const rbl_event* ev, const double* theta_dev, int64_t B, int32_t precision,
                                double* lnl_dev, double* grad_dev, void* workspace, void* hip_stream) {
    int rc = check_call("rbl_loglike_grad", ev, theta_dev, B, precision, lnl_dev, workspace);
    if (rc || B == 0) return rc;
    if (!grad_dev) return fail(RBL_EINVAL, "rbl_loglike_grad: null grad");
    hipStream_t s = (hipStream_t)hip_stream;
    double* rec = (double*)workspace;
    double* jac = (double*)((char*)workspace + align_up(B * kRecStride * (int64_t)sizeof(double)));
    CallTimer tm;
    hipError_t e = launch_chain_setup(theta_dev, B, ev->net, ev->ref, rec, jac, s, tm.setup());
    if (e != hipSuccess) return hip_fail(e, "rbl_loglike_grad: setup launch");
    e = launch_loglike_grad(ev->dev, rec, jac, B, precision == RBL_MIXED, lnl_dev, grad_dev, s, tm.main());
    if (e != hipSuccess) return hip_fail(e, "rbl_loglike_grad: launch");
    tm.done();
    return RBL_OK;
}

extern "C" int rbl_loglike_full(const rbl_event* ev, const double* theta_dev, int64_t B, double* lnl_dev,
                                void* workspace, void* hip_stream) {
    int rc = check_call("rbl_loglike_full", ev, theta_dev, B, RBL_FP64, lnl_dev, workspace);
    if (rc || B == 0) return rc;
    if (!(ev->flags & RBL_KEEP_GRID) || !ev->d_data)
        return fail(RBL_EUNSUPPORTED, "rbl_loglike_full: event built without RBL_KEEP_GRID");
    hipStream_t s = (hipStream_t)hip_stream;
    double* rec = (double*)workspace;
    CallTimer tm;
    hipError_t e = launch_chain_setup(theta_dev, B, ev->net, ev->ref, rec, nullptr, s, tm.setup());
    if (e != hipSuccess) return hip_fail(e, "rbl_loglike_full: setup launch");
    FullArgs a{};
    a.recs = rec;
    a.ref = ev->ref;
    a.n_det = ev->n_det;
    a.n_freq = ev->n_freq;
    a.f_low = ev->f_low;
    a.delta_f = ev->delta_f;
    a.data = ev->d_data;
    a.psd = ev->d_psd;
    a.phasor = ev->dev.phasor;
    a.lnl = lnl_dev;
    double* consts = (double*)((char*)workspace + align_up(B * kRecStride * (int64_t)sizeof(double)));
    double* partials = (double*)((char*)consts + align_up(B * kFullStride * (int64_t)sizeof(double)));
    e = launch_loglike_full(a, B, consts, partials, s, tm.main());
    if (e != hipSuccess) return hip_fail(e, "rbl_loglike_full: launch");
    tm.done();
    return RBL_OK;
}

extern "C" int rbl_strain(int32_t waveform, int32_t n_det, const double* det_tensor, const double* det_vertex,
                          double gmst, double f_low, double delta_f, int64_t n_freq, const double* theta,
                          int32_t taper, double* out_dev, void* hip_stream) {
    if (waveform != RBL_TAYLORF2 && waveform != RBL_PHENOMD_NRTV2) return fail(RBL_EINVAL, "rbl_strain: unknown waveform");
    if (n_det < 1 || n_det > kMaxDet) return fail(RBL_EINVAL, "rbl_strain: n_det must be 1..3");
    if (!det_tensor || !det_vertex || !theta || !out_dev) return fail(RBL_EINVAL, "rbl_strain: null pointer");
    if (!(f_low > 0.0) || !(delta_f > 0.0) || n_freq < 1) return fail(RBL_EINVAL, "rbl_strain: bad grid");
    if (!theta_in_domain(theta)) return fail(RBL_EINVAL, "rbl_strain: theta outside the physical domain");
    Network net{};
    net.n_det = n_det;
    net.gmst = gmst;
    for (int d = 0; d < n_det; ++d) {
        for (int i = 0; i < 9; ++i) net.D[d][i] = det_tensor[9 * d + i];
        for (int i = 0; i < 3; ++i) net.r[d][i] = det_vertex[3 * d + i];
    }
    hipStream_t s = (hipStream_t)hip_stream;
    RefConsts* d_cst = nullptr;
    hipError_t e = hipMalloc((void**)&d_cst, sizeof(RefConsts));
    if (e != hipSuccess) return fail(RBL_ENOMEM, "rbl_strain: device allocation");
    e = launch_ref_setup(theta, net, waveform, d_cst, s);
    if (e == hipSuccess) e = launch_strain(d_cst, waveform, taper, n_det, f_low, delta_f, n_freq, out_dev, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(d_cst);
    if (e != hipSuccess) return hip_fail(e, "rbl_strain");
    return RBL_OK;
}

extern "C" int rbl_event_get_summary(const rbl_event* ev, double* host_out) {
    if (!ev || !host_out) return fail(RBL_EINVAL, "rbl_event_get_summary: null pointer");
    hipError_t e = hipMemcpy(host_out, ev->d_summary, sizeof(double) * ev->n_det * ev->n_bins * 7, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "rbl_event_get_summary");
    return RBL_OK;
}

extern "C" int rbl_event_get_edges(const rbl_event* ev, int64_t* host_out) {
    if (!ev || !host_out) return fail(RBL_EINVAL, "rbl_event_get_edges: null pointer");
    std::copy(ev->edges.begin(), ev->edges.end(), host_out);
    return RBL_OK;
}

extern "C" int rbl_event_info(const rbl_event* ev, int32_t* n_det, int32_t* n_bins, int32_t* waveform,
                              int64_t* footprint_bytes) {
    if (!ev) return fail(RBL_EINVAL, "rbl_event_info: null event");
    if (n_det) *n_det = ev->n_det;
    if (n_bins) *n_bins = ev->n_bins;
    if (waveform) *waveform = ev->waveform;
    if (footprint_bytes) *footprint_bytes = ev->footprint;
    return RBL_OK;
}
