/*
 * rbl — batched relative-binned Whittle log-likelihood and its 13-parameter
 * gradient for binary-neutron-star signals, on one AMD Instinct MI355X (gfx950).
 *
 * The calls follow the statement of the problem in arXiv:2404.11397:
 *   Sec. II A, Eqs. (2)-(3): Whittle log-likelihood with the noise-weighted
 *     inner product <a, b> = 4 Re sum_k a_k conj(b_k) / S_k  df   over the grid
 *     f_k = f_low + k df (both band ends included), up to a theta-independent
 *     constant:  lnL = sum_det [ Re <d, h>_c - <h, h> / 2 ];
 *   Sec. II C, Eqs. (4)-(5): relative binning — the ratio r = h(theta)/h(theta0)
 *     is taken at the bin edges and modelled as linear inside each bin about
 *     the bin centre, so lnL reduces to sums over bins of precomputed summary
 *     data (A0, A1, B0, B1) and the ratio;
 *   Sec. II B: TaylorF2 and IMRPhenomD_NRTidalv2 waveforms; Tab. II: the 13
 *     parameters.
 *
 * Parameter vector theta (float64, 13 per chain, row-major [B][13]):
 *   0 Mc [Msun, detector frame]  1 q = m2/m1  2 chi1  3 chi2  4 Lambda1  5 Lambda2
 *   6 dL [Mpc]  7 tc [s]  8 phic [rad, orbital]  9 iota  10 psi  11 ra  12 dec [rad]
 *
 * Conventions: h_d(f) = (C_d/dL) A(f) exp(-i Psi_int(f)) exp(2i phic)
 *   exp(-2 pi i f (tc + dt_d)), C_d = (1+cos^2 iota)/2 F+_d - i cos(iota) Fx_d,
 *   F = D : e with the detector tensor D, dt_d = -(r_d . n)/c, n the source
 *   direction at hour angle ra - gmst; Earth rotation over a segment ignored.
 *
 * Errors: every call returns RBL_OK (0) or a negative code; rbl_last_error()
 * gives a message (thread-local).  Argument errors are reported before any
 * work is enqueued.  Device errors surface at the call or at the next call.
 * Nothing aborts.  Per-chain domain problems are not call errors: a NaN in a
 * chain's theta gives lnL = NaN and a NaN gradient row; a finite theta outside
 * the physical domain (Mc <= 0, q <= 0, dL <= 0, |chi| >= 1, Lambda < 0) gives
 * lnL = -inf and a zero gradient row.  q > 1 is allowed (labels swapped).
 *
 * Ownership: the caller owns theta, lnL, grad and the workspace (device
 * memory).  An event owns its device buffers from rbl_event_create to
 * rbl_event_free and is immutable in between, so calls on one event from
 * different streams may overlap provided each call has its own workspace.
 * Nothing is retained after a call returns.
 */
#ifndef RBL_H
#define RBL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RBL_OK = 0,
    RBL_EINVAL = -1,   /* null pointer, negative size, bad enum, n_det not 1..3 */
    RBL_EEDGES = -2,   /* bin edges not strictly increasing / outside the grid / ends wrong */
    RBL_EPSD = -3,     /* PSD <= 0 or not finite */
    RBL_ENOMEM = -4,   /* device allocation failed */
    RBL_EDEVICE = -5,  /* HIP runtime error (message in rbl_last_error) */
    RBL_EREF = -6,     /* reference waveform zero or not finite at a bin edge */
    RBL_EUNSUPPORTED = -7 /* feature not available for this event (e.g. no grid kept) */
};

enum { RBL_TAYLORF2 = 0, RBL_PHENOMD_NRTV2 = 1 };
enum { RBL_FP64 = 0, RBL_MIXED = 1 };

/* Event flags. */
#define RBL_KEEP_B2          0x1u  /* keep the second-order B2 term of <h, h> (Sec. II C reading) */
#define RBL_REF_TAPER        0x2u  /* taper the IMRPhenomD_NRTidalv2 reference too (the paper's
                                      pipeline does not, Sec. II C 1) */
#define RBL_KEEP_GRID        0x4u  /* keep data and PSD resident for rbl_loglike_full */
#define RBL_INPUT_ON_DEVICE  0x8u  /* data and psd are device pointers */
#define RBL_CENTRE_NODES     0x10u /* Eq. (5) with r0 = r(f_m), the ratio at each bin centre, and
                                      r1 from the edges: 2 n_bins + 1 waveform evaluations per
                                      chain instead of n_bins + 1 (same summary data); not with
                                      RBL_KEEP_B2 (RBL_EUNSUPPORTED) */

typedef struct rbl_event rbl_event;

typedef struct {
    int32_t n_det;            /* 1..3 */
    int32_t waveform;         /* RBL_TAYLORF2 | RBL_PHENOMD_NRTV2 */
    int32_t n_bins;           /* >= 1 */
    uint32_t flags;           /* RBL_* flags above */
    int64_t n_freq;           /* grid size N >= 2 */
    double f_low;             /* first grid frequency [Hz] > 0 */
    double delta_f;           /* grid spacing [Hz] = 1/T > 0 */
    double gmst;              /* Greenwich mean sidereal time of the segment [rad] */
    const double *data;       /* complex strain, interleaved [n_det][n_freq][2]; host unless
                                 RBL_INPUT_ON_DEVICE; copied, not retained */
    const double *psd;        /* one-sided PSD [n_det][n_freq], > 0 and finite; same placement */
    const double *det_tensor; /* host [n_det][3][3], Earth-fixed, D = (x x^T - y y^T)/2 */
    const double *det_vertex; /* host [n_det][3], Earth-fixed vertex position [m] */
    const double *theta_ref;  /* host [13], the fiducial (reference) parameters theta0 */
    const int64_t *edges;     /* host [n_bins + 1] grid indices of the bin edges: strictly
                                 increasing, first 0, last n_freq - 1 (Sec. II C); or NULL to
                                 place them on the device by the post-Newtonian phase-bound
                                 ansatz of rbl_bin_edges (rbl_event_get_edges returns them) */
} rbl_event_desc;

/* Build the event (the summary-data step of Sec. II C): reference waveform on the
 * full grid, per-(detector, bin) summary data A0, A1, B0, B1 (and B2), and the
 * per-edge coefficient tables used by the likelihood kernels.  Enqueued on
 * `hip_stream` (NULL = default stream) and completed before returning.
 * Returns RBL_EREF if the reference strain vanishes at a bin edge of some
 * detector (the ratio of Eq. (4) is then undefined). */
int rbl_event_create(const rbl_event_desc *desc, void *hip_stream, rbl_event **out);
void rbl_event_free(rbl_event *ev);

/* Bytes of device workspace that rbl_loglike / rbl_loglike_grad need for B chains; for an
 * event created with RBL_KEEP_GRID the size also covers rbl_loglike_full for B chains. */
int64_t rbl_workspace_bytes(const rbl_event *ev, int64_t B, int32_t with_grad);

/* Relative-binned lnL (Eq. (2) with Eqs. (4)-(5)) for B chains.
 * theta_dev [B][13], lnl_dev [B]: device float64.  workspace: device, at least
 * rbl_workspace_bytes(ev, B, 0) bytes, 256-byte aligned.  precision: RBL_FP64 or
 * RBL_MIXED (phase in FP64, reduced to revolutions; sin/cos, amplitude and per-bin
 * products in FP32; final sums in FP64).  Asynchronous on hip_stream.  B = 0 is a no-op. */
int rbl_loglike(const rbl_event *ev, const double *theta_dev, int64_t B, int32_t precision,
                double *lnl_dev, void *workspace, void *hip_stream);

/* lnL and its gradient with respect to the 13 parameters (angles iota and dec as
 * angles), by a hand-written adjoint of the relative-binned sum.  grad_dev [B][13]. */
int rbl_loglike_grad(const rbl_event *ev, const double *theta_dev, int64_t B, int32_t precision,
                     double *lnl_dev, double *grad_dev, void *workspace, void *hip_stream);

/* Largest batch of rbl_loglike_grad_noalloc. */
#define RBL_NOALLOC_MAX_CHAINS 16384

/* rbl_loglike_grad for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): no workspace argument and
 * no allocation.  Same arguments otherwise, same kernels, same results as rbl_loglike_grad.
 * The per-chain records and Jacobians live in a static device array of the library, sized
 * for RBL_NOALLOC_MAX_CHAINS chains (33 MiB), of which each GPU holds its own copy from
 * library load until the process ends.  The call makes no hipMalloc, hipFree or other
 * allocating call; its first call on a device looks up that device's copy of the array once.
 * Every call on one GPU uses that GPU's array: calls that overlap on one GPU (on different
 * streams or from several threads) race and corrupt each other's results, so serialise them
 * (calls on one stream are serial).  The array keeps the last call's contents; nothing in it
 * needs clearing before a call.  Errors: RBL_EINVAL for B > RBL_NOALLOC_MAX_CHAINS, B < 0,
 * a null pointer, an unknown precision, or a current device other than the one the event was
 * created on; RBL_EDEVICE for HIP errors.  B = 0 is a no-op. */
int rbl_loglike_grad_noalloc(const rbl_event *ev, const double *theta_dev, int64_t B, int32_t precision,
                             double *lnl_dev, double *grad_dev, void *hip_stream);

/* Full-grid lnL (Eqs. (2)-(3) without binning), FP64; needs RBL_KEEP_GRID.  Workspace: at
 * least rbl_workspace_bytes(ev, B, 0) bytes of that event, 256-byte aligned.  Used for
 * validation, to report the binning error, and as the likelihood of the reference-parameter
 * search (no reference is needed for it beyond the event's own data). */
int rbl_loglike_full(const rbl_event *ev, const double *theta_dev, int64_t B, double *lnl_dev,
                     void *workspace, void *hip_stream);

/* Reference-parameter search (Sec. II C: the maximum-likelihood estimate that relative
 * binning needs as theta_ref for real data): CMA-ES (Hansen's (mu/mu_w, lambda)-CMA-ES with
 * cumulative step-size adaptation and its default constants) maximising the full-band lnL of
 * Eqs. (2)-(3), taper included, over the box [lo, hi] (host [13] each); the event must have
 * RBL_KEEP_GRID (its own theta_ref does not enter).  n_starts (>= 1) independent runs, run r
 * from starts[r] (host [n_starts][13], inside the box), each with initial step sigma0 (> 0,
 * in box-normalised coordinates) and lambda (>= 4) candidates per generation; candidates
 * outside the box rank last.  The runs advance together: one device evaluation per
 * generation covers the populations of every run still going (lambda n_starts <= 2^20).
 * normals: host [n_starts][generations][lambda][13] standard normals, the caller's random
 * numbers.  Run r ends early, after generations_run[r] generations, when its covariance can
 * no longer be factored, its Cholesky diagonal spans more than 1e7 (conditioning above
 * 1e14), or its largest step exceeds the box width.  Outputs (host): best_theta [13] and
 * best_lnl, the best candidate over all runs (the first one seen on a tie, runs in order);
 * generations_run [n_starts]; trace (may be NULL) [n_starts][generations][15] = (the run's
 * best lnL so far, sigma, mean theta [13]) after each of its generations (rows past
 * generations_run[r] are left untouched).  Synchronous on hip_stream; allocates its device
 * buffers for the duration of the call. */
int rbl_ref_search(const rbl_event *ev, const double *lo, const double *hi, int32_t n_starts, const double *starts,
                   double sigma0, int32_t lambda, int32_t generations, const double *normals, double *best_theta,
                   double *best_lnl, double *trace, int32_t *generations_run, void *hip_stream);

/* Projected strain h_d(f_k; theta) on a grid for one parameter vector (host theta[13]);
 * out_dev [n_det][n_freq][2] complex float64, device.  `taper` selects the Planck taper
 * of IMRPhenomD_NRTidalv2 (ignored for TaylorF2).  Used to make injections. */
int rbl_strain(int32_t waveform, int32_t n_det, const double *det_tensor, const double *det_vertex,
               double gmst, double f_low, double delta_f, int64_t n_freq, const double *theta,
               int32_t taper, double *out_dev, void *hip_stream);

/* Copy the summary data to host: [n_det][n_bins][7] = (Re A0, Im A0, Re A1, Im A1, B0, B1, B2). */
int rbl_event_get_summary(const rbl_event *ev, double *host_out);

/* Copy the event's bin edges to host: [n_bins + 1] grid indices. */
int rbl_event_get_edges(const rbl_event *ev, int64_t *host_out);

/* Event shape and resident device footprint in bytes. */
int rbl_event_info(const rbl_event *ev, int32_t *n_det, int32_t *n_bins, int32_t *waveform,
                   int64_t *footprint_bytes);

/* Bin edges from the post-Newtonian phase-bound ansatz of Sec. II C (host computation):
 * the phase Phi(f) = sum_g sgn(g) (f/f*_g)^g, g in {-5/3, -2/3, 1, 5/3, 7/3}
 * (f* = f_low for g < 0, f_high for g > 0) is split into n_bins equal steps; each step
 * is snapped to the nearest grid index; indices are made strictly increasing.
 * edges_out [n_bins + 1]. */
int rbl_bin_edges(double f_low, double delta_f, int64_t n_freq, int32_t n_bins, int64_t *edges_out);

/* Kernel timing for benchmarks.  With every = n > 0, the first and then every n-th
 * rbl_loglike / rbl_loglike_grad / rbl_loglike_full / rbl_mala_step call records HIP events
 * on its own stream at the start and end of its setup kernel and of its main kernel (the runtime
 * stamps the kernels themselves); every = 0 turns timing off.  Each timed call costs a
 * few microseconds of device time, so a sampled rate disturbs a throughput run less.
 * rbl_profile_read waits for the recorded events, returns the summed milliseconds of the
 * main and setup kernels and the number of timed calls since the last read, and resets
 * the counters.  RBL_EINVAL for every < 0.  Not for concurrent use from several threads. */
int rbl_profile_enable(int32_t every);
int rbl_profile_read(double *main_ms, double *setup_ms, int64_t *calls);
/* Summed milliseconds of the summary-data pass (reference waveform on the grid and the
 * per-bin reductions) of the events created while profiling was enabled; resets. */
int rbl_profile_read_summary(double *ms, int64_t *events);

const char *rbl_last_error(void);

/* Failure injection for tests of the error paths: from the count-th next device allocation
 * (RBL_FAULT_ALLOC) or likelihood launch (RBL_FAULT_LAUNCH) made by the library on, each one
 * fails as if the device had refused it (the call returns RBL_ENOMEM, resp. RBL_EDEVICE, and
 * leaves the library usable) until the hook is cleared with count = 0.  Process-wide. */
enum { RBL_FAULT_ALLOC = 0, RBL_FAULT_LAUNCH = 1 };
int rbl_debug_inject_fault(int32_t kind, int32_t count);

/* ---------------------------------------------------------------------------------------
 * MALA local step (the gradient-based local sampler of Sec. II D) on the device.
 *
 * A chain's state is z [13] = (Mc, q, chi1, chi2, Lambda1, Lambda2, dL, tc, phic, cos iota,
 * psi, ra, sin delta) -- the coordinates in which Tab. II's priors are uniform -- with its
 * lnL and gz = d lnL / dz.  All arrays are device float64, row-major [B][13] / [B]. */

/* Bytes of device workspace (256-byte aligned) that rbl_mala_init / rbl_mala_step need. */
int64_t rbl_mala_workspace_bytes(const rbl_event *ev, int64_t B);

/* lnL and gz at z for B chains (the state before the first step). */
int rbl_mala_init(const rbl_event *ev, const double *z_dev, int64_t B, int32_t precision, double *lnl_dev,
                  double *gz_dev, void *workspace, void *hip_stream);

/* One step for B chains, in place on z, lnl, gz: propose z' = z + (s/2) gz + sqrt(s) xi,
 * evaluate lnL and its gradient at z', accept when z' lies in the prior box [lo, hi] and
 * log u < lnL' - lnL + log q(z|z') - log q(z'|z), log q(b|a) = -sum (b - a - s g(a)/2)^2 / (2 s).
 * step (s, > 0), lo, hi: host [13]; xi_dev [B][13] standard normals and logu_dev [B] (log of
 * uniforms on (0, 1)) are the caller's random numbers; accepted_dev [B] int32 receives 1 / 0.
 * Asynchronous on hip_stream. */
int rbl_mala_step(const rbl_event *ev, double *z_dev, double *lnl_dev, double *gz_dev, int64_t B,
                  int32_t precision, const double *step, const double *lo, const double *hi,
                  const double *xi_dev, const double *logu_dev, int32_t *accepted_dev, void *workspace,
                  void *hip_stream);

/* ---------------------------------------------------------------------------------------
 * Serving: continuous batching of likelihood requests over many resident events (the
 * sampler of Sec. II D evaluates thousands of chains per step; a service answers such
 * batches for many events at once).
 *
 * A server owns a worker thread, n_streams HIP streams of the device that was current at
 * rbl_server_create, and a pool of request buffers (device: theta, lnL, grad and
 * workspace; pinned host: theta and results) in power-of-two size classes of at least
 * 256 chains.  Admission is by HBM footprint: the resident bytes of the registered events
 * plus the bytes of the pool never exceed hbm_budget_bytes.  Requests are admitted in
 * arrival order (FIFO) as soon as a stream is free and a buffer of their class is free
 * or can be allocated within the budget (idle buffers of other classes are released to
 * make room); otherwise they wait (back-pressure).  Admitted requests run concurrently,
 * one launch per stream.  A launch takes along the requests queued behind the head for
 * the same event, precision and gradient flag, up to 8192 chains in all, as one batch
 * (RBL_SERVE_NO_MERGE: one request per launch).  A launch of one request runs as one
 * persistent hipGraph replay (copy in, per-chain setup, likelihood kernel, copy out) kept
 * per (buffer, event, B, precision, gradient); a request with no graph yet, and every
 * merged launch, runs as plain launches, and the request's graph is captured the next
 * time the worker is idle, so that no capture delays a request; RBL_SERVE_NO_GRAPHS
 * makes plain launches always.  While requests are in flight the worker polls their completion
 * events (yielding the core between polls).  Results are bitwise identical to rbl_loglike / rbl_loglike_grad on the same
 * theta: no value is reduced across chains or requests.
 *
 * Times are host CLOCK_MONOTONIC nanoseconds (rbl_clock_ns). */
typedef struct rbl_server rbl_server;

#define RBL_SERVE_NO_GRAPHS 0x1u  /* plain launches instead of graph replays */
#define RBL_SERVE_SPIN      0x2u  /* the worker polls for new requests instead of sleeping
                                     while idle: lowest admission latency, one busy host core */
#define RBL_SERVE_NO_MERGE  0x4u  /* one launch per request: queued requests of the head's
                                     event are not taken into its launch */

typedef struct {
    int64_t t_arrival_ns;  /* as given to rbl_server_submit (or the submit time) */
    int64_t t_admit_ns;    /* launched on a stream */
    int64_t t_done_ns;     /* results copied to the caller's buffers */
    int32_t status;        /* RBL_OK, or the error of the request */
    int32_t stream;        /* index of the stream it ran on */
} rbl_request_info;

typedef struct {
    int64_t budget_bytes, resident_bytes, buffer_bytes;
    int64_t submitted, completed, queued, in_flight, max_in_flight;
    int64_t graphs, graph_launches, plain_launches;
    int64_t buffer_allocs, buffer_releases, admission_waits;
    int64_t merged_launches, merged_requests;  /* launches of several requests, and their requests */
} rbl_server_stats;

/* Create a server.  hbm_budget_bytes > 0; n_streams in 1..16.  RBL_ENOMEM if resources
 * cannot be created. */
int rbl_server_create(int64_t hbm_budget_bytes, int32_t n_streams, uint32_t flags, rbl_server **out);

/* Register a resident event (created by rbl_event_create, owned by the caller, alive
 * until removed).  RBL_ENOMEM if its footprint does not fit in the budget next to the
 * events already registered and the current buffer pool. */
int rbl_server_add_event(rbl_server *srv, const rbl_event *ev, int32_t *event_id);

/* Unregister an event; RBL_EINVAL while requests for it have not been waited for. */
int rbl_server_remove_event(rbl_server *srv, int32_t event_id);

/* Queue one request: B chains of theta_host [B][13] (host float64) for a registered event.
 * lnl_host [B] and, if with_grad, grad_host [B][13] receive the results.  The caller keeps
 * all three buffers alive and untouched until rbl_server_wait returns for the ticket.
 * t_arrival_ns = 0 takes the submit time.  RBL_ENOMEM if the request's buffer can never
 * fit in the budget next to the resident events.  B = 0 completes at once. */
int rbl_server_submit(rbl_server *srv, int32_t event_id, const double *theta_host, int64_t B,
                      int32_t precision, int32_t with_grad, double *lnl_host, double *grad_host,
                      int64_t t_arrival_ns, int64_t *ticket);

/* Block until the request has completed, fill info (may be NULL), release the ticket and
 * return the request's status. */
int rbl_server_wait(rbl_server *srv, int64_t ticket, rbl_request_info *info);

int rbl_server_get_stats(const rbl_server *srv, rbl_server_stats *out);

/* Finish every queued and running request, then release the streams, buffers and graphs. */
void rbl_server_destroy(rbl_server *srv);

/* Host monotonic clock used for request times [ns]. */
int64_t rbl_clock_ns(void);

/* Resident device bytes of an event (summary data and edge tables, plus the grid with
 * RBL_KEEP_GRID). */
int64_t rbl_event_footprint_bytes(const rbl_event *ev);

#ifdef __cplusplus
}
#endif
#endif /* RBL_H */
