// Request server: continuous batching of likelihood requests over resident events.
//
// One worker thread owns the streams, the request-buffer pool and the graph cache.
// Callers queue requests (rbl_server_submit) and block on tickets (rbl_server_wait).
// The worker loop:
//   (1) reap finished launches (event query per stream), copying the results from pinned
//       staging to the callers' buffers;
//   (2) admit queued requests in FIFO order while a stream is free and a buffer fits the
//       HBM budget; each launch takes along the requests further back in the queue for the
//       same event, precision and gradient flag (up to kMergeMaxChains chains in all);
//   (3) while launches are in flight, poll their completion events with the mutex
//       released, yielding the core between polls, until one finishes or a request
//       arrives; when nothing is queued or running, capture one pending graph if any, else
//       sleep on a condition variable (or, with RBL_SERVE_SPIN, poll for arrivals with the
//       mutex released).
// Every launch is either one graph replay or the same operations issued one by one.  A
// single request whose (buffer, event, batch, precision, gradient) has no graph yet runs
// as plain launches, and its graph is captured later, when the worker is idle: a capture
// never delays a request in flight.  Merged launches are always plain launches.
#include <time.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "rbl_host.h"

using namespace rbl;

namespace {

int64_t now_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000LL + ts.tv_nsec;
}

constexpr int64_t kMinClass = 256;  // smallest buffer class [chains]
constexpr int kMaxStreams = 16;
constexpr int64_t kMergeMaxChains = 8192;  // chains of one merged launch, at most

int64_t class_of(int64_t B) {
    int64_t c = kMinClass;
    while (c < B) c <<= 1;
    return c;
}

// Device layout of one request buffer of `cap` chains: theta | lnl | grad | workspace
// (cap is a multiple of 256, so lnl occupies exactly cap doubles and grad follows it, as in
// the pinned result buffer).
struct BufLayout {
    int64_t theta, lnl, grad, ws, total;
    explicit BufLayout(int64_t cap)
        : theta(align_up(cap * 13 * (int64_t)sizeof(double))),
          lnl(align_up(cap * (int64_t)sizeof(double))),
          grad(align_up(cap * 13 * (int64_t)sizeof(double))),
          ws(workspace_bytes(cap, true)),
          total(theta + lnl + grad + ws) {}
};

struct Buffer {
    uint64_t id = 0;
    int64_t cap = 0, bytes = 0;
    char* dev = nullptr;
    double* h_theta = nullptr;  // pinned [cap][13]
    double* h_out = nullptr;    // pinned: lnl [cap], then grad [cap][13]
    bool busy = false;
    int64_t last_use = 0;
};

struct Request {
    int64_t ticket = 0;
    int32_t event = 0;
    const rbl_event* ev = nullptr;
    const double* theta = nullptr;
    int64_t B = 0;
    int32_t precision = RBL_FP64;
    bool grad = false;
    double* lnl = nullptr;
    double* gout = nullptr;
    rbl_request_info info{};
    int state = 0;  // 0 queued, 1 running, 2 done
    bool counted_wait = false;
    Buffer* buf = nullptr;
    int64_t off = 0;  // first chain of this request in its launch
};

struct Slot {
    hipStream_t s = nullptr;
    hipEvent_t done = nullptr;
    std::vector<Request*> cur;  // the requests of the launch in flight (empty: free)
};

using GraphKey = std::tuple<uint64_t, int32_t, int64_t, int32_t, int32_t>;  // buffer, event, B, precision, grad

// A graph to capture when the worker is idle: what enqueue() needs of the request.
struct PendingCapture {
    GraphKey key;
    const rbl_event* ev;
    Buffer* buf;
};

}  // namespace

struct rbl_server {
    int device = 0;
    int64_t budget = 0;
    uint32_t flags = 0;
    mutable std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::unordered_map<int64_t, Request*> reqs;
    int64_t next_ticket = 1;
    std::map<int32_t, const rbl_event*> events;
    std::map<int32_t, int64_t> users;  // requests per event not yet waited for
    int32_t next_event = 0;
    int64_t resident = 0;
    int64_t buffer_bytes = 0;
    std::vector<Slot> slots;
    std::vector<std::unique_ptr<Buffer>> bufs;
    uint64_t next_buf = 1;
    std::map<GraphKey, hipGraphExec_t> graphs;
    std::vector<PendingCapture> pending;  // graphs to capture when idle
    rbl_server_stats st{};
    bool stop = false;
    // Submissions and shutdown, readable by the worker without the mutex: it polls its
    // launches and waits for work with the mutex released, so that submitters are never
    // held off by its polling.
    std::atomic<uint64_t> arrivals{0};
    std::atomic<bool> stopping{false};
    std::thread worker;
};

namespace {

// ---- buffers -----------------------------------------------------------------------------

void drop_graphs_if(rbl_server* S, uint64_t buf_id, int32_t event) {
    for (auto it = S->graphs.begin(); it != S->graphs.end();) {
        if (std::get<0>(it->first) == buf_id || std::get<1>(it->first) == event) {
            (void)hipGraphExecDestroy(it->second);
            it = S->graphs.erase(it);
        } else {
            ++it;
        }
    }
    S->pending.erase(std::remove_if(S->pending.begin(), S->pending.end(),
                                    [&](const PendingCapture& p) {
                                        return std::get<0>(p.key) == buf_id || std::get<1>(p.key) == event;
                                    }),
                     S->pending.end());
}

void free_buffer_memory(Buffer* b) {
    if (b->dev) (void)hipFree(b->dev);
    if (b->h_theta) (void)hipHostFree(b->h_theta);
    if (b->h_out) (void)hipHostFree(b->h_out);
    b->dev = nullptr;
    b->h_theta = b->h_out = nullptr;
}

void release_buffer(rbl_server* S, Buffer* b) {
    drop_graphs_if(S, b->id, -1);
    free_buffer_memory(b);
    S->buffer_bytes -= b->bytes;
    S->st.buffer_releases++;
    S->bufs.erase(std::remove_if(S->bufs.begin(), S->bufs.end(), [&](const std::unique_ptr<Buffer>& p) {
                      return p.get() == b;
                  }),
                  S->bufs.end());
}

Buffer* allocate_buffer(rbl_server* S, int64_t cap) {
    auto b = std::make_unique<Buffer>();
    b->id = S->next_buf++;
    b->cap = cap;
    b->bytes = BufLayout(cap).total;
    if (fault_take(RBL_FAULT_ALLOC)) return nullptr;
    if (hipMalloc((void**)&b->dev, (size_t)b->bytes) != hipSuccess ||
        hipHostMalloc((void**)&b->h_theta, (size_t)(cap * 13 * sizeof(double)), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&b->h_out, (size_t)(cap * 14 * sizeof(double)), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        free_buffer_memory(b.get());
        return nullptr;
    }
    S->buffer_bytes += b->bytes;
    S->st.buffer_allocs++;
    S->bufs.push_back(std::move(b));
    return S->bufs.back().get();
}

// A free buffer for B chains: its own class if free; else a new one of its class within
// the budget; else a free larger one; else a new one after releasing idle buffers
// (least recently used first).  nullptr: wait for running requests.
Buffer* acquire(rbl_server* S, int64_t B) {
    const int64_t cap = class_of(B);
    for (auto& b : S->bufs)
        if (!b->busy && b->cap == cap) return b.get();
    const int64_t need = BufLayout(cap).total;
    if (S->resident + S->buffer_bytes + need <= S->budget) {
        if (Buffer* b = allocate_buffer(S, cap)) return b;
    }
    Buffer* larger = nullptr;
    for (auto& b : S->bufs)
        if (!b->busy && b->cap >= B && (!larger || b->cap < larger->cap)) larger = b.get();
    if (larger) return larger;
    while (S->resident + S->buffer_bytes + need > S->budget) {
        Buffer* victim = nullptr;
        for (auto& b : S->bufs)
            if (!b->busy && (!victim || b->last_use < victim->last_use)) victim = b.get();
        if (!victim) return nullptr;
        release_buffer(S, victim);
    }
    return allocate_buffer(S, cap);
}

// A free buffer for a merged launch of B chains without releasing any: a free one of
// B's class or larger, else a new one of its class within the budget.  nullptr: the
// launch goes ahead with the head request alone.
Buffer* acquire_no_evict(rbl_server* S, int64_t B) {
    const int64_t cap = class_of(B);
    Buffer* best = nullptr;
    for (auto& b : S->bufs)
        if (!b->busy && b->cap >= cap && (!best || b->cap < best->cap)) best = b.get();
    if (best) return best;
    if (S->resident + S->buffer_bytes + BufLayout(cap).total <= S->budget) return allocate_buffer(S, cap);
    return nullptr;
}

// ---- launches ----------------------------------------------------------------------------

hipError_t enqueue(const Request* r, const Buffer* b, hipStream_t s) {
    const int64_t B = r->B;
    const BufLayout lay(b->cap);
    double* d_theta = (double*)b->dev;
    double* d_lnl = (double*)(b->dev + lay.theta);
    double* d_grad = (double*)(b->dev + lay.theta + lay.lnl);
    char* ws = b->dev + lay.theta + lay.lnl + lay.grad;
    double* rec = (double*)ws;
    double* jac = r->grad ? (double*)(ws + align_up(B * kRecStride * (int64_t)sizeof(double))) : nullptr;
    const bool mixed = r->precision == RBL_MIXED;
    hipError_t e = hipMemcpyAsync(d_theta, b->h_theta, (size_t)(B * 13 * sizeof(double)), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    e = launch_chain_setup(d_theta, B, r->ev->net, r->ev->ref, rec, jac, s);
    if (e != hipSuccess) return e;
    e = r->grad ? launch_loglike_grad(r->ev->dev, rec, jac, B, mixed, d_lnl, d_grad, s)
                : launch_loglike(r->ev->dev, rec, B, mixed, d_lnl, s);
    if (e != hipSuccess) return e;
    // lnl [cap] and grad [cap][13] are contiguous on both sides: one copy back
    const size_t out_bytes = r->grad ? (size_t)((b->cap + B * 13) * sizeof(double)) : (size_t)(B * sizeof(double));
    return hipMemcpyAsync(b->h_out, d_lnl, out_bytes, hipMemcpyDeviceToHost, s);
}

hipGraphExec_t capture(const Request* r, const Buffer* b, hipStream_t s) {
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    const hipError_t e = enqueue(r, b, s);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s, &g);
    hipGraphExec_t ex = nullptr;
    if (e == hipSuccess && e2 == hipSuccess && g) {
        if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) ex = nullptr;
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return ex;
}

void complete(rbl_server* S, Request* r, int status) {
    r->info.status = status;
    r->info.t_done_ns = now_ns();
    r->state = 2;
    S->st.completed++;
}

// Launch a group of requests of one event, precision and gradient flag as one batch of
// `total` chains in buffer b (their theta back to back, in group order).  A group of one
// replays its graph when there is one.  Called with the mutex held (lk); the copy of theta
// into the pinned staging and the launches run with it released, so that submitters are
// not held off.  The slot, the buffer and the group's requests are the worker's alone
// meanwhile: a running request cannot be waited for, and its event cannot be removed.
void launch(rbl_server* S, std::unique_lock<std::mutex>& lk, const std::vector<Request*>& group, int64_t total,
            Buffer* b, int si) {
    Slot& sl = S->slots[si];
    Request* r = group.front();
    const int64_t t_admit = now_ns();
    int64_t off = 0;
    for (Request* q : group) {
        q->off = off;
        q->buf = b;
        q->state = 1;
        q->info.stream = si;
        q->info.t_admit_ns = t_admit;
        off += q->B;
    }
    b->busy = true;
    hipGraphExec_t ex = nullptr;
    if (group.size() == 1 && !(S->flags & RBL_SERVE_NO_GRAPHS)) {
        const GraphKey k{b->id, r->event, r->B, r->precision, r->grad ? 1 : 0};
        auto it = S->graphs.find(k);
        if (it != S->graphs.end()) {
            ex = it->second;
        } else if (std::none_of(S->pending.begin(), S->pending.end(),
                                [&](const PendingCapture& p) { return p.key == k; })) {
            S->pending.push_back(PendingCapture{k, r->ev, b});
        }
    }
    lk.unlock();
    for (Request* q : group)
        std::memcpy(b->h_theta + q->off * 13, q->theta, (size_t)(q->B * 13 * sizeof(double)));
    hipError_t e;
    if (ex) {
        e = hipGraphLaunch(ex, sl.s);
    } else {
        Request m = *r;  // the batch: the head's event, precision and gradient flag
        m.B = total;
        e = enqueue(&m, b, sl.s);
    }
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.s);
    if (e != hipSuccess) (void)hipStreamSynchronize(sl.s);
    lk.lock();
    if (ex) {
        S->st.graph_launches++;
    } else {
        S->st.plain_launches++;
        if (group.size() > 1) {
            S->st.merged_launches++;
            S->st.merged_requests += (int64_t)group.size();
        }
    }
    if (e != hipSuccess) {
        b->busy = false;
        const int rc = hip_fail(e, "rbl_server: launch");
        for (Request* q : group) complete(S, q, rc);
        S->cv_done.notify_all();
        return;
    }
    sl.cur = group;
    S->st.in_flight += (int64_t)group.size();
    S->st.max_in_flight = std::max(S->st.max_in_flight, S->st.in_flight);
}

// Capture one pending graph on an idle stream (called only with nothing in flight).
void capture_one(rbl_server* S) {
    const PendingCapture p = S->pending.back();
    S->pending.pop_back();
    if (S->graphs.count(p.key)) return;
    Request r;
    r.event = std::get<1>(p.key);
    r.ev = p.ev;
    r.B = std::get<2>(p.key);
    r.precision = std::get<3>(p.key);
    r.grad = std::get<4>(p.key) != 0;
    if (hipGraphExec_t ex = capture(&r, p.buf, S->slots[0].s)) {
        S->graphs.emplace(p.key, ex);
        S->st.graphs++;
    }
}

// Finished launches: their results are copied to the callers' buffers with the mutex
// released (lk held on entry and on return), then their requests complete.
bool reap(rbl_server* S, std::unique_lock<std::mutex>& lk) {
    std::vector<std::pair<Slot*, int>> fin;
    for (auto& sl : S->slots) {
        if (sl.cur.empty()) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        fin.emplace_back(&sl, q == hipSuccess ? RBL_OK : hip_fail(q, "rbl_server: request"));
    }
    if (fin.empty()) return false;
    lk.unlock();
    for (auto& [sl, status] : fin) {
        if (status != RBL_OK) continue;
        const Buffer* b = sl->cur.front()->buf;
        for (Request* r : sl->cur) {
            std::memcpy(r->lnl, b->h_out + r->off, (size_t)(r->B * sizeof(double)));
            if (r->grad)
                std::memcpy(r->gout, b->h_out + b->cap + r->off * 13, (size_t)(r->B * 13 * sizeof(double)));
        }
    }
    lk.lock();
    for (auto& [sl, status] : fin) {
        Buffer* b = sl->cur.front()->buf;
        for (Request* r : sl->cur) complete(S, r, status);
        b->busy = false;
        b->last_use = now_ns();
        S->st.in_flight -= (int64_t)sl->cur.size();
        sl->cur.clear();
    }
    S->cv_done.notify_all();
    return true;
}

void admit(rbl_server* S, std::unique_lock<std::mutex>& lk) {
    while (!S->queue.empty()) {
        int si = -1;
        for (int i = 0; i < (int)S->slots.size(); ++i)
            if (S->slots[i].cur.empty()) {
                si = i;
                break;
            }
        if (si < 0) return;
        Request* r = S->queue.front();
        std::vector<Request*> group{r};
        int64_t total = r->B;
        if (!(S->flags & RBL_SERVE_NO_MERGE)) {
            for (auto it = std::next(S->queue.begin()); it != S->queue.end(); ++it) {
                Request* q = *it;
                if (q->event == r->event && q->precision == r->precision && q->grad == r->grad &&
                    total + q->B <= kMergeMaxChains) {
                    group.push_back(q);
                    total += q->B;
                }
            }
        }
        Buffer* b = group.size() > 1 ? acquire_no_evict(S, total) : nullptr;
        if (!b) {  // the head alone
            group.resize(1);
            total = r->B;
            b = acquire(S, total);
        }
        if (!b) {
            if (!r->counted_wait) {
                r->counted_wait = true;
                S->st.admission_waits++;
            }
            return;
        }
        if (group.size() == 1) {
            S->queue.pop_front();
        } else {
            for (Request* q : group) q->state = 1;  // running from here on
            S->queue.erase(std::remove_if(S->queue.begin(), S->queue.end(), [](Request* q) { return q->state == 1; }),
                           S->queue.end());
        }
        launch(S, lk, group, total, b, si);
    }
}

void worker_main(rbl_server* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        reap(S, lk);
        admit(S, lk);
        if (S->st.in_flight > 0) {
            // Poll the launches in flight with the mutex released (the slots belong to this
            // thread), until one finishes or a new request arrives.
            const uint64_t seen = S->arrivals.load(std::memory_order_acquire);
            lk.unlock();
            for (bool done = false; !done;) {
                for (auto& sl : S->slots)
                    if (!sl.cur.empty() && hipEventQuery(sl.done) != hipErrorNotReady) done = true;
                if (!done && S->arrivals.load(std::memory_order_acquire) == seen) std::this_thread::yield();
                else done = true;
            }
            lk.lock();
            continue;
        }
        if (!S->queue.empty()) {
            // nothing runs and the head still does not fit: it never will
            Request* r = S->queue.front();
            S->queue.pop_front();
            complete(S, r, fail(RBL_ENOMEM, "rbl_server: request buffer does not fit in the HBM budget"));
            S->cv_done.notify_all();
            continue;
        }
        if (!S->pending.empty() && !S->stop) {
            capture_one(S);
            continue;
        }
        if (S->stop) break;
        if (S->flags & RBL_SERVE_SPIN) {
            const uint64_t seen = S->arrivals.load(std::memory_order_acquire);
            lk.unlock();
            while (S->arrivals.load(std::memory_order_acquire) == seen && !S->stopping.load(std::memory_order_acquire))
                std::this_thread::yield();
            lk.lock();
            continue;
        }
        S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
    }
}

}  // namespace

extern "C" int64_t rbl_clock_ns(void) { return now_ns(); }

extern "C" int rbl_server_create(int64_t hbm_budget_bytes, int32_t n_streams, uint32_t flags, rbl_server** out) {
    if (!out) return fail(RBL_EINVAL, "rbl_server_create: null output");
    *out = nullptr;
    if (hbm_budget_bytes <= 0) return fail(RBL_EINVAL, "rbl_server_create: budget must be positive");
    if (n_streams < 1 || n_streams > kMaxStreams) return fail(RBL_EINVAL, "rbl_server_create: n_streams not in 1..16");
    auto S = std::make_unique<rbl_server>();
    S->budget = hbm_budget_bytes;
    S->flags = flags;
    hipError_t e = hipGetDevice(&S->device);
    if (e != hipSuccess) return hip_fail(e, "rbl_server_create: device");
    S->slots.resize((size_t)n_streams);
    for (auto& sl : S->slots) {
        if ((e = hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess) {
            for (auto& t : S->slots) {
                if (t.s) (void)hipStreamDestroy(t.s);
                if (t.done) (void)hipEventDestroy(t.done);
            }
            return hip_fail(e, "rbl_server_create: streams");
        }
    }
    S->st.budget_bytes = hbm_budget_bytes;
    rbl_server* p = S.release();
    p->worker = std::thread(worker_main, p);
    *out = p;
    return RBL_OK;
}

extern "C" int rbl_server_add_event(rbl_server* S, const rbl_event* ev, int32_t* event_id) {
    if (!S || !ev || !event_id) return fail(RBL_EINVAL, "rbl_server_add_event: null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->resident + ev->footprint + S->buffer_bytes > S->budget)
        return fail(RBL_ENOMEM, "rbl_server_add_event: event footprint exceeds the HBM budget");
    const int32_t id = S->next_event++;
    S->events[id] = ev;
    S->users[id] = 0;
    S->resident += ev->footprint;
    *event_id = id;
    return RBL_OK;
}

extern "C" int rbl_server_remove_event(rbl_server* S, int32_t event_id) {
    if (!S) return fail(RBL_EINVAL, "rbl_server_remove_event: null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->events.find(event_id);
    if (it == S->events.end()) return fail(RBL_EINVAL, "rbl_server_remove_event: unknown event");
    if (S->users[event_id] > 0) return fail(RBL_EINVAL, "rbl_server_remove_event: requests pending");
    S->resident -= it->second->footprint;
    S->events.erase(it);
    S->users.erase(event_id);
    drop_graphs_if(S, 0, event_id);
    return RBL_OK;
}

extern "C" int rbl_server_submit(rbl_server* S, int32_t event_id, const double* theta_host, int64_t B,
                                 int32_t precision, int32_t with_grad, double* lnl_host, double* grad_host,
                                 int64_t t_arrival_ns, int64_t* ticket) {
    const int64_t t_sub = now_ns();
    if (!S || !ticket) return fail(RBL_EINVAL, "rbl_server_submit: null argument");
    if (B < 0 || B > ((int64_t)1 << 31)) return fail(RBL_EINVAL, "rbl_server_submit: B out of range");
    if (precision != RBL_FP64 && precision != RBL_MIXED) return fail(RBL_EINVAL, "rbl_server_submit: unknown precision");
    if (B > 0 && (!theta_host || !lnl_host || (with_grad && !grad_host)))
        return fail(RBL_EINVAL, "rbl_server_submit: null theta or output");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->events.find(event_id);
    if (it == S->events.end()) return fail(RBL_EINVAL, "rbl_server_submit: unknown event");
    if (B > 0 && S->resident + BufLayout(class_of(B)).total > S->budget)
        return fail(RBL_ENOMEM, "rbl_server_submit: request buffer can never fit in the HBM budget");
    auto* r = new Request();
    r->ticket = S->next_ticket++;
    r->event = event_id;
    r->ev = it->second;
    r->theta = theta_host;
    r->B = B;
    r->precision = precision;
    r->grad = with_grad != 0;
    r->lnl = lnl_host;
    r->gout = grad_host;
    r->info.t_arrival_ns = t_arrival_ns > 0 ? t_arrival_ns : t_sub;
    r->info.stream = -1;
    S->reqs[r->ticket] = r;
    S->users[event_id]++;
    S->st.submitted++;
    *ticket = r->ticket;
    if (B == 0) {
        r->info.t_admit_ns = t_sub;
        complete(S, r, RBL_OK);
        return RBL_OK;
    }
    S->queue.push_back(r);
    S->arrivals.fetch_add(1, std::memory_order_release);
    S->cv_work.notify_one();
    return RBL_OK;
}

extern "C" int rbl_server_wait(rbl_server* S, int64_t ticket, rbl_request_info* info) {
    if (!S) return fail(RBL_EINVAL, "rbl_server_wait: null server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(RBL_EINVAL, "rbl_server_wait: unknown ticket");
    Request* r = it->second;
    S->cv_done.wait(lk, [&] { return r->state == 2; });
    if (info) *info = r->info;
    const int status = r->info.status;
    S->users[r->event]--;
    S->reqs.erase(it);
    delete r;
    if (status != RBL_OK) return fail(status, "rbl_server_wait: request failed");
    return RBL_OK;
}

extern "C" int rbl_server_get_stats(const rbl_server* S, rbl_server_stats* out) {
    if (!S || !out) return fail(RBL_EINVAL, "rbl_server_get_stats: null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->budget_bytes = S->budget;
    out->resident_bytes = S->resident;
    out->buffer_bytes = S->buffer_bytes;
    out->queued = (int64_t)S->queue.size();
    return RBL_OK;
}

extern "C" void rbl_server_destroy(rbl_server* S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->stopping.store(true, std::memory_order_release);
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (auto& kv : S->graphs) (void)hipGraphExecDestroy(kv.second);
    S->graphs.clear();
    for (auto& b : S->bufs) free_buffer_memory(b.get());
    S->bufs.clear();
    for (auto& sl : S->slots) {
        (void)hipStreamDestroy(sl.s);
        (void)hipEventDestroy(sl.done);
    }
    for (auto& kv : S->reqs) delete kv.second;
    delete S;
}
