// Continuous-batching server for task-group ordering requests.
//
// The paper's runtime has a host proxy thread that polls a buffer of
// offloaded tasks, forms the task group, reorders it with the heuristic and
// submits it (Section 6.2).  Here many such groups arrive as requests, and the
// waiting groups live on the device:
//   * two device-resident queues, one per size class (n <= small_max_n:
//     enumerated in full; larger: the learned proposal), each a ring of task
//     rows in HBM.  A request is admitted when its rows fit in its ring; the
//     rings are sized so that the server's own device memory (batch plans,
//     network workspaces, result buffers) plus both rings stay within the
//     memory budget, so admission is by memory.  Admitted rows are copied to
//     the ring by an upload stream;
//   * a scheduler thread keeps up to `streams` batches in flight, each on a
//     HIP stream of its own: a free stream takes the oldest admitted requests
//     of one class that lie back to back in their ring (up to the class's
//     batch size) and launches the batch straight from the ring (the batch
//     kernels read the ring through per-group row offsets), after the uploads
//     it depends on; finished batches are retired by polling their events,
//     which frees their ring rows for requests that arrived meanwhile.
// Small groups run a fixed-shape batch (padded with empty groups, so its
// captured graph is replayed); large groups are sampled with the request's
// key (its id unless the caller gives one), so a request's answer does not
// depend on what it was batched with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "tgo_internal.h"

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    uint64_t id = 0;
    uint32_t key = 0;
    int n = 0;
    int cls = 0;           // 0 = full enumeration, 1 = learned proposal
    tgo_task tasks[TGO_MAX_N];
    int64_t t_arrive = 0, t_admit = 0;
    int64_t pos = 0;       // ring position of its first row (monotonic)
    bool launched = false, done = false;
};

// Device-resident queue of one size class: task rows of admitted requests.
// Positions grow monotonically; row p lives at p % cap.  A request never wraps
// (if it does not fit before the end, the rows up to the end are skipped and
// count as held until the ring's head passes them).
struct Ring {
    tgo_task *d = nullptr;   // device rows
    tgo_task *h = nullptr;   // pinned staging mirror
    int64_t cap = 0;         // rows
    int64_t head = 0, tail = 0;
    std::deque<Request *> q;  // admitted requests in ring order
    int64_t waiting = 0;      // of those, not launched yet
};

struct StreamSlot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    int kind = 0;
    std::vector<Request *> reqs;
    tgo_plan *plan = nullptr;
    tgo_surrogate *sur = nullptr;
    int32_t *d_offs = nullptr;
    uint32_t *d_keys = nullptr;
    unsigned char *d_out = nullptr;
    int32_t *h_offs = nullptr;
    uint32_t *h_keys = nullptr;
    unsigned char *h_out = nullptr;
};

}  // namespace

struct tgo_server {
    tgo_model model;
    tgo_server_config cfg;
    int device = 0;
    std::vector<StreamSlot> slots;
    Ring ring[2];
    hipStream_t up = nullptr;     // uploads into the rings
    hipEvent_t up_ev = nullptr;   // after the last upload
    bool up_pending = false;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request *> arrivals[2];  // submitted, not yet admitted
    std::vector<tgo_server_result> done;
    std::thread worker;
    bool stop = false;
    int64_t base_bytes = 0;       // device memory the server holds for itself
    int64_t in_use = 0, max_in_use = 0;
    uint64_t next_id = 1;
    uint64_t submitted = 0, completed = 0, batches = 0, rejected = 0;
    int64_t max_queue = 0;
    std::string error;
    // Test hook, set from TGO_SERVER_INJECT_QUERY_ERROR=k at creation: the
    // k-th completion query of a busy slot is treated as a device error
    // (the batch itself still runs and ends normally on the GPU).
    int inject_query_error = 0;
};

namespace tgo {

constexpr int64_t RING_MAX_ROWS = int64_t(1) << 22;  // 96 MiB of rows per class at most

static size_t result_bytes(int kind) { return kind == 0 ? sizeof(tgo_summary) : sizeof(tgo_search_result); }

static int64_t ring_held(const Ring &r) { return r.tail - r.head; }

// Bytes of device memory held now: the server's own, plus the ring rows held.
static int64_t held_bytes(const tgo_server *S) {
    return S->base_bytes + (int64_t)sizeof(tgo_task) * (ring_held(S->ring[0]) + ring_held(S->ring[1]));
}

// Admit arrivals whose rows fit in their ring (called with the lock held).
static int admit(tgo_server *S) {
    for (int c = 0; c < 2; ++c) {
        Ring &R = S->ring[c];
        int64_t first = -1, last = -1;  // physical rows to upload, [first, last)
        auto flush = [&]() -> int {
            if (first < 0) return 0;
            TGO_HIP(hipMemcpyAsync(R.d + first, R.h + first, sizeof(tgo_task) * (size_t)(last - first),
                                   hipMemcpyHostToDevice, S->up));
            S->up_pending = true;
            first = last = -1;
            return 0;
        };
        while (!S->arrivals[c].empty()) {
            Request *q = S->arrivals[c].front();
            int64_t pos = R.tail;
            const int64_t off = pos % R.cap;
            if (off + q->n > R.cap) pos += R.cap - off;  // skip to the start of the ring
            if (R.q.empty()) {
                R.head = pos;  // nothing is held: the rows skipped are free too
            } else if (pos + q->n - R.head > R.cap) {
                break;  // no room: wait for memory
            }
            const int64_t phys = pos % R.cap;
            if (first >= 0 && phys != last) {  // not right behind the rows staged so far
                const int rc = flush();
                if (rc) return rc;
            }
            std::memcpy(R.h + phys, q->tasks, sizeof(tgo_task) * (size_t)q->n);
            if (first < 0) first = phys;
            last = phys + q->n;
            q->pos = pos;
            q->t_admit = now_ns();
            R.tail = pos + q->n;
            R.q.push_back(q);
            R.waiting += 1;
            S->arrivals[c].pop_front();
        }
        const int rc = flush();
        if (rc) return rc;
    }
    if (S->up_pending) {
        TGO_HIP(hipEventRecord(S->up_ev, S->up));
        S->up_pending = false;
    }
    S->in_use = held_bytes(S);
    S->max_in_use = std::max(S->max_in_use, S->in_use);
    return 0;
}

// Launch the oldest admitted, unlaunched requests of class `kind` that lie
// back to back in the ring, on slot sl (called with the lock held).
static int launch(tgo_server *S, StreamSlot &sl, int kind) {
    const tgo_server_config &c = S->cfg;
    Ring &R = S->ring[kind];
    const int cap = kind == 0 ? c.max_batch : c.max_batch_large;
    sl.reqs.clear();
    int64_t expect = -1;
    for (Request *q : R.q) {
        if (q->launched) continue;
        if ((int)sl.reqs.size() >= cap) break;
        const int64_t phys = q->pos % R.cap;
        if (expect >= 0 && phys != expect) break;  // wrapped: the next batch takes it
        sl.reqs.push_back(q);
        expect = phys + q->n;
    }
    if (sl.reqs.empty()) return 0;
    for (Request *q : sl.reqs) q->launched = true;
    R.waiting -= (int64_t)sl.reqs.size();
    // row offsets into the ring; the exhaustive batch is padded with empty
    // groups to its fixed shape so that its captured graph is replayed
    const int ng = kind == 0 ? c.max_batch : (int)sl.reqs.size();
    int32_t off = (int32_t)(sl.reqs[0]->pos % R.cap);
    for (int g = 0; g < ng; ++g) {
        sl.h_offs[g] = off;
        if (g < (int)sl.reqs.size()) {
            off += sl.reqs[g]->n;
            sl.h_keys[g] = sl.reqs[g]->key;
        } else {
            sl.h_keys[g] = 0;
        }
    }
    sl.h_offs[ng] = off;
    sl.kind = kind;
    hipStream_t st = sl.st;
    TGO_HIP(hipStreamWaitEvent(st, S->up_ev, 0));
    TGO_HIP(hipMemcpyAsync(sl.d_offs, sl.h_offs, sizeof(int32_t) * (ng + 1), hipMemcpyHostToDevice, st));
    int rc;
    if (kind == 0) {
        rc = tgo_batch(sl.plan, R.d, sl.d_offs, ng, (tgo_summary *)sl.d_out, st);
    } else {
        TGO_HIP(hipMemcpyAsync(sl.d_keys, sl.h_keys, sizeof(uint32_t) * ng, hipMemcpyHostToDevice, st));
        rc = tgo_surrogate_search(sl.sur, &S->model, R.d, sl.d_offs, sl.d_keys, ng, c.samples, c.topk, c.seed,
                                  (tgo_search_result *)sl.d_out, st);
    }
    if (rc) return rc;
    TGO_HIP(hipMemcpyAsync(sl.h_out, sl.d_out, result_bytes(kind) * sl.reqs.size(), hipMemcpyDeviceToHost, st));
    TGO_HIP(hipEventRecord(sl.ev, st));
    sl.busy = true;
    S->batches += 1;
    return 0;
}

// Requests submitted and not yet launched: submitted - completed - in flight.
static int64_t queued_now(const tgo_server *S) {
    int64_t inflight = 0;
    for (const StreamSlot &sl : S->slots) inflight += sl.busy ? (int64_t)sl.reqs.size() : 0;
    return (int64_t)(S->submitted - S->completed) - inflight;
}

static void fill_result(tgo_server_result &o, const Request &q, int kind, const unsigned char *raw, int64_t t_done) {
    std::memset(&o, 0, sizeof(o));
    o.id = q.id;
    o.n = q.n;
    o.path = kind;
    o.t_arrive_ns = q.t_arrive;
    o.t_admit_ns = q.t_admit;
    o.t_done_ns = t_done;
    for (int i = 0; i < 16; ++i) o.best[i] = 0xff;
    if (kind == 0) {
        tgo_summary s;
        std::memcpy(&s, raw, sizeof(s));
        o.status = s.status;
        if (s.status == 0) {
            o.best_ns = s.min_ns;
            o.heur_ns = s.heur_ns;
            std::memcpy(o.best, s.best, 16);
        }
    } else {
        tgo_search_result s;
        std::memcpy(&s, raw, sizeof(s));
        o.status = s.status;
        if (s.status == 0) {
            o.best_ns = s.best_ns;
            o.heur_ns = s.heur_ns;
            std::memcpy(o.best, s.best, 16);
        }
    }
}

// Requests done: free their ring rows from the head on (ring order).
static void release(tgo_server *S, int kind) {
    Ring &R = S->ring[kind];
    while (!R.q.empty() && R.q.front()->done) {
        Request *q = R.q.front();
        R.q.pop_front();
        R.head = R.q.empty() ? R.tail : R.q.front()->pos;
        delete q;
    }
    S->in_use = held_bytes(S);
}

static void retire(tgo_server *S, StreamSlot &sl) {
    const int64_t t = now_ns();
    const size_t rb = result_bytes(sl.kind);
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
        tgo_server_result o;
        fill_result(o, *sl.reqs[i], sl.kind, sl.h_out + i * rb, t);
        S->done.push_back(o);
        sl.reqs[i]->done = true;
    }
    S->completed += sl.reqs.size();
    sl.reqs.clear();
    sl.busy = false;
    release(S, sl.kind);
}

// A batch whose completion query reports a device error, or that could not be
// launched: its requests come back with status TGO_EDEVICE, their rows are
// released, the slot is freed and the server stops (a device error is sticky;
// nothing more is launched).
static void fail_slot(tgo_server *S, StreamSlot &sl, const std::string &why) {
    const int64_t t = now_ns();
    if (S->error.empty()) S->error = why;
    for (Request *q : sl.reqs) {
        tgo_server_result o;
        std::memset(&o, 0, sizeof(o));
        o.id = q->id;
        o.n = q->n;
        o.path = sl.kind;
        o.status = TGO_EDEVICE;
        o.t_arrive_ns = q->t_arrive;
        o.t_admit_ns = q->t_admit;
        o.t_done_ns = t;
        o.best_ns = -1;
        o.heur_ns = -1;
        for (int i = 0; i < 16; ++i) o.best[i] = 0xff;
        S->done.push_back(o);
        q->done = true;
    }
    S->completed += sl.reqs.size();
    sl.reqs.clear();
    sl.busy = false;
    release(S, sl.kind);
    S->stop = true;
}

static void worker_main(tgo_server *S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool progressed = false;
        for (StreamSlot &sl : S->slots) {
            if (!sl.busy) continue;
            hipError_t e = hipEventQuery(sl.ev);
            if (S->inject_query_error > 0 && --S->inject_query_error == 0) e = hipErrorLaunchFailure;
            if (e == hipSuccess) {
                retire(S, sl);
                progressed = true;
            } else if (e != hipErrorNotReady) {
                fail_slot(S, sl, std::string("batch failed on the device: ") + hipGetErrorString(e));
                progressed = true;
            }
        }
        if (!S->stop) {
            if (admit(S)) {
                S->error = std::string("admission failed: ") + tgo_last_error();
                S->stop = true;
            }
        }
        for (StreamSlot &sl : S->slots) {
            if (S->stop || sl.busy) continue;
            // the class whose oldest unlaunched request arrived first goes first
            int kind = -1;
            int64_t oldest = INT64_MAX;
            for (int k = 0; k < 2; ++k) {
                if (k == 1 && !sl.sur) continue;
                for (Request *q : S->ring[k].q)
                    if (!q->launched) {
                        if (q->t_arrive < oldest) { oldest = q->t_arrive; kind = k; }
                        break;
                    }
            }
            if (kind < 0) break;
            // with another batch in flight, give a small batch up to
            // window_us (from its oldest request's arrival) to fill
            const int cap = kind == 0 ? S->cfg.max_batch : S->cfg.max_batch_large;
            if (S->cfg.window_us > 0 && S->ring[kind].waiting < cap &&
                now_ns() - oldest < (int64_t)S->cfg.window_us * 1000) {
                bool other_busy = false;
                for (const StreamSlot &o : S->slots) other_busy |= o.busy;
                if (other_busy) break;
            }
            const int rc = launch(S, sl, kind);
            if (rc) {
                fail_slot(S, sl, std::string("launch failed: ") + tgo_last_error());
                break;
            }
            if (!sl.busy) break;
            progressed = true;
        }
        if (S->stop) {
            bool any_busy = false;
            for (StreamSlot &sl : S->slots) any_busy |= sl.busy;
            if (!any_busy) break;
        }
        S->cv.notify_all();
        if (!progressed) {
            bool any_busy = false;
            for (StreamSlot &sl : S->slots) any_busy |= sl.busy;
            if (any_busy) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
                lk.lock();
            } else {
                S->cv.wait_for(lk, std::chrono::milliseconds(1));
            }
        }
    }
    S->cv.notify_all();
}

static void free_slot(StreamSlot &sl) {
    if (sl.st) (void)hipStreamSynchronize(sl.st);
    if (sl.plan) tgo_plan_destroy(sl.plan);
    if (sl.sur) tgo_surrogate_destroy(sl.sur);
    if (sl.d_offs) (void)hipFree(sl.d_offs);
    if (sl.d_keys) (void)hipFree(sl.d_keys);
    if (sl.d_out) (void)hipFree(sl.d_out);
    if (sl.h_offs) (void)hipHostFree(sl.h_offs);
    if (sl.h_keys) (void)hipHostFree(sl.h_keys);
    if (sl.h_out) (void)hipHostFree(sl.h_out);
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.st) (void)hipStreamDestroy(sl.st);
    sl = StreamSlot();
}

}  // namespace tgo

using namespace tgo;

extern "C" {

void tgo_server_config_default(tgo_server_config *c) {
    if (!c) return;
    c->budget_bytes = (int64_t)8 << 30;
    c->streams = 4;
    c->max_batch = 256;
    c->max_batch_large = 64;
    c->small_max_n = 10;
    c->topk = 64;
    c->window_us = 0;
    c->samples = 8192;
    c->seed = 4;
}

void tgo_server_destroy(tgo_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (int c = 0; c < 2; ++c) {
            for (Request *q : S->arrivals[c]) delete q;
            S->arrivals[c].clear();
        }
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (StreamSlot &sl : S->slots) free_slot(sl);
    if (S->up) (void)hipStreamSynchronize(S->up);
    for (int c = 0; c < 2; ++c) {
        for (Request *q : S->ring[c].q) delete q;
        if (S->ring[c].d) (void)hipFree(S->ring[c].d);
        if (S->ring[c].h) (void)hipHostFree(S->ring[c].h);
    }
    if (S->up_ev) (void)hipEventDestroy(S->up_ev);
    if (S->up) (void)hipStreamDestroy(S->up);
    delete S;
}

int tgo_server_create(const tgo_model *model, const tgo_server_config *cfg, tgo_surrogate *sur,
                      tgo_server **out) {
    if (!out || !cfg) return fail(TGO_EINVAL, "NULL argument");
    *out = nullptr;
    Rates r;
    int rc = make_rates(model, &r);
    if (rc) return rc;
    const tgo_server_config &c = *cfg;
    if (c.streams < 1 || c.streams > 8) return fail(TGO_EINVAL, "streams must be in 1..8");
    if (c.max_batch < 1 || c.max_batch > 4096 || c.max_batch_large < 1 || c.max_batch_large > 4096)
        return fail(TGO_EINVAL, "batch sizes must be in 1..4096");
    if (c.small_max_n < 1 || c.small_max_n > 12) return fail(TGO_EINVAL, "small_max_n must be in 1..12");
    if (c.topk < 1 || c.topk > 64 || c.samples < 1 || c.samples > ((int64_t)1 << 32))
        return fail(TGO_EINVAL, "bad search parameters");
    if (c.budget_bytes <= 0) return fail(TGO_EINVAL, "budget must be positive");
    if (c.window_us < 0 || c.window_us > 100000) return fail(TGO_EINVAL, "window_us must be in 0..100000");
    tgo_server *S = new (std::nothrow) tgo_server();
    if (!S) return fail(TGO_ENOMEM, "server");
    S->model = *model;
    S->cfg = c;
    if (const char *e = std::getenv("TGO_SERVER_INJECT_QUERY_ERROR")) S->inject_query_error = std::atoi(e);
    (void)hipGetDevice(&S->device);
    std::vector<float> params;
    if (sur) {
        params.resize(TGO_SURROGATE_PARAMS);
        rc = tgo_surrogate_get_params(sur, params.data(), nullptr);
        if (rc) {
            delete S;
            return rc;
        }
    }
    S->slots.resize(c.streams);
    const int gmax = std::max(c.max_batch, c.max_batch_large);
    int64_t base = 0;
    for (StreamSlot &sl : S->slots) {
        hipError_t e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(&sl.d_offs, sizeof(int32_t) * (gmax + 1));
        if (e == hipSuccess) e = hipMalloc(&sl.d_keys, sizeof(uint32_t) * gmax);
        if (e == hipSuccess) e = hipMalloc(&sl.d_out, sizeof(tgo_summary) * gmax);
        if (e == hipSuccess) e = hipHostMalloc(&sl.h_offs, sizeof(int32_t) * (gmax + 1));
        if (e == hipSuccess) e = hipHostMalloc(&sl.h_keys, sizeof(uint32_t) * gmax);
        if (e == hipSuccess) e = hipHostMalloc(&sl.h_out, sizeof(tgo_summary) * gmax);
        if (e != hipSuccess) {
            tgo_server_destroy(S);
            return hip_fail(e, "server slot");
        }
        base += (int64_t)(sizeof(int32_t) * (gmax + 1) + sizeof(uint32_t) * gmax + sizeof(tgo_summary) * gmax);
        rc = tgo_plan_create(model, c.max_batch, c.small_max_n, 0, &sl.plan);
        if (!rc) base += (int64_t)plan_device_bytes(sl.plan);
        if (!rc && sur) {
            const int64_t rows = std::max<int64_t>(4096, std::min<int64_t>((int64_t)1 << 16,
                                                   (c.samples + 4095) / 4096 * 4096));
            rc = tgo_surrogate_create(rows, c.max_batch_large, &sl.sur);
            if (!rc) rc = tgo_surrogate_set_params(sl.sur, params.data(), sl.st);
            if (!rc) rc = surrogate_reserve(sl.sur, c.max_batch_large, c.samples);
            if (!rc) base += (int64_t)surrogate_device_bytes(sl.sur);
        }
        if (rc) {
            tgo_server_destroy(S);
            return rc;
        }
    }
    // rings: whatever the budget leaves beyond the server's own memory, split
    // between the classes in proportion to their largest request, at most
    // RING_MAX_ROWS rows each; each must hold at least one request of its class
    S->base_bytes = base;
    const int64_t left_rows = (c.budget_bytes - base) / (int64_t)sizeof(tgo_task);
    const int64_t want[2] = {c.small_max_n, sur ? TGO_MAX_N : 0};
    if (left_rows < want[0] + want[1]) {
        tgo_server_destroy(S);
        return fail(TGO_ENOMEM, "budget below the server's own device memory (" + std::to_string(base) +
                                    " bytes) plus one request per class");
    }
    for (int k = 0; k < 2; ++k) {
        Ring &R = S->ring[k];
        R.cap = want[k] ? std::min<int64_t>(RING_MAX_ROWS, left_rows * want[k] / (want[0] + want[1])) : 1;
        hipError_t e = hipMalloc(&R.d, sizeof(tgo_task) * (size_t)R.cap);
        if (e == hipSuccess) e = hipHostMalloc(&R.h, sizeof(tgo_task) * (size_t)R.cap);
        if (e != hipSuccess) {
            tgo_server_destroy(S);
            return fail(TGO_ENOMEM, std::string("server ring: ") + hipGetErrorString(e));
        }
    }
    hipError_t e = hipStreamCreateWithFlags(&S->up, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&S->up_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(S->up_ev, S->up);
    if (e != hipSuccess) {
        tgo_server_destroy(S);
        return hip_fail(e, "server upload stream");
    }
    S->in_use = S->max_in_use = base;
    S->worker = std::thread(worker_main, S);
    *out = S;
    return TGO_OK;
}

int tgo_server_submit(tgo_server *S, const tgo_task *h_tasks, int n, uint32_t key, uint64_t *id) {
    if (!S || !h_tasks) return fail(TGO_EINVAL, "NULL argument");
    if (n < 1 || n > TGO_MAX_N) return fail(TGO_EINVAL, "n must be in 1..16");
    const int kind = n <= S->cfg.small_max_n ? 0 : 1;
    Request *r = new (std::nothrow) Request();
    if (!r) return fail(TGO_ENOMEM, "request");
    r->n = n;
    r->cls = kind;
    std::memcpy(r->tasks, h_tasks, sizeof(tgo_task) * n);
    r->t_arrive = now_ns();
    uint64_t rid = 0;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) {
            delete r;
            return fail(S->error.empty() ? TGO_EINVAL : TGO_EDEVICE, "server is stopping: " + S->error);
        }
        if (kind == 1 && !S->slots[0].sur) {
            S->rejected += 1;
            delete r;
            return fail(TGO_EINVAL, "no surrogate: groups larger than small_max_n are not served");
        }
        r->id = rid = S->next_id++;
        r->key = key ? key : (uint32_t)r->id;
        S->arrivals[kind].push_back(r);
        S->submitted += 1;
        S->max_queue = std::max(S->max_queue, queued_now(S));
    }
    S->cv.notify_all();
    if (id) *id = rid;
    return TGO_OK;
}

int tgo_server_poll(tgo_server *S, tgo_server_result *out, int max, int *count) {
    if (!S || !count || (max > 0 && !out)) return fail(TGO_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    const int k = std::min<int>(max, (int)S->done.size());
    for (int i = 0; i < k; ++i) out[i] = S->done[i];
    S->done.erase(S->done.begin(), S->done.begin() + k);
    *count = k;
    if (!S->error.empty()) return fail(TGO_EDEVICE, S->error);
    return TGO_OK;
}

int tgo_server_drain(tgo_server *S, int64_t timeout_ms) {
    if (!S) return fail(TGO_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    const auto until = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms);
    while (S->completed < S->submitted && S->error.empty()) {
        if (S->cv.wait_until(lk, until) == std::cv_status::timeout && S->completed < S->submitted)
            return fail(TGO_ERANGE, "drain timed out");
    }
    if (!S->error.empty()) return fail(TGO_EDEVICE, S->error);
    return TGO_OK;
}

int tgo_server_get_stats(tgo_server *S, tgo_server_stats *st) {
    if (!S || !st) return fail(TGO_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    st->submitted = S->submitted;
    st->completed = S->completed;
    st->batches = S->batches;
    st->rejected = S->rejected;
    st->in_use_bytes = S->in_use;
    st->max_in_use_bytes = S->max_in_use;
    st->queued = queued_now(S);
    st->max_queued = S->max_queue;
    st->base_bytes = S->base_bytes;
    st->ring_rows[0] = S->ring[0].cap;
    st->ring_rows[1] = S->ring[1].cap;
    st->budget_bytes = S->cfg.budget_bytes;
    return TGO_OK;
}

int tgo_server_replay(tgo_server *S, const tgo_task *h_tasks, const int32_t *h_offs,
                      const int64_t *h_arrival_ns, int n_requests, tgo_server_result *h_out,
                      int64_t timeout_ms) {
    if (!S || !h_tasks || !h_offs || !h_arrival_ns || !h_out || n_requests < 0)
        return fail(TGO_EINVAL, "NULL argument");
    std::vector<uint64_t> ids(n_requests);
    const int64_t t0 = now_ns();
    for (int i = 0; i < n_requests; ++i) {
        const int64_t due = t0 + (h_arrival_ns[i] - h_arrival_ns[0]);
        while (now_ns() < due) {
            const int64_t left = due - now_ns();
            if (left > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(left - 100000));
        }
        const int rc = tgo_server_submit(S, h_tasks + h_offs[i], h_offs[i + 1] - h_offs[i], 0, &ids[i]);
        if (rc) return rc;
    }
    int rc = tgo_server_drain(S, timeout_ms);
    if (rc) return rc;
    std::vector<tgo_server_result> res(n_requests);
    int got = 0;
    while (got < n_requests) {
        int k = 0;
        rc = tgo_server_poll(S, res.data() + got, n_requests - got, &k);
        if (rc) return rc;
        if (k == 0) break;
        got += k;
    }
    // results in request order (ids are consecutive from the first)
    for (int i = 0; i < got; ++i) {
        const uint64_t idx = res[i].id - ids[0];
        if (idx < (uint64_t)n_requests) h_out[idx] = res[i];
    }
    return got == n_requests ? TGO_OK : fail(TGO_ERANGE, "missing results");
}

}  // extern "C"
