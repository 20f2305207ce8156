// Continuous-batching server for task-group ordering requests.
//
// The paper's runtime has a host proxy thread that polls a buffer of
// offloaded tasks, forms the task group, reorders it with the heuristic and
// submits it (Section 6.2).  Here many such groups arrive as requests.  A
// scheduler thread keeps up to `streams` batches in flight, each on its own
// HIP stream: whenever a stream is free it takes the waiting requests of one
// size class that fit the device-memory budget, copies their task tables into
// the stream's device-resident queue buffers and launches the batch; finished
// batches are retired by polling their events, which frees their slots and
// memory for requests that arrived meanwhile.  Small groups (n <= small_max_n)
// are enumerated exhaustively with a fixed-shape batch (graph replay); larger
// groups go through the learned proposal, keyed by the request's key (its id
// unless the caller gives one) so that a request's answer does not depend on
// what it was batched with.
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
    tgo_task tasks[TGO_MAX_N];
    int64_t t_arrive = 0, t_admit = 0;
    size_t bytes = 0;
};

struct StreamSlot {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    int kind = 0;  // 0 = exhaustive batch, 1 = surrogate search
    std::vector<Request> reqs;
    tgo_plan *plan = nullptr;
    tgo_surrogate *sur = nullptr;
    // device queue buffers
    tgo_task *d_tasks = nullptr;
    int32_t *d_offs = nullptr;
    uint32_t *d_keys = nullptr;
    unsigned char *d_out = nullptr;
    // pinned host mirrors
    tgo_task *h_tasks = nullptr;
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
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Request> pending[2];
    std::vector<tgo_server_result> done;
    std::thread worker;
    bool stop = false;
    int64_t in_use = 0;
    uint64_t next_id = 1;
    uint64_t submitted = 0, completed = 0, batches = 0, rejected = 0;
    int64_t max_in_use = 0;
    int max_queue = 0;
    std::string error;
    // Test hook, set from TGO_SERVER_INJECT_QUERY_ERROR=k at creation: the
    // k-th completion query of a busy slot is treated as a device error
    // (the batch itself still runs and ends normally on the GPU).
    int inject_query_error = 0;
};

namespace tgo {

static size_t request_bytes(const tgo_server_config &c, int n) {
    // what a request holds in the stream queue buffers while in flight
    const bool small = n <= c.small_max_n;
    size_t b = sizeof(tgo_task) * TGO_MAX_N + sizeof(int32_t) + sizeof(uint32_t);
    b += small ? sizeof(tgo_summary) : sizeof(tgo_search_result);
    if (!small) b += (size_t)((c.samples + 1023) / 1024) * 64 * 8 * 2;  // candidate keys
    return b;
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

// Launch one batch of `kind` on slot k from the pending queue (called with the lock held).
static int launch(tgo_server *S, StreamSlot &sl, int kind) {
    const tgo_server_config &c = S->cfg;
    std::deque<Request> &q = S->pending[kind];
    sl.reqs.clear();
    const int cap = kind == 0 ? c.max_batch : c.max_batch_large;
    while (!q.empty() && (int)sl.reqs.size() < cap) {
        Request &r = q.front();
        if (S->in_use + (int64_t)r.bytes > c.budget_bytes && !sl.reqs.empty()) break;
        if (S->in_use + (int64_t)r.bytes > c.budget_bytes && S->in_use > 0) break;  // wait for memory
        r.t_admit = now_ns();
        S->in_use += (int64_t)r.bytes;
        sl.reqs.push_back(r);
        q.pop_front();
    }
    if (sl.reqs.empty()) return 0;
    S->max_in_use = std::max(S->max_in_use, S->in_use);
    // host staging: groups back to back; the exhaustive batch is padded with
    // empty groups to its fixed shape so its captured graph is replayed
    int off = 0;
    sl.h_offs[0] = 0;
    const int ng = kind == 0 ? c.max_batch : (int)sl.reqs.size();
    for (int g = 0; g < ng; ++g) {
        if (g < (int)sl.reqs.size()) {
            const Request &r = sl.reqs[g];
            std::memcpy(sl.h_tasks + off, r.tasks, sizeof(tgo_task) * r.n);
            off += r.n;
            sl.h_keys[g] = r.key;
        } else {
            sl.h_keys[g] = 0;
        }
        sl.h_offs[g + 1] = off;
    }
    sl.kind = kind;
    hipStream_t st = sl.st;
    TGO_HIP(hipMemcpyAsync(sl.d_tasks, sl.h_tasks, sizeof(tgo_task) * std::max(off, 1), hipMemcpyHostToDevice, st));
    TGO_HIP(hipMemcpyAsync(sl.d_offs, sl.h_offs, sizeof(int32_t) * (ng + 1), hipMemcpyHostToDevice, st));
    int rc;
    size_t out_bytes;
    if (kind == 0) {
        rc = tgo_batch(sl.plan, sl.d_tasks, sl.d_offs, ng, (tgo_summary *)sl.d_out, st);
        out_bytes = sizeof(tgo_summary) * sl.reqs.size();
    } else {
        TGO_HIP(hipMemcpyAsync(sl.d_keys, sl.h_keys, sizeof(uint32_t) * ng, hipMemcpyHostToDevice, st));
        rc = tgo_surrogate_search(sl.sur, &S->model, sl.d_tasks, sl.d_offs, sl.d_keys, ng, c.samples, c.topk,
                                  c.seed, (tgo_search_result *)sl.d_out, st);
        out_bytes = sizeof(tgo_search_result) * sl.reqs.size();
    }
    if (rc) return rc;
    TGO_HIP(hipMemcpyAsync(sl.h_out, sl.d_out, out_bytes, hipMemcpyDeviceToHost, st));
    TGO_HIP(hipEventRecord(sl.ev, st));
    sl.busy = true;
    S->batches += 1;
    return 0;
}

static void retire(tgo_server *S, StreamSlot &sl) {
    const int64_t t = now_ns();
    const size_t rb = sl.kind == 0 ? sizeof(tgo_summary) : sizeof(tgo_search_result);
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
        tgo_server_result o;
        fill_result(o, sl.reqs[i], sl.kind, sl.h_out + i * rb, t);
        S->done.push_back(o);
        S->in_use -= (int64_t)sl.reqs[i].bytes;
    }
    S->completed += sl.reqs.size();
    sl.reqs.clear();
    sl.busy = false;
}

// A batch whose completion query reports a device error: its requests are
// returned with status TGO_EDEVICE, their memory released, the slot freed and
// the server stopped (a device error is sticky; nothing more is launched).
static void fail_slot(tgo_server *S, StreamSlot &sl, const std::string &why) {
    const int64_t t = now_ns();
    if (S->error.empty()) S->error = why;
    for (const Request &q : sl.reqs) {
        tgo_server_result o;
        std::memset(&o, 0, sizeof(o));
        o.id = q.id;
        o.n = q.n;
        o.path = sl.kind;
        o.status = TGO_EDEVICE;
        o.t_arrive_ns = q.t_arrive;
        o.t_admit_ns = q.t_admit;
        o.t_done_ns = t;
        o.best_ns = -1;
        o.heur_ns = -1;
        for (int i = 0; i < 16; ++i) o.best[i] = 0xff;
        S->done.push_back(o);
        S->in_use -= (int64_t)q.bytes;
    }
    S->completed += sl.reqs.size();
    sl.reqs.clear();
    sl.busy = false;
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
        for (StreamSlot &sl : S->slots) {
            if (sl.busy) continue;
            // the class whose oldest request has waited longest goes first
            int kind = -1;
            int64_t oldest = INT64_MAX;
            for (int k = 0; k < 2; ++k)
                if (!S->pending[k].empty() && S->pending[k].front().t_arrive < oldest &&
                    (k == 0 || sl.sur)) {
                    oldest = S->pending[k].front().t_arrive;
                    kind = k;
                }
            if (kind < 0) break;
            const int rc = launch(S, sl, kind);
            if (rc) {
                // the admitted requests come back failed; nothing more is launched
                fail_slot(S, sl, std::string("launch failed: ") + tgo_last_error());
                break;
            }
            if (!sl.busy) break;  // nothing admissible right now
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
    c->pad = 0;
    c->samples = 8192;
    c->seed = 4;
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
    for (StreamSlot &sl : S->slots) {
        hipError_t e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(&sl.d_tasks, sizeof(tgo_task) * TGO_MAX_N * gmax);
        if (e == hipSuccess) e = hipMalloc(&sl.d_offs, sizeof(int32_t) * (gmax + 1));
        if (e == hipSuccess) e = hipMalloc(&sl.d_keys, sizeof(uint32_t) * gmax);
        if (e == hipSuccess) e = hipMalloc(&sl.d_out, sizeof(tgo_summary) * gmax);
        if (e == hipSuccess) e = hipHostMalloc(&sl.h_tasks, sizeof(tgo_task) * TGO_MAX_N * gmax);
        if (e == hipSuccess) e = hipHostMalloc(&sl.h_offs, sizeof(int32_t) * (gmax + 1));
        if (e == hipSuccess) e = hipHostMalloc(&sl.h_keys, sizeof(uint32_t) * gmax);
        if (e == hipSuccess) e = hipHostMalloc(&sl.h_out, sizeof(tgo_summary) * gmax);
        if (e != hipSuccess) {
            tgo_server_destroy(S);
            return hip_fail(e, "server slot");
        }
        rc = tgo_plan_create(model, c.max_batch, &sl.plan);
        if (!rc && sur) {
            const int64_t rows = std::max<int64_t>(4096, std::min<int64_t>((int64_t)1 << 16,
                                                   (c.samples + 4095) / 4096 * 4096));
            rc = tgo_surrogate_create(rows, c.max_batch_large, &sl.sur);
            if (!rc) rc = tgo_surrogate_set_params(sl.sur, params.data(), sl.st);
        }
        if (rc) {
            tgo_server_destroy(S);
            return rc;
        }
    }
    S->worker = std::thread(worker_main, S);
    *out = S;
    return TGO_OK;
}

int tgo_server_submit(tgo_server *S, const tgo_task *h_tasks, int n, uint32_t key, uint64_t *id) {
    if (!S || !h_tasks) return fail(TGO_EINVAL, "NULL argument");
    if (n < 1 || n > TGO_MAX_N) return fail(TGO_EINVAL, "n must be in 1..16");
    Request r;
    r.n = n;
    std::memcpy(r.tasks, h_tasks, sizeof(tgo_task) * n);
    r.t_arrive = now_ns();
    r.bytes = request_bytes(S->cfg, n);
    const int kind = n <= S->cfg.small_max_n ? 0 : 1;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop)
            return fail(S->error.empty() ? TGO_EINVAL : TGO_EDEVICE, "server is stopping: " + S->error);
        if (kind == 1 && !S->slots[0].sur) {
            S->rejected += 1;
            return fail(TGO_EINVAL, "no surrogate: groups larger than small_max_n are not served");
        }
        if ((int64_t)r.bytes > S->cfg.budget_bytes) {
            S->rejected += 1;
            return fail(TGO_ENOMEM, "request larger than the whole memory budget");
        }
        r.id = S->next_id++;
        r.key = key ? key : (uint32_t)r.id;
        S->pending[kind].push_back(r);
        S->submitted += 1;
        S->max_queue = std::max(S->max_queue, (int)(S->pending[0].size() + S->pending[1].size()));
    }
    S->cv.notify_all();
    if (id) *id = r.id;
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
    st->queued = (int64_t)(S->pending[0].size() + S->pending[1].size());
    st->max_queued = S->max_queue;
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

void tgo_server_destroy(tgo_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->pending[0].clear();
        S->pending[1].clear();
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (StreamSlot &sl : S->slots) {
        if (sl.st) hipStreamSynchronize(sl.st);
        if (sl.plan) tgo_plan_destroy(sl.plan);
        if (sl.sur) tgo_surrogate_destroy(sl.sur);
        if (sl.d_tasks) hipFree(sl.d_tasks);
        if (sl.d_offs) hipFree(sl.d_offs);
        if (sl.d_keys) hipFree(sl.d_keys);
        if (sl.d_out) hipFree(sl.d_out);
        if (sl.h_tasks) hipHostFree(sl.h_tasks);
        if (sl.h_offs) hipHostFree(sl.h_offs);
        if (sl.h_keys) hipHostFree(sl.h_keys);
        if (sl.h_out) hipHostFree(sl.h_out);
        if (sl.ev) hipEventDestroy(sl.ev);
        if (sl.st) hipStreamDestroy(sl.st);
    }
    delete S;
}

}  // extern "C"
