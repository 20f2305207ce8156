// C ABI entry points: argument validation, model constants, launches.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "tgo_internal.h"

namespace tgo {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return TGO_EDEVICE;
}

int make_rates(const tgo_model *m, Rates *r) {
    if (!m) return fail(TGO_EINVAL, "model is NULL");
    if (m->dma_engines != 1 && m->dma_engines != 2) return fail(TGO_EINVAL, "dma_engines must be 1 or 2");
    if (m->q_log2 < 0 || m->q_log2 > 10) return fail(TGO_EINVAL, "q_log2 must be in 0..10");
    const int q = 1 << m->q_log2;
    if (m->p_htd < 1 || m->p_htd > q || m->p_dth < 1 || m->p_dth > q)
        return fail(TGO_EINVAL, "overlap rates must satisfy 1 <= p <= q");
    r->q_log2 = m->q_log2;
    r->one_dma = m->dma_engines == 1 ? 1 : 0;
    r->p_h = (uint32_t)m->p_htd;
    r->p_d = (uint32_t)m->p_dth;
    r->inv_ph = 1.0 / (double)m->p_htd;
    r->c_ph = ((double)m->p_htd - 0.5) * r->inv_ph;
    r->inv_pd = 1.0 / (double)m->p_dth;
    r->c_pd = ((double)m->p_dth - 0.5) * r->inv_pd;
    return TGO_OK;
}

// One workspace per (device, stream): calls on different streams never share
// one, and calls on one stream are ordered by the stream itself.
struct StreamWs {
    int dev = 0;
    hipStream_t st = nullptr;
    void *ptr = nullptr;
    size_t bytes = 0;
};
static std::mutex g_ws_mu;
static std::vector<StreamWs> g_ws;

int workspace(size_t bytes, void **ptr, hipStream_t st) {
    int dev = 0;
    TGO_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    StreamWs *w = nullptr;
    for (StreamWs &e : g_ws)
        if (e.dev == dev && e.st == st) { w = &e; break; }
    if (!w) {
        g_ws.emplace_back();
        w = &g_ws.back();
        w->dev = dev;
        w->st = st;
    }
    if (w->bytes < bytes) {
        // Earlier calls on this stream may still use the old buffer.
        if (w->ptr) {
            TGO_HIP(hipStreamSynchronize(st));
            TGO_HIP(hipFree(w->ptr));
            w->ptr = nullptr;
            w->bytes = 0;
        }
        size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) return fail(TGO_ENOMEM, std::string("workspace: ") + hipGetErrorString(e));
        w->ptr = p;
        w->bytes = want;
    }
    *ptr = w->ptr;
    return TGO_OK;
}

}  // namespace tgo

using namespace tgo;

extern "C" {

const char *tgo_strerror(int code) {
    switch (code) {
        case TGO_OK: return "ok";
        case TGO_EINVAL: return "invalid argument";
        case TGO_ERANGE: return "value out of range";
        case TGO_ENOMEM: return "out of memory";
        case TGO_EDEVICE: return "device error";
        default: return "unknown error";
    }
}

const char *tgo_last_error(void) { return g_err.c_str(); }

int tgo_version(void) { return 1; }

int tgo_evaluate(const tgo_model *model, const tgo_task *d_tasks, int n, const uint8_t *d_orders,
                 int64_t m, int64_t *d_out, tgo_stream stream) {
    Rates r;
    int rc = make_rates(model, &r);
    if (rc) return rc;
    if (n < 1 || n > TGO_MAX_N) return fail(TGO_EINVAL, "n must be in 1..16");
    if (m < 0) return fail(TGO_EINVAL, "m must be >= 0");
    if (m > 0 && (!d_tasks || !d_orders || !d_out)) return fail(TGO_EINVAL, "NULL buffer");
    return launch_evaluate(r, d_tasks, n, d_orders, m, d_out, (hipStream_t)stream);
}

int tgo_exhaustive(const tgo_model *model, const tgo_task *d_tasks, int n, int64_t *d_per_order,
                   tgo_summary *d_summary, tgo_stream stream) {
    Rates r;
    int rc = make_rates(model, &r);
    if (rc) return rc;
    if (n < 1 || n > TGO_MAX_EXHAUSTIVE_N) return fail(TGO_EINVAL, "n must be in 1..13");
    if (d_per_order && n > 12) return fail(TGO_EINVAL, "per-ordering output needs n <= 12");
    if (!d_tasks || !d_summary) return fail(TGO_EINVAL, "NULL buffer");
    return launch_exhaustive(r, d_tasks, n, d_per_order, d_summary, (hipStream_t)stream);
}

int tgo_exhaustive_noalloc(const tgo_model *model, const tgo_task *d_tasks, int n, int64_t *d_per_order,
                           tgo_summary *d_summary, tgo_stream stream) {
    Rates r;
    int rc = make_rates(model, &r);
    if (rc) return rc;
    if (n < 1 || n > TGO_MAX_EXHAUSTIVE_N) return fail(TGO_EINVAL, "n must be in 1..13");
    if (d_per_order && n > 12) return fail(TGO_EINVAL, "per-ordering output needs n <= 12");
    if (!d_tasks || !d_summary) return fail(TGO_EINVAL, "NULL buffer");
    return launch_exhaustive_noalloc(r, d_tasks, n, d_per_order, d_summary, (hipStream_t)stream);
}

int tgo_heuristic(const tgo_model *model, const tgo_task *d_tasks, const int32_t *d_offs,
                  int n_groups, uint8_t *d_orders, int64_t *d_ns, tgo_stream stream) {
    Rates r;
    int rc = make_rates(model, &r);
    if (rc) return rc;
    if (n_groups < 0) return fail(TGO_EINVAL, "n_groups must be >= 0");
    if (n_groups > 0 && (!d_tasks || !d_offs || !d_orders || !d_ns)) return fail(TGO_EINVAL, "NULL buffer");
    return launch_heuristic(r, d_tasks, d_offs, n_groups, d_orders, 16, d_ns, 1, (hipStream_t)stream);
}

int tgo_rounds(const tgo_model *model, const tgo_task *d_tasks, int workers, int rounds,
               int64_t *d_per_order, tgo_summary *d_summary, uint16_t *d_groups, tgo_stream stream) {
    Rates r;
    int rc = make_rates(model, &r);
    if (rc) return rc;
    if (workers < 1 || rounds < 1 || workers * rounds > TGO_MAX_N)
        return fail(TGO_EINVAL, "need workers >= 1, rounds >= 1, workers * rounds <= 16");
    uint64_t count = 1;
    for (int i = 0; i < rounds; ++i) {
        count *= factorial(workers);
        if (count > 0xffffffffull) return fail(TGO_EINVAL, "(workers!)^rounds must be below 2^32");
    }
    if (d_per_order && count > TGO_ROUNDS_MAX_PER_ORDER)
        return fail(TGO_EINVAL, "per-ordering output needs (workers!)^rounds <= 479001600");
    if (!d_tasks || !d_summary) return fail(TGO_EINVAL, "NULL buffer");
    return launch_rounds(r, d_tasks, workers, rounds, d_per_order, d_summary, d_groups,
                         (hipStream_t)stream);
}

static int check_memory_args(const tgo_model *model, Rates *r, int n, int max_n, int64_t capacity) {
    int rc = make_rates(model, r);
    if (rc) return rc;
    if (n < 1 || n > max_n) return fail(TGO_EINVAL, "n out of range");
    if (capacity < 1 || capacity > TGO_MAX_CAPACITY) return fail(TGO_EINVAL, "capacity must be in 1..2^62");
    return TGO_OK;
}

int tgo_exhaustive_mem(const tgo_model *model, const tgo_task *d_tasks, const int64_t *d_mem, int n,
                       int64_t capacity, int64_t *d_per_order, tgo_summary *d_summary, tgo_stream stream) {
    Rates r;
    int rc = check_memory_args(model, &r, n, TGO_MAX_MEM_N, capacity);
    if (rc) return rc;
    if (!d_tasks || !d_mem || !d_summary) return fail(TGO_EINVAL, "NULL buffer");
    return launch_memory(r, d_tasks, d_mem, n, capacity, d_per_order, d_summary, (hipStream_t)stream);
}

int tgo_evaluate_mem(const tgo_model *model, const tgo_task *d_tasks, const int64_t *d_mem, int n,
                     int64_t capacity, const uint8_t *d_orders, int64_t m, int64_t *d_out, tgo_stream stream) {
    Rates r;
    int rc = check_memory_args(model, &r, n, TGO_MAX_N, capacity);
    if (rc) return rc;
    if (m < 0 || m > ((int64_t)1 << 40)) return fail(TGO_EINVAL, "m must be in 0..2^40");
    if (m > 0 && (!d_tasks || !d_mem || !d_orders || !d_out)) return fail(TGO_EINVAL, "NULL buffer");
    return launch_memory_evaluate(r, d_tasks, d_mem, n, capacity, d_orders, m, d_out, (hipStream_t)stream);
}

int tgo_predict(const tgo_model *model, const tgo_task *h_tasks, int n, const uint8_t *h_order,
                int64_t *out_ns) {
    Rates r;
    int rc = make_rates(model, &r);
    if (rc) return rc;
    if (n < 1 || n > TGO_MAX_N) return fail(TGO_EINVAL, "n must be in 1..16");
    if (!h_tasks || !h_order || !out_ns) return fail(TGO_EINVAL, "NULL argument");
    // a buffer of its own (no shared workspace): tasks, ordering, result
    const size_t tb = sizeof(tgo_task) * (size_t)n;
    char *d = nullptr;
    TGO_HIP(hipMalloc((void **)&d, tb + 256 + 16 + 8));
    tgo_task *dt = (tgo_task *)d;
    uint8_t *dord = (uint8_t *)(d + tb);
    int64_t *dout = (int64_t *)(d + tb + 256);
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMemcpyAsync(dt, h_tasks, tb, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(dord, h_order, (size_t)n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        rc = launch_evaluate(r, dt, n, dord, 1, dout, st);
        if (rc == TGO_OK) e = hipMemcpyAsync(out_ns, dout, 8, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess && rc == TGO_OK) e = hipStreamSynchronize(st);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(d);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "tgo_predict");
    if (*out_ns < 0) return fail((int)*out_ns, "invalid ordering or tasks out of range");
    return TGO_OK;
}

int tgo_rank(int n, const uint8_t *h_order, uint64_t *rank) {
    if (n < 1 || n > TGO_MAX_N || !h_order || !rank) return fail(TGO_EINVAL, "bad argument");
    uint32_t seen = 0;
    for (int i = 0; i < n; ++i) {
        if (h_order[i] >= n || ((seen >> h_order[i]) & 1u)) return fail(TGO_EINVAL, "not a permutation");
        seen |= 1u << h_order[i];
    }
    uint64_t r = 0;
    for (int i = 0; i < n; ++i) {
        uint64_t c = 0;
        for (int j = i + 1; j < n; ++j) c += h_order[j] < h_order[i];
        r = r * (uint64_t)(n - i) + c;
    }
    *rank = r;
    return TGO_OK;
}

int tgo_unrank(int n, uint64_t rank, uint8_t *h_order) {
    if (n < 1 || n > TGO_MAX_N || !h_order) return fail(TGO_EINVAL, "bad argument");
    if (rank >= factorial(n)) return fail(TGO_ERANGE, "rank >= n!");
    uint8_t rest[16];
    for (int i = 0; i < n; ++i) rest[i] = (uint8_t)i;
    int left = n;
    for (int i = 0; i < n; ++i) {
        const uint64_t f = factorial(n - 1 - i);
        const int c = (int)(rank / f);
        rank %= f;
        h_order[i] = rest[c];
        for (int j = c; j < left - 1; ++j) rest[j] = rest[j + 1];
        --left;
    }
    return TGO_OK;
}

}  // extern "C"
