// Real task execution on the device, for validating the model (Sections 4.2
// and 4.3): each task is an HtD copy from pinned host memory, a kernel and a
// DtH copy back, launched with the schemes of Section 3.2 on HIP streams
// (one stream per command queue, events for the dependencies inside a task),
// and timed with events.  Also the two calibration fits the model needs: the
// linear kernel model T = eta * m + gamma (Eq. 1), the same line for
// transfer time against size, and the overlapped-transfer rates (Section
// 4.2.1) from measured overlapping copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <thread>
#include <vector>

#include "tgo_internal.h"

// Synthetic kernel (the paper's synthetic tasks scale a vector; the
// iteration count sets the duration): iters passes of x = x * s + b over
// n floats.
__global__ __launch_bounds__(256) void tgo_hw_scale_kernel(float *x, int64_t n, int iters, float s, float b) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int it = 0; it < iters; ++it)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
            x[i] = x[i] * s + b;
}

// Register-resident variant: one load and one store per float, 64 dependent
// multiply-adds per pass in between, so the duration is set by the ALUs and
// the kernel hardly touches device memory.
__global__ __launch_bounds__(256) void tgo_hw_fma_kernel(float *x, int64_t n, int iters, float s, float b) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        float v = x[i];
        for (int it = 0; it < iters; ++it)
#pragma unroll
            for (int k = 0; k < 64; ++k) v = v * s + b;
        x[i] = v;
    }
}

// One thread waits until `ticks` of the constant-rate wall clock have passed
// (bounded by max_polls reads of the clock).
__global__ void tgo_hw_delay_kernel(int64_t ticks, int64_t max_polls) {
    if (threadIdx.x != 0) return;
    const int64_t t0 = wall_clock64();
    for (int64_t i = 0; i < max_polls; ++i) {
        if (wall_clock64() - t0 >= ticks) break;
        __builtin_amdgcn_s_sleep(2);
    }
}

namespace {

constexpr int64_t GATE_NS = 2000000;

int launch_task_kernel(float *buf, const tgo_hw_task &t, int max_blocks, hipStream_t st) {
    if (t.kern_iters <= 0 || t.kern_elems <= 0) return TGO_OK;
    const int64_t want = (t.kern_elems + 255) / 256;
    const int blocks = (int)std::min<int64_t>(want, max_blocks);
    if (t.kern_kind == TGO_HW_KERNEL_ALU)
        hipLaunchKernelGGL(tgo_hw_fma_kernel, dim3(blocks), dim3(256), 0, st, buf, t.kern_elems, t.kern_iters,
                           0.999f, 0.001f);
    else
        hipLaunchKernelGGL(tgo_hw_scale_kernel, dim3(blocks), dim3(256), 0, st, buf, t.kern_elems, t.kern_iters,
                           0.999f, 0.001f);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}  // streams held back while the host enqueues

struct TaskBufs {
    void *host_in = nullptr, *host_out = nullptr;
    void *dev_in = nullptr, *dev_out = nullptr;
    float *dev_k = nullptr;
};

}  // namespace

struct tgo_hw {
    int device = 0;
    int max_tasks = 0;
    int64_t max_bytes = 0, max_elems = 0;
    int64_t clock_khz = 0;
    int blocks = 1024;
    hipStream_t sh = nullptr, sk = nullptr, sd = nullptr;
    std::vector<TaskBufs> bufs;
    hipEvent_t t0 = nullptr;
    std::vector<hipEvent_t> ev;  // 6 per task slot: HtD, K, DtH start and end
    // the proxy's Algorithm 1 runs on the device: its own stream and buffers
    hipStream_t sp = nullptr;
    tgo_task *p_tasks = nullptr;
    int32_t *p_offs = nullptr;
    uint8_t *p_order = nullptr;
    int64_t *p_ns = nullptr;
};

namespace tgo {

static void hw_free(tgo_hw *hw) {
    for (auto &b : hw->bufs) {
        if (b.host_in) (void)hipHostFree(b.host_in);
        if (b.host_out) (void)hipHostFree(b.host_out);
        if (b.dev_in) (void)hipFree(b.dev_in);
        if (b.dev_out) (void)hipFree(b.dev_out);
        if (b.dev_k) (void)hipFree(b.dev_k);
    }
    for (auto e : hw->ev) (void)hipEventDestroy(e);
    if (hw->t0) (void)hipEventDestroy(hw->t0);
    if (hw->sh) (void)hipStreamDestroy(hw->sh);
    if (hw->sk) (void)hipStreamDestroy(hw->sk);
    if (hw->sd) (void)hipStreamDestroy(hw->sd);
    if (hw->sp) (void)hipStreamDestroy(hw->sp);
    if (hw->p_tasks) (void)hipFree(hw->p_tasks);
    delete hw;
}

static int64_t ns_between(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1;
    return (int64_t)llround((double)ms * 1e6);
}

static void delay(tgo_hw *hw, hipStream_t st, int64_t ns) {
    const int64_t ticks = ns * hw->clock_khz / 1000000;
    // each poll sleeps ~128 cycles; the bound is far above the wait asked for
    const int64_t polls = 64 + ticks * 64;
    hipLaunchKernelGGL(tgo_hw_delay_kernel, dim3(1), dim3(64), 0, st, ticks, polls);
}

}  // namespace tgo

using namespace tgo;

extern "C" {

int tgo_hw_create(int max_tasks, int64_t max_bytes, int64_t max_kern_elems, tgo_hw **out) {
    if (!out) return fail(TGO_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_tasks < 1 || max_tasks > TGO_MAX_N) return fail(TGO_EINVAL, "max_tasks must be in 1..16");
    if (max_bytes < 0 || max_kern_elems < 0) return fail(TGO_EINVAL, "sizes must be >= 0");
    tgo_hw *hw = new tgo_hw();
    hw->max_tasks = max_tasks;
    hw->max_bytes = max_bytes;
    hw->max_elems = max_kern_elems;
    auto bail = [&](hipError_t e, const char *what) {
        hw_free(hw);
        return hip_fail(e, what);
    };
    hipError_t e = hipGetDevice(&hw->device);
    if (e != hipSuccess) return bail(e, "hipGetDevice");
    int khz = 0;
    e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, hw->device);
    if (e != hipSuccess || khz <= 0) return bail(e == hipSuccess ? hipErrorInvalidValue : e, "wall clock rate");
    hw->clock_khz = khz;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hw->device) == hipSuccess && cus > 0)
        hw->blocks = cus * 4;
    if ((e = hipStreamCreateWithFlags(&hw->sh, hipStreamNonBlocking)) != hipSuccess) return bail(e, "stream");
    if ((e = hipStreamCreateWithFlags(&hw->sk, hipStreamNonBlocking)) != hipSuccess) return bail(e, "stream");
    if ((e = hipStreamCreateWithFlags(&hw->sd, hipStreamNonBlocking)) != hipSuccess) return bail(e, "stream");
    if ((e = hipStreamCreateWithFlags(&hw->sp, hipStreamNonBlocking)) != hipSuccess) return bail(e, "stream");
    if ((e = hipMalloc((void **)&hw->p_tasks, 1024)) != hipSuccess) return bail(e, "hipMalloc");
    hw->p_offs = (int32_t *)((char *)hw->p_tasks + 512);
    hw->p_order = (uint8_t *)((char *)hw->p_tasks + 640);
    hw->p_ns = (int64_t *)((char *)hw->p_tasks + 768);
    if ((e = hipEventCreate(&hw->t0)) != hipSuccess) return bail(e, "event");
    hw->ev.resize(6 * max_tasks, nullptr);
    for (auto &ev : hw->ev)
        if ((e = hipEventCreate(&ev)) != hipSuccess) return bail(e, "event");
    hw->bufs.resize(max_tasks);
    const size_t nb = (size_t)std::max<int64_t>(max_bytes, 4);
    const size_t kb = sizeof(float) * (size_t)std::max<int64_t>(max_kern_elems, 1);
    for (auto &b : hw->bufs) {
        if ((e = hipHostMalloc(&b.host_in, nb, hipHostMallocDefault)) != hipSuccess) return bail(e, "hipHostMalloc");
        if ((e = hipHostMalloc(&b.host_out, nb, hipHostMallocDefault)) != hipSuccess) return bail(e, "hipHostMalloc");
        if ((e = hipMalloc(&b.dev_in, nb)) != hipSuccess) return bail(e, "hipMalloc");
        if ((e = hipMalloc(&b.dev_out, nb)) != hipSuccess) return bail(e, "hipMalloc");
        if ((e = hipMalloc((void **)&b.dev_k, kb)) != hipSuccess) return bail(e, "hipMalloc");
        std::fill((unsigned char *)b.host_in, (unsigned char *)b.host_in + nb, (unsigned char)1);
        if ((e = hipMemset(b.dev_out, 0, nb)) != hipSuccess) return bail(e, "hipMemset");
        if ((e = hipMemset(b.dev_k, 0, kb)) != hipSuccess) return bail(e, "hipMemset");
    }
    if ((e = hipDeviceSynchronize()) != hipSuccess) return bail(e, "hipDeviceSynchronize");
    *out = hw;
    return TGO_OK;
}

void tgo_hw_destroy(tgo_hw *hw) {
    if (!hw) return;
    (void)hipSetDevice(hw->device);
    (void)hipDeviceSynchronize();
    hw_free(hw);
}

}  // extern "C"

namespace tgo {

// Run n tasks in launch order seq.  Groups of g consecutive positions form
// the units of the one-DMA transfer queue (every HtD of a group, then its
// DtHs).  With R > 1 task x is worker x / R's task x % R and its HtD waits
// for the DtH of task x - 1 (an event wait on the in-order HtD queue).
// seq: task per launch position.  gend (one DMA engine): bit j set if
// position j ends a launch group.  R > 1: task x waits for the DtH of task
// x - 1 unless x % R == 0 (multi-round workers).  gate (may be NULL): the
// HtD at position j waits for the DtH at position gate[j] (< 0: none).
static int hw_run_impl(tgo_hw *hw, const tgo_hw_task *h_tasks, int n, const uint8_t *seq, uint32_t gend, int R,
                       const int *gate, int dma_engines, int64_t *h_total_ns, tgo_hw_times *h_cmds) {
    uint32_t seen = 0;
    for (int i = 0; i < n; ++i) {
        if (seq[i] >= n || ((seen >> seq[i]) & 1u)) return fail(TGO_EINVAL, "not a permutation");
        seen |= 1u << seq[i];
        const tgo_hw_task &t = h_tasks[i];
        if (t.htd_bytes < 0 || t.htd_bytes > hw->max_bytes || t.dth_bytes < 0 || t.dth_bytes > hw->max_bytes ||
            t.kern_elems < 0 || t.kern_elems > hw->max_elems || t.kern_iters < 0 ||
            (t.kern_kind != TGO_HW_KERNEL_HBM && t.kern_kind != TGO_HW_KERNEL_ALU))
            return fail(TGO_EINVAL, "task exceeds the runner's buffers");
    }
    TGO_HIP(hipSetDevice(hw->device));
    hipStream_t sx = hw->sh;                            // transfer queue(s)
    hipStream_t sd = dma_engines == 2 ? hw->sd : hw->sh;
    // hold every stream until the host has enqueued the whole group
    delay(hw, hw->sh, GATE_NS);
    TGO_HIP(hipEventRecord(hw->t0, hw->sh));
    TGO_HIP(hipStreamWaitEvent(hw->sk, hw->t0, 0));
    if (sd != sx) TGO_HIP(hipStreamWaitEvent(sd, hw->t0, 0));
    auto E = [&](int x, int c) { return hw->ev[6 * x + c]; };
    auto htd = [&](int i) -> int {
        const int x = seq[i];
        const tgo_hw_task &t = h_tasks[x];
        if (R > 1 && x % R) TGO_HIP(hipStreamWaitEvent(sx, E(x - 1, 5), 0));  // the worker's previous task
        if (gate && gate[i] >= 0) TGO_HIP(hipStreamWaitEvent(sx, E(seq[gate[i]], 5), 0));  // memory given back
        TGO_HIP(hipEventRecord(E(x, 0), sx));
        if (t.htd_bytes > 0)
            TGO_HIP(hipMemcpyAsync(hw->bufs[x].dev_in, hw->bufs[x].host_in, (size_t)t.htd_bytes,
                                   hipMemcpyHostToDevice, sx));
        TGO_HIP(hipEventRecord(E(x, 1), sx));
        return TGO_OK;
    };
    auto kern = [&](int x) -> int {
        const tgo_hw_task &t = h_tasks[x];
        TGO_HIP(hipStreamWaitEvent(hw->sk, E(x, 1), 0));
        TGO_HIP(hipEventRecord(E(x, 2), hw->sk));
        if (int rc = launch_task_kernel(hw->bufs[x].dev_k, t, hw->blocks, hw->sk)) return rc;
        TGO_HIP(hipEventRecord(E(x, 3), hw->sk));
        return TGO_OK;
    };
    auto dth = [&](int x) -> int {
        const tgo_hw_task &t = h_tasks[x];
        TGO_HIP(hipStreamWaitEvent(sd, E(x, 3), 0));
        TGO_HIP(hipEventRecord(E(x, 4), sd));
        if (t.dth_bytes > 0)
            TGO_HIP(hipMemcpyAsync(hw->bufs[x].host_out, hw->bufs[x].dev_out, (size_t)t.dth_bytes,
                                   hipMemcpyDeviceToHost, sd));
        TGO_HIP(hipEventRecord(E(x, 5), sd));
        return TGO_OK;
    };
    int rc;
    if (dma_engines == 2) {
        // three queues, commands in launch order (Section 3.2, two DMA engines)
        for (int i = 0; i < n; ++i) {
            const int x = seq[i];
            if ((rc = htd(i)) || (rc = kern(x)) || (rc = dth(x))) return rc;
        }
    } else {
        // one transfer queue: per group every HtD, then every DtH; kernels on their own queue
        for (int b = 0; b < n;) {
            int e = b + 1;
            while (e < n && !((gend >> (e - 1)) & 1u)) ++e;
            for (int i = b; i < e; ++i)
                if ((rc = htd(i)) || (rc = kern(seq[i]))) return rc;
            for (int i = b; i < e; ++i)
                if ((rc = dth(seq[i]))) return rc;
            b = e;
        }
    }
    TGO_HIP(hipStreamSynchronize(hw->sh));
    TGO_HIP(hipStreamSynchronize(hw->sk));
    TGO_HIP(hipStreamSynchronize(hw->sd));
    int64_t total = 0;
    for (int x = 0; x < n; ++x) {
        tgo_hw_times c;
        for (int k = 0; k < 3; ++k) {
            c.start_ns[k] = ns_between(hw->t0, E(x, 2 * k));
            c.end_ns[k] = ns_between(hw->t0, E(x, 2 * k + 1));
            total = std::max(total, c.end_ns[k]);
        }
        if (h_cmds) h_cmds[x] = c;
    }
    *h_total_ns = total;
    return TGO_OK;
}

// Heuristic setup (Section 6.2) on the device: a host proxy loop.  Task
// (w, r) is offered when the DtH of (w, r - 1) has ended (seen by polling its
// event); the proxy takes every offered task as a group, orders it with
// Algorithm 1 (run on the device from the tasks' solo durations h_dur) and
// enqueues it; it looks again once the HtD of the group's last task has
// started (its start event has been reached), or at the next arrival.
static int hw_proxy_impl(tgo_hw *hw, const Rates &r, const tgo_hw_task *h_tasks, const tgo_task *h_dur, int T,
                         int R, int dma_engines, int64_t *h_total_ns, uint8_t *h_seq, uint16_t *h_groups,
                         tgo_hw_times *h_cmds) {
    const int n = T * R;
    for (int i = 0; i < n; ++i) {
        const tgo_hw_task &t = h_tasks[i];
        if (t.htd_bytes < 0 || t.htd_bytes > hw->max_bytes || t.dth_bytes < 0 || t.dth_bytes > hw->max_bytes ||
            t.kern_elems < 0 || t.kern_elems > hw->max_elems || t.kern_iters < 0 ||
            (t.kern_kind != TGO_HW_KERNEL_HBM && t.kern_kind != TGO_HW_KERNEL_ALU))
            return fail(TGO_EINVAL, "task exceeds the runner's buffers");
    }
    TGO_HIP(hipSetDevice(hw->device));
    hipStream_t sx = hw->sh;
    hipStream_t sd = dma_engines == 2 ? hw->sd : hw->sh;
    auto E = [&](int x, int c) { return hw->ev[6 * x + c]; };
    auto enqueue = [&](const uint8_t *ord, int g) -> int {
        auto htd = [&](int x) -> int {
            const tgo_hw_task &t = h_tasks[x];
            TGO_HIP(hipEventRecord(E(x, 0), sx));
            if (t.htd_bytes > 0)
                TGO_HIP(hipMemcpyAsync(hw->bufs[x].dev_in, hw->bufs[x].host_in, (size_t)t.htd_bytes,
                                       hipMemcpyHostToDevice, sx));
            TGO_HIP(hipEventRecord(E(x, 1), sx));
            const tgo_hw_task &tk = h_tasks[x];
            TGO_HIP(hipStreamWaitEvent(hw->sk, E(x, 1), 0));
            TGO_HIP(hipEventRecord(E(x, 2), hw->sk));
            if (int rc = launch_task_kernel(hw->bufs[x].dev_k, tk, hw->blocks, hw->sk)) return rc;
            TGO_HIP(hipEventRecord(E(x, 3), hw->sk));
            return TGO_OK;
        };
        auto dth = [&](int x) -> int {
            const tgo_hw_task &t = h_tasks[x];
            TGO_HIP(hipStreamWaitEvent(sd, E(x, 3), 0));
            TGO_HIP(hipEventRecord(E(x, 4), sd));
            if (t.dth_bytes > 0)
                TGO_HIP(hipMemcpyAsync(hw->bufs[x].host_out, hw->bufs[x].dev_out, (size_t)t.dth_bytes,
                                       hipMemcpyDeviceToHost, sd));
            TGO_HIP(hipEventRecord(E(x, 5), sd));
            return TGO_OK;
        };
        int rc;
        if (dma_engines == 2) {
            for (int i = 0; i < g; ++i)
                if ((rc = htd(ord[i])) || (rc = dth(ord[i]))) return rc;
        } else {
            for (int i = 0; i < g; ++i)
                if ((rc = htd(ord[i]))) return rc;
            for (int i = 0; i < g; ++i)
                if ((rc = dth(ord[i]))) return rc;
        }
        return TGO_OK;
    };
    // Algorithm 1 on a group, on the device (synchronous)
    auto order_group = [&](const uint8_t *mem, int g, uint8_t *out) -> int {
        tgo_task tk[TGO_MAX_N];
        for (int i = 0; i < g; ++i) tk[i] = h_dur[mem[i]];
        const int32_t offs[2] = {0, g};
        TGO_HIP(hipMemcpyAsync(hw->p_tasks, tk, sizeof(tgo_task) * g, hipMemcpyHostToDevice, hw->sp));
        TGO_HIP(hipMemcpyAsync(hw->p_offs, offs, sizeof(offs), hipMemcpyHostToDevice, hw->sp));
        int rc = launch_heuristic(r, hw->p_tasks, hw->p_offs, 1, hw->p_order, 16, hw->p_ns, 1, hw->sp);
        if (rc) return rc;
        uint8_t ord[16];
        TGO_HIP(hipMemcpyAsync(ord, hw->p_order, 16, hipMemcpyDeviceToHost, hw->sp));
        TGO_HIP(hipStreamSynchronize(hw->sp));
        for (int i = 0; i < g; ++i) {
            if (ord[i] >= g) return fail(TGO_ERANGE, "heuristic failed on a group");
            out[i] = mem[ord[i]];
        }
        return TGO_OK;
    };
    delay(hw, hw->sh, GATE_NS);
    TGO_HIP(hipEventRecord(hw->t0, hw->sh));
    TGO_HIP(hipStreamWaitEvent(hw->sk, hw->t0, 0));
    if (sd != sx) TGO_HIP(hipStreamWaitEvent(sd, hw->t0, 0));
    uint32_t buffer = 0, submitted = 0, done = 0;
    for (int w = 0; w < T; ++w) buffer |= 1u << (w * R);
    bool armed = true;
    int trig = -1, nsub = 0;
    uint16_t gend = 0;
    uint8_t seq[TGO_MAX_N];
    const uint32_t all = (n == 32) ? ~0u : ((1u << n) - 1u);
    int rc = TGO_OK;
    // every task is submitted once and completes, so the loop ends; a
    // device error ends it at once, and so does a wall-clock limit
    const auto start = std::chrono::steady_clock::now();
    while (done != all) {
        if (std::chrono::steady_clock::now() - start > std::chrono::seconds(120))
            return fail(TGO_ERANGE, "proxy: tasks did not complete within 120 s");
        bool progress = false;
        for (int x = 0; x < n; ++x) {
            if (!((submitted >> x) & 1u) || ((done >> x) & 1u)) continue;
            const hipError_t q = hipEventQuery(E(x, 5));
            if (q == hipSuccess) {
                done |= 1u << x;
                if (x % R + 1 < R) buffer |= 1u << (x + 1);
                progress = true;
            } else if (q != hipErrorNotReady) {
                return hip_fail(q, "hipEventQuery");
            }
        }
        if (!armed && trig >= 0) {
            const hipError_t q = hipEventQuery(E(trig, 0));
            if (q == hipSuccess) armed = true;
            else if (q != hipErrorNotReady) return hip_fail(q, "hipEventQuery");
        }
        if (armed && buffer) {
            uint8_t mem[TGO_MAX_N], ord[TGO_MAX_N];
            int g = 0;
            for (int x = 0; x < n; ++x)
                if ((buffer >> x) & 1u) mem[g++] = (uint8_t)x;
            if ((rc = order_group(mem, g, ord))) return rc;
            if ((rc = enqueue(ord, g))) return rc;
            for (int i = 0; i < g; ++i) {
                seq[nsub + i] = ord[i];
                submitted |= 1u << ord[i];
            }
            nsub += g;
            gend |= (uint16_t)(1u << (nsub - 1));
            trig = ord[g - 1];
            buffer = 0;
            armed = false;
            progress = true;
        }
        if (!progress) std::this_thread::yield();
    }
    TGO_HIP(hipStreamSynchronize(hw->sh));
    TGO_HIP(hipStreamSynchronize(hw->sk));
    TGO_HIP(hipStreamSynchronize(hw->sd));
    int64_t total = 0;
    for (int x = 0; x < n; ++x) {
        tgo_hw_times c;
        for (int k = 0; k < 3; ++k) {
            c.start_ns[k] = ns_between(hw->t0, E(x, 2 * k));
            c.end_ns[k] = ns_between(hw->t0, E(x, 2 * k + 1));
            total = std::max(total, c.end_ns[k]);
        }
        if (h_cmds) h_cmds[x] = c;
    }
    *h_total_ns = total;
    if (h_seq)
        for (int i = 0; i < TGO_MAX_N; ++i) h_seq[i] = i < n ? seq[i] : (uint8_t)0xff;
    if (h_groups) *h_groups = gend;
    return TGO_OK;
}

}  // namespace tgo

extern "C" {

int tgo_hw_run_proxy(tgo_hw *hw, const tgo_model *model, const tgo_hw_task *h_tasks, const tgo_task *h_dur,
                     int workers, int rounds, int64_t *h_total_ns, uint8_t *h_seq, uint16_t *h_groups,
                     tgo_hw_times *h_cmds) {
    Rates r;
    int rc = make_rates(model, &r);
    if (rc) return rc;
    if (!hw || !h_tasks || !h_dur || !h_total_ns) return fail(TGO_EINVAL, "NULL argument");
    if (workers < 1 || rounds < 1 || workers * rounds > hw->max_tasks)
        return fail(TGO_EINVAL, "need 1 <= workers * rounds <= max_tasks");
    return hw_proxy_impl(hw, r, h_tasks, h_dur, workers, rounds, model->dma_engines, h_total_ns, h_seq, h_groups,
                         h_cmds);
}

int tgo_hw_run(tgo_hw *hw, const tgo_hw_task *h_tasks, int n, const uint8_t *h_order, int dma_engines,
               int64_t *h_total_ns, tgo_hw_times *h_cmds) {
    if (!hw || !h_tasks || !h_order || !h_total_ns) return fail(TGO_EINVAL, "NULL argument");
    if (n < 1 || n > hw->max_tasks) return fail(TGO_EINVAL, "n must be in 1..max_tasks");
    if (dma_engines != 1 && dma_engines != 2) return fail(TGO_EINVAL, "dma_engines must be 1 or 2");
    return hw_run_impl(hw, h_tasks, n, h_order, 1u << (n - 1), 1, nullptr, dma_engines, h_total_ns, h_cmds);
}

int tgo_hw_run_rounds(tgo_hw *hw, const tgo_hw_task *h_tasks, int workers, int rounds, const uint8_t *h_seq,
                      int dma_engines, int64_t *h_total_ns, tgo_hw_times *h_cmds) {
    if (!hw || !h_tasks || !h_seq || !h_total_ns) return fail(TGO_EINVAL, "NULL argument");
    if (workers < 1 || rounds < 1 || workers * rounds > hw->max_tasks)
        return fail(TGO_EINVAL, "need 1 <= workers * rounds <= max_tasks");
    if (dma_engines != 1 && dma_engines != 2) return fail(TGO_EINVAL, "dma_engines must be 1 or 2");
    const int n = workers * rounds;
    // round r of the sequence must hold exactly the tasks (w, r)
    for (int i = 0; i < n; ++i)
        if (h_seq[i] >= n || h_seq[i] % rounds != i / workers)
            return fail(TGO_EINVAL, "h_seq must list round r's tasks at positions r*workers ..");
    uint32_t gend = 0;
    for (int r = 0; r < rounds; ++r) gend |= 1u << ((r + 1) * workers - 1);
    return hw_run_impl(hw, h_tasks, n, h_seq, gend, rounds, nullptr, dma_engines, h_total_ns, h_cmds);
}

int tgo_hw_run_mem(tgo_hw *hw, const tgo_hw_task *h_tasks, int n, const uint8_t *h_order, const int64_t *h_mem,
                   int64_t capacity, int dma_engines, int64_t *h_total_ns, tgo_hw_times *h_cmds) {
    if (!hw || !h_tasks || !h_order || !h_mem || !h_total_ns) return fail(TGO_EINVAL, "NULL argument");
    if (n < 1 || n > hw->max_tasks) return fail(TGO_EINVAL, "n must be in 1..max_tasks");
    if (dma_engines != 1 && dma_engines != 2) return fail(TGO_EINVAL, "dma_engines must be 1 or 2");
    if (capacity < 1 || capacity > TGO_MAX_CAPACITY) return fail(TGO_EINVAL, "capacity must be in 1..2^62");
    for (int i = 0; i < n; ++i) {
        if (h_order[i] >= n) return fail(TGO_EINVAL, "not a permutation");
        if (h_mem[i] < 0 || h_mem[i] > capacity) return fail(TGO_EINVAL, "every footprint must fit the capacity");
    }
    int gate[TGO_MAX_N];
    uint32_t gend = 0;
    if (dma_engines == 2) {
        // the HtD at position j starts once every position before a_j has
        // ended its DtH, a_j the first position from which the footprints
        // through j fit
        for (int j = 0; j < n; ++j) {
            int64_t held = h_mem[h_order[j]];
            int a = j;
            while (a > 0 && held + h_mem[h_order[a - 1]] <= capacity) held += h_mem[h_order[--a]];
            gate[j] = a - 1;
        }
    } else {
        // greedy sub-groups whose footprints fit together
        int64_t held = 0;
        for (int j = 0; j < n; ++j) {
            if (j > 0 && held + h_mem[h_order[j]] > capacity) {
                gend |= 1u << (j - 1);
                held = 0;
            }
            held += h_mem[h_order[j]];
        }
        gend |= 1u << (n - 1);
    }
    return hw_run_impl(hw, h_tasks, n, h_order, gend, 1, dma_engines == 2 ? gate : nullptr, dma_engines,
                       h_total_ns, h_cmds);
}

int tgo_hw_overlap(tgo_hw *hw, int64_t htd_bytes, int64_t dth_bytes, int64_t dth_delay_ns, int64_t *h_times) {
    if (!hw || !h_times) return fail(TGO_EINVAL, "NULL argument");
    if (htd_bytes < 0 || htd_bytes > hw->max_bytes || dth_bytes < 0 || dth_bytes > hw->max_bytes ||
        dth_delay_ns < 0 || dth_delay_ns > 10000000000ll)
        return fail(TGO_EINVAL, "sizes out of range");
    TGO_HIP(hipSetDevice(hw->device));
    delay(hw, hw->sh, GATE_NS);
    TGO_HIP(hipEventRecord(hw->t0, hw->sh));
    TGO_HIP(hipStreamWaitEvent(hw->sd, hw->t0, 0));
    TGO_HIP(hipEventRecord(hw->ev[0], hw->sh));
    if (htd_bytes > 0)
        TGO_HIP(hipMemcpyAsync(hw->bufs[0].dev_in, hw->bufs[0].host_in, (size_t)htd_bytes,
                               hipMemcpyHostToDevice, hw->sh));
    TGO_HIP(hipEventRecord(hw->ev[1], hw->sh));
    if (dth_delay_ns > 0) delay(hw, hw->sd, dth_delay_ns);
    TGO_HIP(hipEventRecord(hw->ev[4], hw->sd));
    if (dth_bytes > 0)
        TGO_HIP(hipMemcpyAsync(hw->bufs[0].host_out, hw->bufs[0].dev_out, (size_t)dth_bytes,
                               hipMemcpyDeviceToHost, hw->sd));
    TGO_HIP(hipEventRecord(hw->ev[5], hw->sd));
    TGO_HIP(hipStreamSynchronize(hw->sh));
    TGO_HIP(hipStreamSynchronize(hw->sd));
    h_times[0] = ns_between(hw->t0, hw->ev[0]);
    h_times[1] = ns_between(hw->t0, hw->ev[1]);
    h_times[2] = ns_between(hw->t0, hw->ev[4]);
    h_times[3] = ns_between(hw->t0, hw->ev[5]);
    return TGO_OK;
}

int tgo_fit_line(const double *h_x, const double *h_y, int n, double *slope, double *intercept) {
    if (!h_x || !h_y || !slope || !intercept || n < 2) return fail(TGO_EINVAL, "need n >= 2 points");
    double mx = 0, my = 0;
    for (int i = 0; i < n; ++i) { mx += h_x[i]; my += h_y[i]; }
    mx /= n;
    my /= n;
    double sxx = 0, sxy = 0;
    for (int i = 0; i < n; ++i) {
        sxx += (h_x[i] - mx) * (h_x[i] - mx);
        sxy += (h_x[i] - mx) * (h_y[i] - my);
    }
    if (!(sxx > 0)) return fail(TGO_EINVAL, "x values are all equal");
    *slope = sxy / sxx;
    *intercept = my - *slope * mx;
    return TGO_OK;
}

int tgo_fit_overlap(const int64_t *h_times, const int64_t *h_solo, int n, double *rho_htd, double *rho_dth) {
    if (!h_times || !h_solo || !rho_htd || !rho_dth || n < 1) return fail(TGO_EINVAL, "bad argument");
    double wh = 0, sh = 0, wd = 0, sd = 0;
    for (int i = 0; i < n; ++i) {
        const int64_t *t = h_times + 4 * i;
        const double h0 = (double)t[0], h1 = (double)t[1], d0 = (double)t[2], d1 = (double)t[3];
        const double L = std::min(h1, d1) - std::max(h0, d0);
        if (L <= 0) continue;
        // solo work = time outside the overlap at full speed + rho * overlap
        sh += (double)h_solo[2 * i] - ((h1 - h0) - L);
        sd += (double)h_solo[2 * i + 1] - ((d1 - d0) - L);
        wh += L;
        wd += L;
    }
    if (!(wh > 0)) return fail(TGO_EINVAL, "no experiment overlaps");
    *rho_htd = sh / wh;
    *rho_dth = sd / wd;
    return TGO_OK;
}

}  // extern "C"
