// Per-ordering evaluation (one lane per given ordering) and the ordering
// heuristic of Section 5.1 (Algorithm 1, one lane per group).
#include <hip/hip_runtime.h>

#include "heur_dev.h"
#include "tables_dev.h"
#include "tgo_internal.h"

namespace tgo {

constexpr int EV_THREADS = 256;
constexpr int HEU_THREADS = 32;

template <typename TT>
__global__ __launch_bounds__(EV_THREADS) void evaluate_kernel(const tgo_task *__restrict__ tasks,
                                                              int n, Rates r,
                                                              const uint8_t *__restrict__ orders,
                                                              int64_t m, int64_t *out) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int MODE = sizeof(TT) == 4 ? 0 : 1;
    __shared__ Quad<TT> Ht[MAXN];
    __shared__ DRec<TT> Dt[MAXN];
    __shared__ int mode;
    if (threadIdx.x == 0) mode = classify_group(tasks, n, r);
    if ((int)threadIdx.x < n) table_entry<TT>(tasks[threadIdx.x], r, &Ht[threadIdx.x], &Dt[threadIdx.x]);
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (mode < 0) {
        if (MODE == 0)
            for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) out[i] = mode;
        return;
    }
    if (mode != MODE) return;
    View<TT, 1, EV_THREADS> v;
    v.H = Ht;
    v.D = Dt;
    v.Q = reinterpret_cast<Slot<TT> *>(smem) + threadIdx.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
        const uint8_t *o = orders + i * n;
        uint32_t seen = 0;
        bool ok = true;
        for (int j = 0; j < n; ++j) {
            const uint32_t x = o[j];
            ok = ok && x < (uint32_t)n && !((seen >> x) & 1u);
            seen |= 1u << (x & 15u);
        }
        if (!ok) {
            out[i] = TGO_EINVAL;
            continue;
        }
        Lane<TT> st = lane_init<TT>();
        for (int j = 0; j < n; ++j) window(st, j, (uint32_t)o[j], v, r);
        out[i] = (int64_t)tail(st, r);
    }
}

int launch_evaluate(const Rates &r, const tgo_task *d_tasks, int n, const uint8_t *d_orders,
                    int64_t m, int64_t *d_out, hipStream_t st) {
    if (m == 0) return TGO_OK;
    int64_t blocks = (m + EV_THREADS - 1) / EV_THREADS;
    if (blocks > 8192) blocks = 8192;
    const size_t shm32 = sizeof(Slot<uint32_t>) * EV_THREADS * n;
    const size_t shm64 = sizeof(Slot<uint64_t>) * EV_THREADS * n;
    hipLaunchKernelGGL(evaluate_kernel<uint32_t>, dim3((unsigned)blocks), dim3(EV_THREADS), shm32, st,
                       d_tasks, n, r, d_orders, m, d_out);
    hipLaunchKernelGGL(evaluate_kernel<uint64_t>, dim3((unsigned)blocks), dim3(EV_THREADS), shm64, st,
                       d_tasks, n, r, d_orders, m, d_out);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

// ---------------------------------------------------------------- heuristic

// One lane per group; the group's tables and the lane's queue live in LDS,
// interleaved by lane.  Always runs the 64-bit time path.
__global__ __launch_bounds__(HEU_THREADS) void heuristic_kernel(const tgo_task *__restrict__ tasks,
                                                                const int32_t *__restrict__ offs,
                                                                int n_groups, Rates r,
                                                                uint8_t *orders, int order_stride,
                                                                int64_t *ns, int ns_stride) {
    using TT = uint64_t;
    __shared__ Quad<TT> Ht[MAXN * HEU_THREADS];
    __shared__ DRec<TT> Dt[MAXN * HEU_THREADS];
    __shared__ Slot<TT> Qs[MAXN * HEU_THREADS];
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_groups) return;
    const int base = offs[g];
    const int n = offs[g + 1] - base;
    uint8_t *orow = orders + (size_t)g * order_stride;
    int64_t *nsg = ns + (size_t)g * ns_stride;
    for (int i = 0; i < 16; ++i) orow[i] = 0xff;
    if (n < 1 || n > MAXN) {
        *nsg = TGO_EINVAL;
        return;
    }
    const tgo_task *t = tasks + base;
    const int cls = classify_group(t, n, r);
    if (cls < 0) {
        *nsg = cls;
        return;
    }
    View<TT, HEU_THREADS, HEU_THREADS> v;
    v.H = Ht + threadIdx.x;
    v.D = Dt + threadIdx.x;
    v.Q = Qs + threadIdx.x;
    for (int x = 0; x < n; ++x)
        table_entry<TT>(t[x], r, &Ht[x * blockDim.x + threadIdx.x], &Dt[x * blockDim.x + threadIdx.x]);

    uint8_t ord[MAXN];
    *nsg = heuristic_order(n, v, r, ord);
    for (int i = 0; i < n; ++i) orow[i] = ord[i];
}

int launch_heuristic(const Rates &r, const tgo_task *d_tasks, const int32_t *d_offs, int n_groups,
                     uint8_t *d_orders, int order_stride, int64_t *d_ns, int ns_stride,
                     hipStream_t st) {
    if (n_groups == 0) return TGO_OK;
    const int blocks = (n_groups + HEU_THREADS - 1) / HEU_THREADS;
    hipLaunchKernelGGL(heuristic_kernel, dim3(blocks), dim3(HEU_THREADS), 0, st, d_tasks, d_offs,
                       n_groups, r, d_orders, order_stride, d_ns, ns_stride);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

}  // namespace tgo
