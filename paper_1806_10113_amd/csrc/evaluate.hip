// Per-ordering evaluation (one lane per given ordering) and the ordering
// heuristic of Section 5.1 (Algorithm 1, one lane per group).
#include <hip/hip_runtime.h>

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

struct Fit3 {
    int64_t th, tk, td;
};

// |h_c - (t_K - t_HtD)| + |k_c - (t_DtH - max(t_HtD + h_c, t_K))|
__device__ __forceinline__ int64_t fit(int64_t h, int64_t k, const Fit3 &u) {
    const int64_t a = h - (u.tk - u.th);
    const int64_t kstart = (u.th + h) > u.tk ? (u.th + h) : u.tk;
    const int64_t b = k - (u.td - kstart);
    return (a < 0 ? -a : a) + (b < 0 ? -b : b);
}

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

    uint32_t rt = (n == 32) ? ~0u : ((1u << n) - 1u);
    // select_first: largest k - h; ties to larger d, then lower index
    int first = -1;
    int64_t bkh = 0, bd = 0;
    for (int x = 0; x < n; ++x) {
        const int64_t kh = t[x].kern_ns - t[x].htd_ns, d = t[x].dth_ns;
        if (first < 0 || kh > bkh || (kh == bkh && d > bd)) { first = x; bkh = kh; bd = d; }
    }
    uint8_t ord[MAXN];
    ord[0] = (uint8_t)first;
    rt &= ~(1u << first);
    Lane<TT> st = lane_init<TT>();
    window(st, 0, (uint32_t)first, v, r);
    int pos = 1;
    while (__popc(rt) > 2) {
        Fit3 u;
        u.th = (int64_t)st.t;
        u.tk = (int64_t)st.ck;
        u.td = (int64_t)tail(st, r);
        int best = -1;
        int64_t bf = 0;
        for (int c = 0; c < n; ++c) {
            if (!((rt >> c) & 1u)) continue;
            const int64_t f = fit(t[c].htd_ns, t[c].kern_ns, u);
            if (best < 0 || f < bf) { best = c; bf = f; }
        }
        ord[pos] = (uint8_t)best;
        rt &= ~(1u << best);
        window(st, pos, (uint32_t)best, v, r);
        ++pos;
    }
    if (__popc(rt) == 2) {
        const int a = __ffs(rt) - 1;
        const int b = 31 - __clz(rt);
        Fit3 u;
        u.th = (int64_t)st.t;
        u.tk = (int64_t)st.ck;
        u.td = (int64_t)tail(st, r);
        int bx = -1, by = -1;
        int64_t bs = 0, bdy = 0;
        for (int o = 0; o < 2; ++o) {
            const int x = o == 0 ? a : b, y = o == 0 ? b : a;
            const int64_t s1 = fit(t[x].htd_ns, t[x].kern_ns, u);
            Lane<TT> s2 = st;
            window(s2, pos, (uint32_t)x, v, r);
            Fit3 w;
            w.th = (int64_t)s2.t;
            w.tk = (int64_t)s2.ck;
            w.td = (int64_t)tail(s2, r);
            const int64_t sc = s1 + fit(t[y].htd_ns, t[y].kern_ns, w) + t[y].dth_ns;
            const int64_t dy = t[y].dth_ns;
            if (bx < 0 || sc < bs || (sc == bs && dy < bdy)) { bx = x; by = y; bs = sc; bdy = dy; }
        }
        ord[pos] = (uint8_t)bx;
        ord[pos + 1] = (uint8_t)by;
        window(st, pos, (uint32_t)bx, v, r);
        window(st, pos + 1, (uint32_t)by, v, r);
        pos += 2;
    } else if (__popc(rt) == 1) {
        const int x = __ffs(rt) - 1;
        ord[pos] = (uint8_t)x;
        window(st, pos, (uint32_t)x, v, r);
        ++pos;
    }
    *nsg = (int64_t)tail(st, r);
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
