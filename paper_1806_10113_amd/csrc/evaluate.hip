// Per-ordering evaluation (one lane per given ordering) and the ordering
// heuristic of Section 5.1 (Algorithm 1, one wave per group).
#include <hip/hip_runtime.h>

#include "enum_dev.h"
#include "heur_dev.h"
#include "tables_dev.h"
#include "tgo_internal.h"

namespace tgo {

constexpr int EV_THREADS = 256;
constexpr int HEU_WAVES = 4;  // groups per block of the heuristic, one wave each

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
        out[i] = (int64_t)simulate_order(n, [o](int j) { return (uint32_t)o[j]; }, v, r);
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

// The group's status as classify_group computes it, with one lane per task
// (the per-task terms are combined by wave reductions; same result).
__device__ int classify_group_wave(const tgo_task *t, int n, const Rates &r, int lane) {
    const uint64_t q = 1ull << r.q_log2;
    int bad = 0;
    uint64_t mx = 0, sum = 0;
    if (lane < n) {
        const int64_t h = t[lane].htd_ns, k = t[lane].kern_ns, d = t[lane].dth_ns;
        const int64_t lim = int64_t(1) << 40;
        if (h < 0 || k < 0 || d < 0 || h >= lim || k >= lim || d >= lim) {
            bad = 1;
        } else {
            const uint64_t qh = q * (uint64_t)h, qd = q * (uint64_t)d;
            mx = qh > qd ? qh : qd;
            sum = (qh + r.p_h - 1) / r.p_h + (uint64_t)k + (qd + r.p_d - 1) / r.p_d;
        }
    }
    for (int m = 32; m >= 1; m >>= 1) {
        bad |= __shfl_xor(bad, m);
        const uint64_t mx2 = shfl_xor64(mx, m);
        mx = mx2 > mx ? mx2 : mx;
        sum += shfl_xor64(sum, m);
    }
    if (bad) return TGO_ERANGE;
    const uint64_t lim32 = 1ull << 31;
    return (mx < lim32 && sum + time_bound_slack(n) < lim32) ? 0 : 1;
}

// Wave-wide choice, the same on every lane after the butterfly: the lane
// with the smallest key (a, b, i) in lexicographic order.
__device__ __forceinline__ int wave_pick(int64_t a, int64_t b, int i) {
    for (int m = 32; m >= 1; m >>= 1) {
        const int64_t a2 = (int64_t)shfl_xor64((uint64_t)a, m), b2 = (int64_t)shfl_xor64((uint64_t)b, m);
        const int i2 = __shfl_xor(i, m);
        if (a2 < a || (a2 == a && (b2 < b || (b2 == b && i2 < i)))) { a = a2; b = b2; i = i2; }
    }
    return i;
}

// One wave per group.  The simulation of the ordered set is the same on
// every lane (tables and queue shared by the wave); each selection step
// scores the remaining tasks on their own lanes and picks with the serial
// version's tie rules (select_first: largest K - HtD, then longest DtH, then
// lowest index; select_next: smallest fit, then lowest index).  Always runs
// the 64-bit time path.
__global__ __launch_bounds__(HEU_WAVES * 64) void heuristic_kernel(const tgo_task *__restrict__ tasks,
                                                                   const int32_t *__restrict__ offs,
                                                                   int n_groups, Rates r,
                                                                   uint8_t *orders, int order_stride,
                                                                   int64_t *ns, int ns_stride) {
    using TT = uint64_t;
    __shared__ Quad<TT> Ht[HEU_WAVES][MAXN];
    __shared__ DRec<TT> Dt[HEU_WAVES][MAXN];
    __shared__ Slot<TT> Qs[HEU_WAVES][MAXN];
    __shared__ uint8_t Os[HEU_WAVES][16];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int g = blockIdx.x * HEU_WAVES + w;
    if (g >= n_groups) return;
    const int base = offs[g];
    const int n = offs[g + 1] - base;
    uint8_t *orow = orders + (size_t)g * order_stride;
    int64_t *nsg = ns + (size_t)g * ns_stride;
    if (n < 1 || n > MAXN) {
        if (lane < 16) orow[lane] = 0xff;
        if (lane == 0) *nsg = TGO_EINVAL;
        return;
    }
    const tgo_task *t = tasks + base;
    const int cls = classify_group_wave(t, n, r, lane);
    if (cls < 0) {
        if (lane < 16) orow[lane] = 0xff;
        if (lane == 0) *nsg = cls;
        return;
    }
    if (lane < n) table_entry<TT>(t[lane], r, &Ht[w][lane], &Dt[w][lane]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    View<TT, 1, 1> v;
    v.H = Ht[w];
    v.D = Dt[w];
    v.Q = Qs[w];
    constexpr int64_t BIG = INT64_MAX;
    constexpr int NONE = 1 << 20;

    uint32_t rt = (1u << n) - 1u;
    int first;
    {
        // largest K - HtD, then longest DtH: the smallest (HtD - K, -DtH)
        int64_t a = BIG, b = BIG;
        int id = NONE;
        if (lane < n) {
            const Quad<TT> q = v.task((uint32_t)lane);
            a = (int64_t)q.h - (int64_t)q.k;
            b = -(int64_t)q.d;
            id = lane;
        }
        first = wave_pick(a, b, id);
    }
    if (lane == 0) Os[w][0] = (uint8_t)first;
    rt &= ~(1u << first);
    Lane<TT> st = lane_init<TT>();
    window(st, 0, (uint32_t)first, v, r);
    int pos = 1;
    while (__popc(rt) > 2) {
        const Fit3 u = fit_state<TT, 1, 1>(st, r);
        int64_t f = BIG;
        int id = NONE;
        if (lane < n && ((rt >> lane) & 1u)) {
            const Quad<TT> q = v.task((uint32_t)lane);
            f = fit((int64_t)q.h, (int64_t)q.k, u);
            id = lane;
        }
        const int best = wave_pick(f, 0, id);
        if (lane == 0) Os[w][pos] = (uint8_t)best;
        rt &= ~(1u << best);
        window(st, pos, (uint32_t)best, v, r);
        ++pos;
    }
    if (__popc(rt) == 2) {
        // select_last: both orders of the last two, scored on every lane
        const int a = __ffs(rt) - 1;
        const int b = 31 - __clz(rt);
        const Fit3 u = fit_state<TT, 1, 1>(st, r);
        int bx = -1, by = -1;
        int64_t bs = 0, bdy = 0;
        for (int o = 0; o < 2; ++o) {
            const int x = o == 0 ? a : b, y = o == 0 ? b : a;
            const Quad<TT> tx = v.task((uint32_t)x), ty = v.task((uint32_t)y);
            const int64_t s1 = fit((int64_t)tx.h, (int64_t)tx.k, u);
            Lane<TT> s2 = st;
            window(s2, pos, (uint32_t)x, v, r);
            const Fit3 wf = fit_state<TT, 1, 1>(s2, r);
            const int64_t sc = s1 + fit((int64_t)ty.h, (int64_t)ty.k, wf) + (int64_t)ty.d;
            const int64_t dy = (int64_t)ty.d;
            if (bx < 0 || sc < bs || (sc == bs && dy < bdy)) { bx = x; by = y; bs = sc; bdy = dy; }
        }
        if (lane == 0) {
            Os[w][pos] = (uint8_t)bx;
            Os[w][pos + 1] = (uint8_t)by;
        }
        window(st, pos, (uint32_t)bx, v, r);
        window(st, pos + 1, (uint32_t)by, v, r);
        pos += 2;
    } else if (__popc(rt) == 1) {
        const int x = __ffs(rt) - 1;
        if (lane == 0) Os[w][pos] = (uint8_t)x;
        window(st, pos, (uint32_t)x, v, r);
        ++pos;
    }
    const int64_t T = (int64_t)tail(st, r);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < 16) orow[lane] = lane < n ? Os[w][lane] : (uint8_t)0xff;
    if (lane == 0) *nsg = T;
}

int launch_heuristic(const Rates &r, const tgo_task *d_tasks, const int32_t *d_offs, int n_groups,
                     uint8_t *d_orders, int order_stride, int64_t *d_ns, int ns_stride,
                     hipStream_t st) {
    if (n_groups == 0) return TGO_OK;
    const int blocks = (n_groups + HEU_WAVES - 1) / HEU_WAVES;
    hipLaunchKernelGGL(heuristic_kernel, dim3(blocks), dim3(HEU_WAVES * 64), 0, st, d_tasks, d_offs,
                       n_groups, r, d_orders, order_stride, d_ns, ns_stride);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

}  // namespace tgo
