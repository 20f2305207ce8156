// Task groups whose kernels may run concurrently (CKE).
//
// The paper's model keeps one kernel queue (Section 4.1, last paragraph): a
// kernel that exhausts the device overlaps the next one only at its tail, and
// devices do not disclose how they run concurrent kernels.  Its NoReorder
// experiments do use one command queue per kernel (Section 6.2), Section 3.2
// states when kernels from different queues can overlap (while the device's
// resources are not exhausted), and the conclusion leaves concurrent kernels
// to future work.  Reading used here:
//   * the device has `capacity` units of computing resources; kernel x holds
//     units[x] of them (1 .. capacity) from its start to its end;
//   * kernels are dispatched in launch order: K at position j starts once its
//     HtD has ended, the kernel at position j - 1 has started, and its units
//     fit beside those of the running kernels; it takes its solo time;
//   * transfers follow the launch schemes of Section 3.2 as everywhere else
//     (two DMA engines: HtD and DtH FIFO queues; one engine: every HtD, then
//     every DtH, on one queue), with the Section 4.2.1 overlap rates.
// With every kernel holding the whole capacity this is the one-queue model.
//
// Kernel ends no longer follow one chain, so the window formulation of the
// other paths does not apply; each lane steps the events of one ordering
// (64-bit time): at each instant every finished command retires, then every
// ready head starts and the kernel dispatcher takes what fits, until nothing
// changes; time then advances to the earliest completion.
#include <hip/hip_runtime.h>

#include "enum_dev.h"
#include "heur_dev.h"
#include "tables_dev.h"
#include "tgo_internal.h"

namespace tgo {

constexpr int CK_THREADS = 256;
constexpr uint32_t CK_MAX_BLOCKS = 8192;
constexpr int32_t CK_MAX_CAPACITY = 1 << 30;

struct CTab {
    int64_t h[MAXN], k[MAXN], d[MAXN];
    int32_t u[MAXN];
};

__device__ __forceinline__ uint32_t ck_nib(uint64_t v, int i) { return (uint32_t)(v >> (4 * i)) & 15u; }

// Block-wide load of the task table; 0, TGO_ERANGE (a duration outside
// [0, 2^40)) or TGO_EINVAL (a unit count outside 1..cap).
__device__ int ctab_load(const tgo_task *__restrict__ tasks, const int32_t *__restrict__ units, int n, int cap,
                         CTab &tb, int *flag) {
    if (threadIdx.x == 0) *flag = 0;
    __syncthreads();
    if ((int)threadIdx.x < n) {
        const tgo_task t = tasks[threadIdx.x];
        const int32_t u = units[threadIdx.x];
        if (t.htd_ns < 0 || t.kern_ns < 0 || t.dth_ns < 0 || t.htd_ns >= MAX_DURATION ||
            t.kern_ns >= MAX_DURATION || t.dth_ns >= MAX_DURATION)
            atomicOr(flag, 1);
        if (u < 1 || u > cap) atomicOr(flag, 2);
        tb.h[threadIdx.x] = t.htd_ns;
        tb.k[threadIdx.x] = t.kern_ns;
        tb.d[threadIdx.x] = t.dth_ns;
        tb.u[threadIdx.x] = u;
    }
    __syncthreads();
    const int f = *flag;
    return (f & 1) ? TGO_ERANGE : (f & 2) ? TGO_EINVAL : 0;
}

struct CkeOut {
    int64_t T;           // end of the last command
    int64_t th, tk, td;  // ends of the last position's HtD, K and DtH
};

// One ordering (seq: task at position j in nibble j, n positions).  kend:
// this lane's kernel end times by position (stride kst).
template <bool ONE>
__device__ CkeOut cke_sim(uint64_t seq, int n, const CTab &tb, int cap, const Rates &r, int64_t *kend, int kst) {
    const int64_t q = int64_t(1) << r.q_log2;
    int64_t t = 0;
    int hc = 0, dc = 0, xo = 0;  // next queue entry: HtD, DtH (two engines); transfer queue (one)
    bool hrun = false, drun = false;
    int hpos = 0, dpos = 0, hdone = 0;
    int64_t uh = 0, ud = 0;
    int kc = 0, held = 0;
    uint32_t krun = 0, kdone = 0;
    CkeOut o = {0, 0, 0, 0};
    for (;;) {
        bool changed = true;
        while (changed) {
            changed = false;
            if (hrun && uh == 0) {
                hrun = false;
                ++hdone;
                if (hpos == n - 1) o.th = t;
                changed = true;
            }
            if (drun && ud == 0) {
                drun = false;
                if (dpos == n - 1) o.td = t;
                changed = true;
            }
            for (uint32_t m = krun; m; m &= m - 1) {
                const int p = __ffs(m) - 1;
                if (kend[p * kst] == t) {
                    krun &= ~(1u << p);
                    kdone |= 1u << p;
                    held -= tb.u[ck_nib(seq, p)];
                    if (p == n - 1) o.tk = t;
                    changed = true;
                }
            }
            if constexpr (!ONE) {
                if (!hrun && hc < n) {
                    hpos = hc++;
                    uh = q * tb.h[ck_nib(seq, hpos)];
                    hrun = true;
                    changed = true;
                }
                if (!drun && dc < n && ((kdone >> dc) & 1u)) {
                    dpos = dc++;
                    ud = q * tb.d[ck_nib(seq, dpos)];
                    drun = true;
                    changed = true;
                }
            } else {
                if (!hrun && !drun) {
                    if (xo < n) {
                        hpos = xo++;
                        uh = q * tb.h[ck_nib(seq, hpos)];
                        hrun = true;
                        changed = true;
                    } else if (xo < 2 * n && ((kdone >> (xo - n)) & 1u)) {
                        dpos = xo - n;
                        ++xo;
                        ud = q * tb.d[ck_nib(seq, dpos)];
                        drun = true;
                        changed = true;
                    }
                }
            }
            // in-order dispatch of the kernels whose HtD has ended and that fit
            while (kc < n && kc < hdone && held + tb.u[ck_nib(seq, kc)] <= cap) {
                const uint32_t x = ck_nib(seq, kc);
                kend[kc * kst] = t + tb.k[x];
                krun |= 1u << kc;
                held += tb.u[x];
                ++kc;
                changed = true;
            }
        }
        if (!hrun && !drun && !krun) break;
        const bool both = !ONE && hrun && drun;
        const int64_t rh = both ? (int64_t)r.p_h : q, rd = both ? (int64_t)r.p_d : q;
        const int64_t INF = INT64_MAX;
        const int64_t eh = hrun ? (uh + rh - 1) / rh : INF;
        const int64_t ed = drun ? (ud + rd - 1) / rd : INF;
        int64_t dt = eh < ed ? eh : ed;
        for (uint32_t m = krun; m; m &= m - 1) {
            const int p = __ffs(m) - 1;
            const int64_t e = kend[p * kst] - t;
            dt = e < dt ? e : dt;
        }
        if (hrun) uh = eh == dt ? 0 : uh - rh * dt;
        if (drun) ud = ed == dt ? 0 : ud - rd * dt;
        t += dt;
    }
    o.T = t;
    return o;
}

// rank (lexicographic) -> task at each position, one per nibble
__device__ __forceinline__ uint64_t ck_unrank(int n, uint64_t rk) {
    uint64_t list = 0;
    for (int i = n - 1; i >= 0; --i) list = (list << 4) | (uint64_t)i;
    uint64_t f = fact_c(n - 1), seq = 0;
    for (int i = 0; i < n; ++i) {
        const uint64_t c = f ? rk / f : 0;
        rk -= c * f;
        if (n - 1 - i > 0) f /= (uint64_t)(n - 1 - i);
        seq |= ((list >> (4 * c)) & 15u) << (4 * i);
        const uint64_t lo = list & ((1ull << (4 * c)) - 1ull);
        const uint64_t hi = (list >> (4 * c + 4)) << (4 * c);
        list = lo | hi;
    }
    return seq;
}

template <bool ONE, bool STORE>
__global__ __launch_bounds__(CK_THREADS) void cke_enum_kernel(const tgo_task *__restrict__ tasks,
                                                             const int32_t *__restrict__ units, int n, int cap,
                                                             Rates r, uint32_t count, int64_t *out,
                                                             Partial *partials) {
    __shared__ CTab tb;
    __shared__ int flag;
    __shared__ int64_t kq[MAXN * CK_THREADS];
    const int st = ctab_load(tasks, units, n, cap, tb, &flag);
    if (st != 0) {
        if (threadIdx.x == 0) {
            Partial p = {};
            p.status = st;
            partials[blockIdx.x] = p;
        }
        return;
    }
    Partial p;
    p.min_t = ~0ull; p.min_r = ~0ull; p.max_t = 0; p.max_r = ~0ull;
    p.sum_lo = 0; p.sum_hi = 0; p.fp = 0; p.status = 0; p.pad = 0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t rk = blockIdx.x * blockDim.x + threadIdx.x; rk < count; rk += stride) {
        const uint64_t T = (uint64_t)cke_sim<ONE>(ck_unrank(n, rk), n, tb, cap, r, kq + threadIdx.x, CK_THREADS).T;
        if constexpr (STORE) out[rk] = (int64_t)T;
        if (T < p.min_t) { p.min_t = T; p.min_r = rk; }
        if (T + 1 > p.max_t) { p.max_t = T + 1; p.max_r = rk; }
        add128(p.sum_lo, p.sum_hi, T, 0);
        p.fp += (2ull * rk + 1ull) * T;
    }
    for (int m = 32; m >= 1; m >>= 1) {
        const uint64_t mt = shfl_xor64(p.min_t, m), mr = shfl_xor64(p.min_r, m);
        const uint64_t xt = shfl_xor64(p.max_t, m), xr = shfl_xor64(p.max_r, m);
        const uint64_t sl = shfl_xor64(p.sum_lo, m), sh = shfl_xor64(p.sum_hi, m);
        const uint64_t f = shfl_xor64(p.fp, m);
        merge_min(p.min_t, p.min_r, mt, mr);
        merge_max(p.max_t, p.max_r, xt, xr);
        add128(p.sum_lo, p.sum_hi, sl, sh);
        p.fp += f;
    }
    __shared__ Partial wsum[CK_THREADS / 64];
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x / 64] = p;
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial o = wsum[0];
        for (int i = 1; i < CK_THREADS / 64; ++i) {
            merge_min(o.min_t, o.min_r, wsum[i].min_t, wsum[i].min_r);
            merge_max(o.max_t, o.max_r, wsum[i].max_t, wsum[i].max_r);
            add128(o.sum_lo, o.sum_hi, wsum[i].sum_lo, wsum[i].sum_hi);
            o.fp += wsum[i].fp;
        }
        o.status = 0;
        o.pad = 0;
        partials[blockIdx.x] = o;
    }
}

// T of given orderings (rows of n bytes), or a negative TGO_E*.
template <bool ONE>
__global__ __launch_bounds__(CK_THREADS) void cke_evaluate_kernel(const tgo_task *__restrict__ tasks,
                                                                 const int32_t *__restrict__ units, int n, int cap,
                                                                 Rates r, const uint8_t *__restrict__ orders,
                                                                 int64_t m, int64_t *out) {
    __shared__ CTab tb;
    __shared__ int flag;
    __shared__ int64_t kq[MAXN * CK_THREADS];
    const int st = ctab_load(tasks, units, n, cap, tb, &flag);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    if (st != 0) {
        out[i] = st;
        return;
    }
    uint64_t seq = 0;
    uint32_t seen = 0;
    for (int j = 0; j < n; ++j) {
        const uint32_t x = orders[i * n + j];
        if (x < (uint32_t)n) seen |= 1u << x;
        seq |= (uint64_t)(x & 15u) << (4 * j);
    }
    if (seen != (1u << n) - 1u) {
        out[i] = TGO_EINVAL;
        return;
    }
    out[i] = cke_sim<ONE>(seq, n, tb, cap, r, kq + threadIdx.x, CK_THREADS).T;
}

// Algorithm 1 (Section 5.1) with `update` simulating the ordered set under
// the same rule; one thread.  Writes heur / heur_ns of the summary.
template <bool ONE>
__global__ __launch_bounds__(64) void cke_heuristic_kernel(const tgo_task *__restrict__ tasks,
                                                           const int32_t *__restrict__ units, int n, int cap,
                                                           Rates r, tgo_summary *out) {
    __shared__ CTab tb;
    __shared__ int flag;
    __shared__ int64_t kq[MAXN];
    const int st = ctab_load(tasks, units, n, cap, tb, &flag);
    if (threadIdx.x != 0) return;
    if (st != 0) {
        out->heur_ns = st;
        return;
    }
    auto update = [&](uint64_t seq, int len) {
        const CkeOut o = cke_sim<ONE>(seq, len, tb, cap, r, kq, 1);
        Fit3 u;
        u.th = o.th;
        u.tk = o.tk;
        u.td = o.td;
        return u;
    };
    uint64_t seq = 0;
    uint32_t rt = (1u << n) - 1u;
    int first = 0;
    for (int x = 1; x < n; ++x) {
        const int64_t kh = tb.k[x] - tb.h[x], bkh = tb.k[first] - tb.h[first];
        if (kh > bkh || (kh == bkh && tb.d[x] > tb.d[first])) first = x;
    }
    seq = (uint64_t)first;
    rt &= ~(1u << first);
    int pos = 1;
    while (__popc(rt) > 2) {
        const Fit3 u = update(seq, pos);
        int best = -1;
        int64_t bf = 0;
        for (int c = 0; c < n; ++c) {
            if (!((rt >> c) & 1u)) continue;
            const int64_t f = fit(tb.h[c], tb.k[c], u);
            if (best < 0 || f < bf) { best = c; bf = f; }
        }
        seq |= (uint64_t)best << (4 * pos);
        ++pos;
        rt &= ~(1u << best);
    }
    if (__popc(rt) == 2) {
        const int a = __ffs(rt) - 1, b = 31 - __clz(rt);
        const Fit3 u = update(seq, pos);
        int bx = -1, by = -1;
        int64_t bs = 0, bdy = 0;
        for (int o = 0; o < 2; ++o) {
            const int x = o == 0 ? a : b, y = o == 0 ? b : a;
            const int64_t s1 = fit(tb.h[x], tb.k[x], u);
            const Fit3 w = update(seq | ((uint64_t)x << (4 * pos)), pos + 1);
            const int64_t sc = s1 + fit(tb.h[y], tb.k[y], w) + tb.d[y];
            if (bx < 0 || sc < bs || (sc == bs && tb.d[y] < bdy)) { bx = x; by = y; bs = sc; bdy = tb.d[y]; }
        }
        seq |= ((uint64_t)bx << (4 * pos)) | ((uint64_t)by << (4 * (pos + 1)));
        pos += 2;
    } else if (__popc(rt) == 1) {
        seq |= (uint64_t)(__ffs(rt) - 1) << (4 * pos);
        ++pos;
    }
    for (int j = 0; j < 16; ++j) out->heur[j] = j < n ? (uint8_t)ck_nib(seq, j) : (uint8_t)0xff;
    out->heur_ns = cke_sim<ONE>(seq, n, tb, cap, r, kq, 1).T;
}

static int check_cke(const tgo_model *model, Rates *r, int n, int max_n, int32_t cap) {
    int rc = make_rates(model, r);
    if (rc) return rc;
    if (n < 1 || n > max_n) return fail(TGO_EINVAL, "n out of range");
    if (cap < 1 || cap > CK_MAX_CAPACITY) return fail(TGO_EINVAL, "capacity must be in 1..2^30");
    return TGO_OK;
}

}  // namespace tgo

using namespace tgo;

extern "C" {

int tgo_exhaustive_cke(const tgo_model *model, const tgo_task *d_tasks, const int32_t *d_units, int n,
                       int32_t capacity, int64_t *d_per_order, tgo_summary *d_summary, tgo_stream stream) {
    Rates r;
    int rc = check_cke(model, &r, n, TGO_MAX_CKE_N, capacity);
    if (rc) return rc;
    if (!d_tasks || !d_units || !d_summary) return fail(TGO_EINVAL, "NULL buffer");
    hipStream_t st = (hipStream_t)stream;
    const uint64_t count = factorial(n);
    const uint64_t want = (count + CK_THREADS - 1) / CK_THREADS;
    const uint32_t blocks = (uint32_t)(want < CK_MAX_BLOCKS ? want : CK_MAX_BLOCKS);
    Partial *parts = nullptr;
    rc = workspace(sizeof(Partial) * blocks, (void **)&parts, st);
    if (rc) return rc;
    const uint32_t c32 = (uint32_t)count;
    const bool one = r.one_dma != 0;
    if (one) {
        if (d_per_order)
            hipLaunchKernelGGL((cke_enum_kernel<true, true>), dim3(blocks), dim3(CK_THREADS), 0, st, d_tasks, d_units,
                               n, capacity, r, c32, d_per_order, parts);
        else
            hipLaunchKernelGGL((cke_enum_kernel<true, false>), dim3(blocks), dim3(CK_THREADS), 0, st, d_tasks,
                               d_units, n, capacity, r, c32, nullptr, parts);
    } else {
        if (d_per_order)
            hipLaunchKernelGGL((cke_enum_kernel<false, true>), dim3(blocks), dim3(CK_THREADS), 0, st, d_tasks,
                               d_units, n, capacity, r, c32, d_per_order, parts);
        else
            hipLaunchKernelGGL((cke_enum_kernel<false, false>), dim3(blocks), dim3(CK_THREADS), 0, st, d_tasks,
                               d_units, n, capacity, r, c32, nullptr, parts);
    }
    TGO_HIP(hipGetLastError());
    rc = launch_summary_finalize(parts, (int)blocks, n, 1, count, count, d_summary, st);
    if (rc) return rc;
    if (one)
        hipLaunchKernelGGL(cke_heuristic_kernel<true>, dim3(1), dim3(64), 0, st, d_tasks, d_units, n, capacity, r,
                           d_summary);
    else
        hipLaunchKernelGGL(cke_heuristic_kernel<false>, dim3(1), dim3(64), 0, st, d_tasks, d_units, n, capacity, r,
                           d_summary);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

int tgo_evaluate_cke(const tgo_model *model, const tgo_task *d_tasks, const int32_t *d_units, int n,
                     int32_t capacity, const uint8_t *d_orders, int64_t m, int64_t *d_out, tgo_stream stream) {
    Rates r;
    int rc = check_cke(model, &r, n, TGO_MAX_N, capacity);
    if (rc) return rc;
    if (m < 0 || m > ((int64_t)1 << 40)) return fail(TGO_EINVAL, "m must be in 0..2^40");
    if (m == 0) return TGO_OK;
    if (!d_tasks || !d_units || !d_orders || !d_out) return fail(TGO_EINVAL, "NULL buffer");
    hipStream_t st = (hipStream_t)stream;
    const int64_t blocks = (m + CK_THREADS - 1) / CK_THREADS;
    if (r.one_dma)
        hipLaunchKernelGGL(cke_evaluate_kernel<true>, dim3((uint32_t)blocks), dim3(CK_THREADS), 0, st, d_tasks,
                           d_units, n, capacity, r, d_orders, m, d_out);
    else
        hipLaunchKernelGGL(cke_evaluate_kernel<false>, dim3((uint32_t)blocks), dim3(CK_THREADS), 0, st, d_tasks,
                           d_units, n, capacity, r, d_orders, m, d_out);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

}  // extern "C"
