// Exhaustive evaluation of every launch ordering of one task group.
//
// Brute force over all n! orderings (the search that Section 1 and
// Section 5.1 rule out at runtime on a CPU), reduced to the best, worst and
// average ordering (the quantities plotted in Section 6).
//
// One lane per subtree (see enum_dev.h); lanes meet their ranks in increasing
// order, so the reduction keeps the lowest rank on ties.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "enum_dev.h"
#include "tables_dev.h"
#include "tgo_internal.h"

namespace tgo {

constexpr int EX_THREADS = 256;
constexpr int EX_MAX_BLOCKS_PER_PASS = 4096;

// Per-lane accumulators over all ranks the lane owns.
template <typename TT>
struct Acc {
    TT min_t;        // smallest T seen
    TT max_t1;       // largest T seen, plus one (0 = none yet)
    uint64_t min_r, max_r;
    uint64_t sum_lo, sum_hi;
    uint64_t fp;
};

template <typename TT>
__device__ __forceinline__ void acc_init(Acc<TT> &a) {
    a.min_t = inf_time<TT>();
    a.max_t1 = 0;
    a.min_r = ~0ull;
    a.max_r = ~0ull;
    a.sum_lo = 0;
    a.sum_hi = 0;
    a.fp = 0;
}

// Fold a finished subtree (first rank r0) into the lane accumulators.  The
// lane meets its subtrees in increasing rank order, so strict comparisons
// keep the lowest rank on ties.  fingerprint: sum of (2r+1) T with
// r = r0 + l is 2 (r0 sum T + sum l T) + sum T.
template <typename TT>
__device__ __forceinline__ void fold(Acc<TT> &a, const Sub<TT> &u, uint64_t r0) {
    if (u.min_t < a.min_t) { a.min_t = u.min_t; a.min_r = r0 + u.min_l; }
    if (u.max_t1 > a.max_t1) { a.max_t1 = u.max_t1; a.max_r = r0 + u.max_l; }
    const uint64_t lo = a.sum_lo + u.sum;
    a.sum_hi += lo < a.sum_lo ? 1ull : 0ull;
    a.sum_lo = lo;
    a.fp += 2ull * (r0 * u.sum + u.s2) + u.sum;
}

template <typename TT>
using ExView = View<TT, 1, EX_THREADS>;

// Reduce a block's lane accumulators into one Partial (thread 0 writes it).
__device__ void block_reduce_write(Partial p, Partial *dst) {
    __shared__ Partial wsum[EX_THREADS / 64];
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
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) wsum[w] = p;
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial o = wsum[0];
        for (int i = 1; i < (int)(blockDim.x / 64); ++i) {
            merge_min(o.min_t, o.min_r, wsum[i].min_t, wsum[i].min_r);
            merge_max(o.max_t, o.max_r, wsum[i].max_t, wsum[i].max_r);
            add128(o.sum_lo, o.sum_hi, wsum[i].sum_lo, wsum[i].sum_hi);
            o.fp += wsum[i].fp;
        }
        o.status = 0;
        o.pad = 0;
        *dst = o;
    }
}

// MODE: 0 = 32-bit time path, 1 = 64-bit.  Both instantiations are launched;
// a block whose group does not belong to its mode returns at once.  DMA is
// the launch scheme (DMA_TWO or DMA_ONE, fixed per instantiation).
template <typename TT, int M, bool STORE, int DMA>
__global__ __launch_bounds__(EX_THREADS) void exhaustive_kernel(const tgo_task *__restrict__ tasks,
                                                                int n, Rates r, uint32_t n_sub,
                                                                int64_t *out, Partial *partials) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int MODE = sizeof(TT) == 4 ? 0 : 1;
    __shared__ Quad<TT> Ht[MAXN];
    __shared__ DRec<TT> Dt[MAXN];
    __shared__ int mode;
    if (threadIdx.x == 0) mode = classify_group(tasks, n, r);
    if ((int)threadIdx.x < n) table_entry<TT>(tasks[threadIdx.x], r, &Ht[threadIdx.x], &Dt[threadIdx.x]);
    __syncthreads();
    if (mode < 0) {
        if (MODE == 0 && threadIdx.x == 0) {
            Partial p = {};
            p.status = mode;
            partials[blockIdx.x] = p;
        }
        return;
    }
    if (mode != MODE) return;

    ExView<TT> v;
    v.H = Ht;
    v.D = Dt;
    v.Q = reinterpret_cast<Slot<TT> *>(smem) + threadIdx.x;
    Ctx c;
    c.n = n;
    c.r = r;
    c.out_sub = nullptr;

    Acc<TT> a;
    acc_init(a);
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n_sub; s += stride) {
        Lane<TT> st;
        const uint64_t list = prefix<DMA>(st, s, n, M, v, r);
        const uint64_t r0 = (uint64_t)s * factorial(M);
        if constexpr (STORE) c.out_sub = out + r0;
        Sub<TT> u;
        sub_init(u);
        level<TT, M, STORE, 1, EX_THREADS, DMA>(c, v, st, (uint32_t)list, 0u, u);
        fold(a, u, r0);
    }
    Partial p;
    p.min_t = (uint64_t)a.min_t;
    p.min_r = a.min_r;
    if constexpr (sizeof(TT) == 4) {
        p.min_t = a.min_t == inf_time<TT>() ? ~0ull : (uint64_t)a.min_t;
    }
    p.max_t = (uint64_t)a.max_t1;
    p.max_r = a.max_r;
    p.sum_lo = a.sum_lo;
    p.sum_hi = a.sum_hi;
    p.fp = a.fp;
    p.status = 0;
    p.pad = 0;
    block_reduce_write(p, &partials[blockIdx.x]);
}

__device__ inline void unrank_dev(int n, uint64_t r, uint8_t *out) {
    uint64_t list = 0;
    for (int i = n - 1; i >= 0; --i) list = (list << 4) | (uint64_t)i;
    uint64_t f = 1;
    for (int i = 2; i <= n - 1; ++i) f *= (uint64_t)i;
    for (int i = 0; i < n; ++i) {
        const uint64_t cd = f ? r / f : 0;
        r -= cd * f;
        if (n - 1 - i > 0) f /= (uint64_t)(n - 1 - i);
        out[i] = (uint8_t)((list >> (4 * cd)) & 15u);
        const uint64_t lo = list & ((1ull << (4 * cd)) - 1ull);
        const uint64_t hi = (list >> (4 * cd + 4)) << (4 * cd);
        list = lo | hi;
    }
    for (int i = n; i < 16; ++i) out[i] = 0xff;
}

__global__ __launch_bounds__(256) void exhaustive_finalize(const Partial *__restrict__ parts,
                                                           int nparts, int n, uint64_t count,
                                                           tgo_summary *out) {
    __shared__ Partial red[256];
    __shared__ int status;
    if (threadIdx.x == 0) status = 0;
    __syncthreads();
    Partial p;
    p.min_t = ~0ull; p.min_r = ~0ull; p.max_t = 0; p.max_r = ~0ull;
    p.sum_lo = 0; p.sum_hi = 0; p.fp = 0; p.status = 0; p.pad = 0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        const Partial q = parts[i];
        if (q.status != 0) atomicMin(&status, q.status);
        merge_min(p.min_t, p.min_r, q.min_t, q.min_r);
        merge_max(p.max_t, p.max_r, q.max_t, q.max_r);
        add128(p.sum_lo, p.sum_hi, q.sum_lo, q.sum_hi);
        p.fp += q.fp;
    }
    red[threadIdx.x] = p;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            Partial q = red[threadIdx.x + s];
            Partial &o = red[threadIdx.x];
            merge_min(o.min_t, o.min_r, q.min_t, q.min_r);
            merge_max(o.max_t, o.max_r, q.max_t, q.max_r);
            add128(o.sum_lo, o.sum_hi, q.sum_lo, q.sum_hi);
            o.fp += q.fp;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        tgo_summary s;
        const Partial &o = red[0];
        s.n = n;
        s.status = status;
        s.count = count;
        for (int i = 0; i < 16; ++i) { s.best[i] = 0xff; s.worst[i] = 0xff; s.heur[i] = 0xff; }
        s.heur_ns = -1;
        if (status != 0) {
            s.min_ns = s.max_ns = 0;
            s.argmin_rank = s.argmax_rank = 0;
            s.sum_lo = s.sum_hi = 0;
            s.fingerprint = 0;
            s.mean_ns = 0.0;
        } else {
            s.min_ns = (int64_t)o.min_t;
            s.argmin_rank = o.min_r;
            s.max_ns = (int64_t)(o.max_t - 1);
            s.argmax_rank = o.max_r;
            s.sum_lo = o.sum_lo;
            s.sum_hi = o.sum_hi;
            s.fingerprint = o.fp;
            // mean = sum / count: whole part exactly, then the fraction
            double mean;
            if (o.sum_hi == 0) {
                const uint64_t qt = o.sum_lo / count, rm = o.sum_lo % count;
                mean = (double)qt + (double)rm / (double)count;
            } else {
                mean = ((double)o.sum_hi * 18446744073709551616.0 + (double)o.sum_lo) / (double)count;
            }
            s.mean_ns = mean;
            unrank_dev(n, o.min_r, s.best);
            unrank_dev(n, o.max_r, s.worst);
        }
        *out = s;
    }
}

// Positions enumerated depth-first per lane: enough subtrees to fill the GPU.
// TGO_EXHAUSTIVE_M overrides the choice for tuning experiments (1..5, or
// 1..6 with one DMA engine).
static int choose_m(int n, bool one_dma) {
    const int cap = one_dma ? 6 : 5;
    if (const char *e = std::getenv("TGO_EXHAUSTIVE_M")) {
        const int m = std::atoi(e);
        if (m >= 1 && m <= cap && m <= n) return m;
    }
    // two engines: 4 levels beat 5 at n = 12 on MI355X (fewer live
    // snapshots, one more wave per SIMD); deeper walks only pay when
    // subtrees are scarce.  One engine: a window is a handful of operations,
    // so the per-subtree prefix decode is worth amortising over 6 levels.
    const int top = one_dma ? 6 : 4;
    int m = 1;
    for (int c = top; c >= 1; --c) {
        if (c > n) continue;
        const uint64_t sub = factorial(n) / factorial(c);
        if (sub >= 32768 || c == 1) { m = c; break; }
    }
    if (n <= 5) m = n < 1 ? 1 : n;
    return m;
}

template <int M, bool STORE, int DMA>
static void launch_pair(dim3 grid, size_t shm32, size_t shm64, hipStream_t st, const tgo_task *t,
                        int n, const Rates &r, uint32_t n_sub, int64_t *out, Partial *parts) {
    hipLaunchKernelGGL((exhaustive_kernel<uint32_t, M, STORE, DMA>), grid, dim3(EX_THREADS), shm32, st, t, n, r,
                       n_sub, out, parts);
    hipLaunchKernelGGL((exhaustive_kernel<uint64_t, M, STORE, DMA>), grid, dim3(EX_THREADS), shm64, st, t, n, r,
                       n_sub, out, parts);
}

template <bool STORE, int DMA>
static void launch_m(int m, dim3 grid, size_t shm32, size_t shm64, hipStream_t st,
                     const tgo_task *t, int n, const Rates &r, uint32_t n_sub, int64_t *out,
                     Partial *parts) {
    switch (m) {
        case 1: launch_pair<1, STORE, DMA>(grid, shm32, shm64, st, t, n, r, n_sub, out, parts); break;
        case 2: launch_pair<2, STORE, DMA>(grid, shm32, shm64, st, t, n, r, n_sub, out, parts); break;
        case 3: launch_pair<3, STORE, DMA>(grid, shm32, shm64, st, t, n, r, n_sub, out, parts); break;
        case 4: launch_pair<4, STORE, DMA>(grid, shm32, shm64, st, t, n, r, n_sub, out, parts); break;
        case 5: launch_pair<5, STORE, DMA>(grid, shm32, shm64, st, t, n, r, n_sub, out, parts); break;
        default:
            if constexpr (DMA == DMA_ONE)
                launch_pair<6, STORE, DMA>(grid, shm32, shm64, st, t, n, r, n_sub, out, parts);
            else
                launch_pair<5, STORE, DMA>(grid, shm32, shm64, st, t, n, r, n_sub, out, parts);
            break;
    }
}

int launch_exhaustive(const Rates &r, const tgo_task *d_tasks, int n, int64_t *d_per_order,
                      tgo_summary *d_out, hipStream_t st) {
    const bool one = r.one_dma != 0;
    const int m = choose_m(n, one);
    const uint64_t n_sub64 = factorial(n) / factorial(m);
    if (n_sub64 >= (1ull << 32)) return fail(TGO_EINVAL, "group too large to enumerate");
    const uint32_t n_sub = (uint32_t)n_sub64;
    const uint64_t lanes_per_pass = (uint64_t)EX_THREADS * EX_MAX_BLOCKS_PER_PASS;
    const uint64_t passes = (n_sub64 + lanes_per_pass - 1) / lanes_per_pass;
    const uint64_t per_block = (uint64_t)EX_THREADS * passes;
    const uint32_t blocks = (uint32_t)((n_sub64 + per_block - 1) / per_block);
    Partial *parts = nullptr;
    int rc = workspace(sizeof(Partial) * blocks, (void **)&parts);
    if (rc) return rc;
    // the kernel-completion queue is read only by the two-engine DtH events
    const size_t shm32 = one ? 0 : sizeof(Slot<uint32_t>) * EX_THREADS * n;
    const size_t shm64 = one ? 0 : sizeof(Slot<uint64_t>) * EX_THREADS * n;
    const dim3 g(blocks);
    if (one) {
        if (d_per_order)
            launch_m<true, DMA_ONE>(m, g, shm32, shm64, st, d_tasks, n, r, n_sub, d_per_order, parts);
        else
            launch_m<false, DMA_ONE>(m, g, shm32, shm64, st, d_tasks, n, r, n_sub, nullptr, parts);
    } else {
        if (d_per_order)
            launch_m<true, DMA_TWO>(m, g, shm32, shm64, st, d_tasks, n, r, n_sub, d_per_order, parts);
        else
            launch_m<false, DMA_TWO>(m, g, shm32, shm64, st, d_tasks, n, r, n_sub, nullptr, parts);
    }
    TGO_HIP(hipGetLastError());
    hipLaunchKernelGGL(exhaustive_finalize, dim3(1), dim3(256), 0, st, parts, (int)blocks, n,
                       factorial(n), d_out);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

}  // namespace tgo
