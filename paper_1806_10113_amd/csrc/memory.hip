// Task groups under a device-memory limit (the reading and the lane
// simulators are described in mem_dev.h): every ordering, T of given
// orderings, and Algorithm 1 with its update step under the limit.
//
// Enumeration.  Lexicographic ranks put the orderings that share their first
// n - M positions in one block of M! consecutive ranks.  One lane owns such a
// block: it places the prefix once, then walks the last M positions depth
// first in ascending task order (which is rank order), keeping the state
// after each placed position and extending a copy of it for every choice of
// the next one.  With two DMA engines a placed position's state is the
// instant its HtD ends, so only the events after that instant are stepped
// again per extension; with one DMA engine the state is the chain's running
// ends and the open sub-group.  Work per ordering is then mostly the last
// position's events instead of all 3n of them.
//
// The 32-bit instantiation runs when every instant and work amount of the
// group fits 31 bits (the same bound as the single-group enumeration); the
// 64-bit twin runs otherwise; each block of the other one returns at once.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <type_traits>

#include "enum_dev.h"
#include "heur_dev.h"
#include "mem_dev.h"
#include "tables_dev.h"
#include "tgo_internal.h"

namespace tgo {

constexpr int MEM_THREADS = 256;
// Blocks per launch at most: about 8 rounds of the resident blocks with two
// engines (2,048 at 8 waves per SIMD), where subtrees vary most in cost
// (n = 12: 16,384 blocks 10.4 / 14.9 / 16.2 ms at capacity 100 / 60 / 40 %
// against 10.7 / 15.6 / 16.9 ms with 8,192); with one engine 8,192 (16,384
// was 4-6 % slower, 4,096 the same).
constexpr int MEM_MAX_BLOCKS_TWO = 16384;
constexpr int MEM_MAX_BLOCKS_ONE = 8192;

__constant__ uint32_t MEM_FACT[13] = {1u,      1u,       2u,        6u,         24u,        120u,     720u,
                                      5040u,   40320u,   362880u,   3628800u,   39916800u,  479001600u};

// Task tables of the block (n <= 16 threads fill them).  Returns the block's
// status: 0 (this instantiation runs), 1 (the other width runs), or a
// negative TGO_E* code.
template <typename TT>
__device__ __forceinline__ int mem_tables(const tgo_task *__restrict__ tasks, const int64_t *__restrict__ mem,
                                          int n, uint64_t cap, const Rates &r, MemTab<TT> &tb, int *flag) {
    constexpr int MODE = sizeof(TT) == 4 ? 0 : 1;
    if (threadIdx.x == 0) *flag = classify_group(tasks, n, r);
    __syncthreads();
    if ((int)threadIdx.x < n) {
        const tgo_task t = tasks[threadIdx.x];
        const int64_t m = mem[threadIdx.x];
        if (m < 0 || (uint64_t)m > cap) atomicMin(flag, (int)TGO_EINVAL);
        const uint64_t q = 1ull << r.q_log2;
        tb.h[threadIdx.x] = (TT)t.htd_ns;
        tb.k[threadIdx.x] = (TT)t.kern_ns;
        tb.d[threadIdx.x] = (TT)t.dth_ns;
        tb.qh[threadIdx.x] = (TT)(q * (uint64_t)t.htd_ns);
        tb.qd[threadIdx.x] = (TT)(q * (uint64_t)t.dth_ns);
        tb.m[threadIdx.x] = (uint64_t)m;
    }
    __syncthreads();
    const int f = *flag;
    return f < 0 ? f : (f == MODE ? 0 : 1);
}

template <typename TT>
__device__ __forceinline__ void mem_push(GSim<TT> &s, uint32_t x, const MemTab<TT> &tb, uint64_t cap,
                                         const Rates &r, const KQ<TT> &kq) {
    gsim_push(s, x, tb, cap, r, kq);
}
template <typename TT>
__device__ __forceinline__ void mem_push(Chain<TT> &c, uint32_t x, const MemTab<TT> &tb, uint64_t cap,
                                         const Rates &, const KQ<TT> &) {
    chain_push(c, x, tb, cap);
}
template <typename TT>
__device__ __forceinline__ TT mem_finish(GSim<TT> &s, const MemTab<TT> &tb, const Rates &r, const KQ<TT> &kq) {
    return gsim_finish(s, tb, r, kq);
}
template <typename TT>
__device__ __forceinline__ TT mem_finish(Chain<TT> &c, const MemTab<TT> &tb, const Rates &, const KQ<TT> &) {
    return chain_finish(c, tb);
}

// Per-lane reduction over the lane's ranks, visited in increasing order.
struct MAcc {
    uint64_t min_t, min_r, max_t1, max_r, sum_lo, sum_hi, fp, rank;
};

template <bool STORE>
__device__ __forceinline__ void mem_leaf(MAcc &a, uint64_t T, int64_t *out) {
    const uint64_t rk = a.rank++;
    if constexpr (STORE) out[rk] = (int64_t)T;
    if (T < a.min_t) { a.min_t = T; a.min_r = rk; }
    if (T + 1 > a.max_t1) { a.max_t1 = T + 1; a.max_r = rk; }
    add128(a.sum_lo, a.sum_hi, T, 0);
    a.fp += (2 * rk + 1) * T;
}

// Depth-first walk of the last D positions over the tasks in `rem`
// (ascending task index = lexicographic rank order).
template <int D, bool STORE, typename S, typename TT>
__device__ __forceinline__ void mem_dfs(const S &s, uint32_t rem, const MemTab<TT> &tb, uint64_t cap,
                                        const Rates &r, const KQ<TT> &kq, MAcc &a, int64_t *out) {
    uint32_t m = rem;
    for (int i = 0; i < D; ++i) {
        const uint32_t x = (uint32_t)(__ffs(m) - 1);
        m &= m - 1;
        S c = s;
        mem_push(c, x, tb, cap, r, kq);
        if constexpr (D == 1) {
            mem_leaf<STORE>(a, (uint64_t)mem_finish(c, tb, r, kq), out);
        } else {
            mem_dfs<D - 1, STORE>(c, rem & ~(1u << x), tb, cap, r, kq, a, out);
        }
    }
}

// 32-bit time path: VGPRs capped for 8 waves per SIMD with two DMA engines
// (64 VGPRs; the per-lane queue is 12 KB per block, so 8 blocks fit per CU)
// and 6 with one.  The compiler spills some saved walk state to scratch,
// which the extra waves more than pay for: at n = 12, capacity 100 / 60 /
// 40 / 25 % of the footprint, 12.4 / 18.2 / 19.9 / 19.9 ms uncapped (90
// VGPRs, 5 waves), 11.1 / 16.0 / 17.4 / 17.5 ms at 7 waves, 10.8 / 15.6 /
// 16.9 / 16.9 ms at 8; one engine 1.20-1.24 -> 1.16-1.22 ms.
template <typename TT, bool ONE>
constexpr int mem_min_waves() { return sizeof(TT) == 4 ? (ONE ? 6 : 8) : 1; }

template <typename TT, bool ONE, bool STORE, int M>
__global__ __launch_bounds__(MEM_THREADS) __attribute__((amdgpu_waves_per_eu(mem_min_waves<TT, ONE>()))) void mem_enum_kernel(const tgo_task *__restrict__ tasks,
                                                               const int64_t *__restrict__ mem, int n,
                                                               uint64_t cap, Rates r, uint32_t n_sub,
                                                               int64_t *out, Partial *partials) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ MemTab<TT> tb;
    __shared__ int flag;
    const int st = mem_tables<TT>(tasks, mem, n, cap, r, tb, &flag);
    if (st < 0) {
        if (sizeof(TT) == 4 && threadIdx.x == 0) {
            Partial p = {};
            p.status = st;
            partials[blockIdx.x] = p;
        }
        return;
    }
    if (st != 0) return;
    using S = typename std::conditional<ONE, Chain<TT>, GSim<TT>>::type;
    // two engines: the lane's kernel-end queue, n slots (none with one engine)
    const KQ<TT> kq{reinterpret_cast<TT *>(smem) + threadIdx.x, MEM_THREADS};
    MAcc a;
    a.min_t = ~0ull; a.min_r = ~0ull; a.max_t1 = 0; a.max_r = ~0ull;
    a.sum_lo = 0; a.sum_hi = 0; a.fp = 0; a.rank = 0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t sub = blockIdx.x * blockDim.x + threadIdx.x; sub < n_sub; sub += stride) {
        S s;
        if constexpr (ONE) chain_init(s);
        else gsim_init(s);
        // prefix: position i takes digit c of the factorial base (radix n - i)
        uint64_t list = 0;
        for (int i = n - 1; i >= 0; --i) list = (list << 4) | (uint64_t)i;
        uint32_t rest = sub;
        for (int i = 0; i < n - M; ++i) {
            const uint32_t block = MEM_FACT[n - 1 - i] / MEM_FACT[M];
            const uint32_t c = rest / block;
            rest -= c * block;
            const uint32_t x = (uint32_t)(list >> (4 * c)) & 15u;
            const uint64_t lo = list & ((1ull << (4 * c)) - 1ull);
            list = lo | ((list >> (4 * c + 4)) << (4 * c));
            mem_push(s, x, tb, cap, r, kq);
        }
        uint32_t remset = 0;
        for (int i = 0; i < M; ++i) remset |= 1u << ((list >> (4 * i)) & 15u);
        a.rank = (uint64_t)sub * MEM_FACT[M];
        mem_dfs<M, STORE>(s, remset, tb, cap, r, kq, a, out);
    }
    Partial p;
    p.min_t = a.min_t; p.min_r = a.min_r; p.max_t = a.max_t1; p.max_r = a.max_r;
    p.sum_lo = a.sum_lo; p.sum_hi = a.sum_hi; p.fp = a.fp; p.status = 0; p.pad = 0;
    for (int o = 32; o >= 1; o >>= 1) {
        const uint64_t mt = shfl_xor64(p.min_t, o), mr = shfl_xor64(p.min_r, o);
        const uint64_t xt = shfl_xor64(p.max_t, o), xr = shfl_xor64(p.max_r, o);
        const uint64_t sl = shfl_xor64(p.sum_lo, o), sh = shfl_xor64(p.sum_hi, o);
        const uint64_t f = shfl_xor64(p.fp, o);
        merge_min(p.min_t, p.min_r, mt, mr);
        merge_max(p.max_t, p.max_r, xt, xr);
        add128(p.sum_lo, p.sum_hi, sl, sh);
        p.fp += f;
    }
    __shared__ Partial wsum[MEM_THREADS / 64];
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x / 64] = p;
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial o = wsum[0];
        for (int i = 1; i < MEM_THREADS / 64; ++i) {
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

// Simulate the group launched in ord[0..len) alone: (end of its last HtD,
// kernel, DtH) -- Algorithm 1's update -- in 64-bit time.
template <bool ONE>
__device__ Fit3 mem_update(const uint8_t *ord, int len, const MemTab<uint64_t> &tb, uint64_t cap,
                           const Rates &r, const KQ<uint64_t> &kq) {
    Fit3 u;
    if constexpr (ONE) {
        Chain<uint64_t> c;
        chain_init(c);
        for (int i = 0; i < len; ++i) chain_push(c, ord[i], tb, cap);
        u.th = (int64_t)c.x;
        u.tk = (int64_t)c.kp;
        u.td = (int64_t)chain_finish(c, tb);
    } else {
        GSim<uint64_t> s;
        gsim_init(s);
        for (int i = 0; i < len; ++i) gsim_push(s, ord[i], tb, cap, r, kq);
        u.th = (int64_t)s.t;
        u.tk = (int64_t)s.kp;
        u.td = (int64_t)gsim_finish(s, tb, r, kq);
    }
    return u;
}

// Algorithm 1 under the limit (one thread): the selection rules of the
// unconstrained heuristic (heur_dev.h), every update simulated under it.
template <bool ONE>
__global__ __launch_bounds__(64) void mem_heuristic_kernel(const tgo_task *__restrict__ tasks,
                                                           const int64_t *__restrict__ mem, int n, uint64_t cap,
                                                           Rates r, tgo_summary *out) {
    __shared__ MemTab<uint64_t> tb;
    __shared__ int flag;
    __shared__ uint64_t kqs[MAXN];
    const KQ<uint64_t> kq{kqs, 1};
    const int st = mem_tables<uint64_t>(tasks, mem, n, cap, r, tb, &flag);
    if (threadIdx.x != 0) return;
    if (st < 0) {
        out->heur_ns = st;
        return;
    }
    uint8_t ord[MAXN];
    uint32_t rt = (1u << n) - 1u;
    int first = 0;
    for (int x = 1; x < n; ++x) {
        const int64_t kh = (int64_t)tb.k[x] - (int64_t)tb.h[x];
        const int64_t bkh = (int64_t)tb.k[first] - (int64_t)tb.h[first];
        if (kh > bkh || (kh == bkh && tb.d[x] > tb.d[first])) first = x;
    }
    ord[0] = (uint8_t)first;
    rt &= ~(1u << first);
    int pos = 1;
    while (__popc(rt) > 2) {
        const Fit3 u = mem_update<ONE>(ord, pos, tb, cap, r, kq);
        int best = -1;
        int64_t bf = 0;
        for (int c = 0; c < n; ++c) {
            if (!((rt >> c) & 1u)) continue;
            const int64_t f = fit((int64_t)tb.h[c], (int64_t)tb.k[c], u);
            if (best < 0 || f < bf) { best = c; bf = f; }
        }
        ord[pos++] = (uint8_t)best;
        rt &= ~(1u << best);
    }
    if (__popc(rt) == 2) {
        const int a = __ffs(rt) - 1, b = 31 - __clz(rt);
        const Fit3 u = mem_update<ONE>(ord, pos, tb, cap, r, kq);
        int bx = -1, by = -1;
        int64_t bs = 0, bdy = 0;
        for (int o = 0; o < 2; ++o) {
            const int x = o == 0 ? a : b, y = o == 0 ? b : a;
            ord[pos] = (uint8_t)x;
            const Fit3 w = mem_update<ONE>(ord, pos + 1, tb, cap, r, kq);
            const int64_t dy = (int64_t)tb.d[y];
            const int64_t sc = fit((int64_t)tb.h[x], (int64_t)tb.k[x], u) +
                               fit((int64_t)tb.h[y], (int64_t)tb.k[y], w) + dy;
            if (bx < 0 || sc < bs || (sc == bs && dy < bdy)) { bx = x; by = y; bs = sc; bdy = dy; }
        }
        ord[pos] = (uint8_t)bx;
        ord[pos + 1] = (uint8_t)by;
        pos += 2;
    } else if (__popc(rt) == 1) {
        ord[pos++] = (uint8_t)(__ffs(rt) - 1);
    }
    const Fit3 f = mem_update<ONE>(ord, n, tb, cap, r, kq);
    for (int j = 0; j < 16; ++j) out->heur[j] = j < n ? ord[j] : (uint8_t)0xff;
    out->heur_ns = f.td;
}

// T of given orderings (rows of n bytes) under the limit; one lane per row,
// 64-bit time.
template <bool ONE>
__global__ __launch_bounds__(MEM_THREADS) void mem_evaluate_kernel(const tgo_task *__restrict__ tasks,
                                                                   const int64_t *__restrict__ mem, int n,
                                                                   uint64_t cap, Rates r,
                                                                   const uint8_t *__restrict__ orders, int64_t m,
                                                                   int64_t *out) {
    __shared__ MemTab<uint64_t> tb;
    __shared__ int flag;
    __shared__ uint64_t kqs[MAXN * MEM_THREADS];
    const KQ<uint64_t> kq{kqs + threadIdx.x, MEM_THREADS};
    const int st = mem_tables<uint64_t>(tasks, mem, n, cap, r, tb, &flag);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    if (st < 0) {
        out[i] = st;
        return;
    }
    uint8_t ord[MAXN];
    uint32_t seen = 0;
    for (int j = 0; j < n; ++j) {
        const uint8_t x = orders[i * n + j];
        if (x >= n || ((seen >> x) & 1u)) {
            out[i] = TGO_EINVAL;
            return;
        }
        seen |= 1u << x;
        ord[j] = x;
    }
    out[i] = mem_update<ONE>(ord, n, tb, cap, r, kq).td;
}

template <typename TT, bool ONE, bool STORE>
static void launch_enum_width(int M, dim3 grid, hipStream_t st, const tgo_task *t, const int64_t *mem, int n,
                              uint64_t cap, const Rates &r, uint32_t n_sub, int64_t *out, Partial *parts) {
    const size_t shm = ONE ? 0 : sizeof(TT) * MEM_THREADS * (size_t)n;
#define TGO_MEM_ENUM(MM)                                                                                         \
    hipLaunchKernelGGL((mem_enum_kernel<TT, ONE, STORE, MM>), grid, dim3(MEM_THREADS), shm, st, t, mem, n, cap, \
                       r, n_sub, out, parts)
    switch (M) {
        case 1: TGO_MEM_ENUM(1); break;
        case 2: TGO_MEM_ENUM(2); break;
        case 3: TGO_MEM_ENUM(3); break;
        case 4: TGO_MEM_ENUM(4); break;
        default: TGO_MEM_ENUM(5); break;
    }
#undef TGO_MEM_ENUM
}

template <bool ONE, bool STORE>
static void launch_enum(int M, dim3 grid, hipStream_t st, const tgo_task *t, const int64_t *mem, int n,
                        uint64_t cap, const Rates &r, uint32_t n_sub, int64_t *out, Partial *parts) {
    launch_enum_width<uint32_t, ONE, STORE>(M, grid, st, t, mem, n, cap, r, n_sub, out, parts);
    launch_enum_width<uint64_t, ONE, STORE>(M, grid, st, t, mem, n, cap, r, n_sub, out, parts);
}

// Positions walked depth first per lane, or n if smaller: 4 with two DMA
// engines (12.4 vs 14.9 ms at n = 12: one more wave per SIMD), 5 with one
// (a few per cent faster); TGO_MEM_M overrides it for tuning experiments
// (1..5).
static int choose_mem_m(int n, bool one_dma) {
    int m = one_dma ? 5 : 4;
    if (const char *e = std::getenv("TGO_MEM_M")) {
        const int v = std::atoi(e);
        if (v >= 1 && v <= 5) m = v;
    }
    return m < n ? m : n;
}

int launch_memory(const Rates &r, const tgo_task *d_tasks, const int64_t *d_mem, int n, int64_t cap,
                  int64_t *d_per_order, tgo_summary *d_out, hipStream_t st) {
    const int M = choose_mem_m(n, r.one_dma != 0);
    const uint64_t count = factorial(n);
    const uint32_t n_sub = (uint32_t)(count / factorial(M));
    const uint64_t want = ((uint64_t)n_sub + MEM_THREADS - 1) / MEM_THREADS;
    const uint64_t most = r.one_dma ? MEM_MAX_BLOCKS_ONE : MEM_MAX_BLOCKS_TWO;
    const uint32_t blocks = (uint32_t)(want < most ? want : most);
    Partial *parts = nullptr;
    int rc = workspace(sizeof(Partial) * blocks, (void **)&parts, st);
    if (rc) return rc;
    const uint64_t c = (uint64_t)cap;
    const dim3 g(blocks);
    if (r.one_dma) {
        if (d_per_order) launch_enum<true, true>(M, g, st, d_tasks, d_mem, n, c, r, n_sub, d_per_order, parts);
        else launch_enum<true, false>(M, g, st, d_tasks, d_mem, n, c, r, n_sub, nullptr, parts);
    } else {
        if (d_per_order) launch_enum<false, true>(M, g, st, d_tasks, d_mem, n, c, r, n_sub, d_per_order, parts);
        else launch_enum<false, false>(M, g, st, d_tasks, d_mem, n, c, r, n_sub, nullptr, parts);
    }
    TGO_HIP(hipGetLastError());
    rc = launch_summary_finalize(parts, (int)blocks, n, 1, count, count, d_out, st);
    if (rc) return rc;
    if (r.one_dma)
        hipLaunchKernelGGL(mem_heuristic_kernel<true>, dim3(1), dim3(64), 0, st, d_tasks, d_mem, n, c, r, d_out);
    else
        hipLaunchKernelGGL(mem_heuristic_kernel<false>, dim3(1), dim3(64), 0, st, d_tasks, d_mem, n, c, r, d_out);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

int launch_memory_evaluate(const Rates &r, const tgo_task *d_tasks, const int64_t *d_mem, int n, int64_t cap,
                           const uint8_t *d_orders, int64_t m, int64_t *d_out, hipStream_t st) {
    if (m == 0) return TGO_OK;
    const int64_t blocks = (m + MEM_THREADS - 1) / MEM_THREADS;
    if (r.one_dma)
        hipLaunchKernelGGL(mem_evaluate_kernel<true>, dim3((uint32_t)blocks), dim3(MEM_THREADS), 0, st, d_tasks,
                           d_mem, n, (uint64_t)cap, r, d_orders, m, d_out);
    else
        hipLaunchKernelGGL(mem_evaluate_kernel<false>, dim3((uint32_t)blocks), dim3(MEM_THREADS), 0, st, d_tasks,
                           d_mem, n, (uint64_t)cap, r, d_orders, m, d_out);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

}  // namespace tgo
