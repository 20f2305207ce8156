// Batched exhaustive evaluation: thousands of task groups of uneven size in
// one persistent launch, replayed from a HIP graph, with an autotuned work
// decomposition.  Per group the result is the same summary as for a single
// group (best / worst / mean over every ordering) plus the ordering of the
// heuristic of Section 5.1.
//
// Work decomposition.  Group g of size n is split into n!/m(n) subtrees
// (enum_dev.h), one lane per subtree; a wave-sized tile holds
// 64 * lane_mult consecutive subtrees of one group, so the four waves of a
// block work on up to four different groups, each with its own task table in
// LDS.  Waves pull tiles from a device counter until the batch is drained (a
// persistent grid), which balances groups whose work differs by a factor of
// 10!/4! without any host-side schedule.  Per-group results are combined with
// 64-bit atomics on packed (time, rank) keys, so they do not depend on the
// order in which tiles finish.
#include <type_traits>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <string>
#include <vector>

#include "enum_dev.h"
#include "tables_dev.h"
#include "tgo_internal.h"

namespace tgo {

constexpr int BT_THREADS = 256;
constexpr int BT_WAVES = BT_THREADS / 64;
constexpr int BT_MAX_N = 12;  // 12! < 2^29 keeps a rank in the low word of a key
constexpr int BT_MAX_M = 5;

struct BatchCfg {
    int8_t m[BT_MAX_N + 1];  // positions enumerated per lane, by group size
    int32_t lane_mult;       // subtrees per lane in one tile
    int32_t blocks;          // persistent grid size
};

struct GroupAcc {
    unsigned long long minkey;  // (T << 32) | rank, smallest
    unsigned long long maxkey;  // (T << 32) | (2^32 - 1 - rank), largest
    unsigned long long sum;     // sum of T (n <= 12 and T < 2^31: no overflow)
    unsigned long long fp;      // sum of (2 rank + 1) T mod 2^64
    int32_t status, n;
    int32_t wide, pad;          // 1: the group runs the 64-bit path (per-tile partials)
};

struct BatchHdr {
    unsigned int next_tile;
    unsigned int total_tiles;
    unsigned int next_wide;     // 64-bit path: tiles handed out / in total
    unsigned int total_wide;
};

// Groups whose times could reach 2^31 ns take the 64-bit path: a group of S
// subtrees is cut into W = min(S, wide_tiles) tiles of consecutive subtrees,
// one wave each, and every tile writes a partial summary of its own; the
// finalize reduces a group's partials.  No packed keys: T may need 46 bits.
constexpr int BT_WIDE_M = 3;              // positions enumerated per lane (64-bit path)
constexpr size_t BT_WIDE_BUDGET = 64u << 20;  // bytes of partials per plan
constexpr int BT_WIDE_TILES_MAX = 256;

__device__ __forceinline__ uint32_t subtrees_of(int n, int m) {
    return (uint32_t)(fact_c(n) / fact_c(m));
}

// One block: per-group status and tile counts, exclusive scan into tile_off,
// accumulators reset, tile counter reset.
__device__ __forceinline__ uint32_t wide_tiles_of(int n, int wide_tiles) {
    const uint32_t S = subtrees_of(n, n < BT_WIDE_M ? n : BT_WIDE_M);
    return S < (uint32_t)wide_tiles ? S : (uint32_t)wide_tiles;
}

// Inclusive block scan of v (1024 threads) in sc; returns the exclusive prefix.
__device__ __forceinline__ uint32_t block_exscan(uint32_t v, uint32_t *sc) {
    sc[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t x = threadIdx.x >= (unsigned)off ? sc[threadIdx.x - off] : 0u;
        __syncthreads();
        sc[threadIdx.x] += x;
        __syncthreads();
    }
    return sc[threadIdx.x] - v;
}

__global__ __launch_bounds__(1024) void batch_prepare(const tgo_task *__restrict__ tasks,
                                                      const int32_t *__restrict__ offs, int G,
                                                      Rates r, BatchCfg cfg, int wide_tiles, int max_n, GroupAcc *acc,
                                                      uint32_t *tile_off, uint32_t *wtile_off, BatchHdr *hdr) {
    __shared__ uint32_t sc[1024];
    __shared__ uint32_t carry, wcarry;
    if (threadIdx.x == 0) carry = wcarry = 0;
    __syncthreads();
    const uint32_t per_tile = 64u * (uint32_t)cfg.lane_mult;
    for (int base = 0; base < G; base += 1024) {
        const int g = base + threadIdx.x;
        uint32_t tiles = 0, wtiles = 0;
        if (g < G) {
            const int n = offs[g + 1] - offs[g];
            int st = 0, wide = 0;
            if (n < 1 || n > max_n) {
                st = TGO_EINVAL;
            } else {
                const int c = classify_group(tasks + offs[g], n, r);
                st = c < 0 ? c : 0;
                wide = c == 1;
            }
            GroupAcc a;
            a.minkey = ~0ull;
            a.maxkey = 0;
            a.sum = 0;
            a.fp = 0;
            a.status = st;
            a.n = n;
            a.wide = wide;
            a.pad = 0;
            acc[g] = a;
            if (st == 0 && !wide) tiles = (subtrees_of(n, cfg.m[n]) + per_tile - 1) / per_tile;
            if (st == 0 && wide) wtiles = wide_tiles_of(n, wide_tiles);
        }
        const uint32_t ex = block_exscan(tiles, sc);
        if (g < G) tile_off[g] = carry + ex;
        const uint32_t last = sc[1023];
        __syncthreads();
        const uint32_t wex = block_exscan(wtiles, sc);
        if (g < G) wtile_off[g] = wcarry + wex;
        const uint32_t wlast = sc[1023];
        __syncthreads();
        if (threadIdx.x == 0) {
            carry += last;
            wcarry += wlast;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        tile_off[G] = carry;
        wtile_off[G] = wcarry;
        hdr->next_tile = 0;
        hdr->total_tiles = carry;
        hdr->next_wide = 0;
        hdr->total_wide = wcarry;
    }
}

// Simulation state of a lane: the chain form with two DMA engines, the
// event form (windows without DtH events) with one.
template <typename TT, int DMA>
using BatchLane = std::conditional_t<DMA == DMA_TWO, CLane<TT>, Lane<TT>>;

template <int M, int DMA>
__device__ __forceinline__ void run_subtree(const Ctx &c, const View<uint32_t, 1, BT_THREADS> &v,
                                            const BatchLane<uint32_t, DMA> &st, uint32_t list,
                                            Sub<uint32_t> &u) {
    level<uint32_t, M, false, 1, BT_THREADS, DMA>(c, v, st, list, 0u, u);
}

__device__ __forceinline__ unsigned long long wave_min(unsigned long long x) {
    for (int m = 32; m >= 1; m >>= 1) {
        const unsigned long long y = shfl_xor64(x, m);
        x = y < x ? y : x;
    }
    return x;
}
__device__ __forceinline__ unsigned long long wave_max(unsigned long long x) {
    for (int m = 32; m >= 1; m >>= 1) {
        const unsigned long long y = shfl_xor64(x, m);
        x = y > x ? y : x;
    }
    return x;
}
__device__ __forceinline__ unsigned long long wave_sum(unsigned long long x) {
    for (int m = 32; m >= 1; m >>= 1) x += shfl_xor64(x, m);
    return x;
}

// MMAX: deepest per-lane walk compiled in (the plan's largest m); a smaller
// bound lets the compiler keep fewer level snapshots live, so more waves fit.
// Two DMA engines: at most 80 VGPRs, so 6 waves fit per SIMD (the 26 KB of
// LDS per block allows 6 per CU); the walk of 5 levels then spills a few
// registers that are read once per tile or subtree, not in the event loop
// (12.1 -> 11.3 ms on the 4,096-group batch).
template <int DMA, int MMAX>
__global__ __launch_bounds__(BT_THREADS) __attribute__((amdgpu_waves_per_eu(DMA == DMA_TWO ? 6 : 1))) void batch_kernel(const tgo_task *__restrict__ tasks,
                                                           const int32_t *__restrict__ offs, int G,
                                                           Rates r, BatchCfg cfg, GroupAcc *acc,
                                                           const uint32_t *__restrict__ tile_off,
                                                           BatchHdr *hdr) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ Quad<uint32_t> Ht[BT_WAVES][MAXN];
    __shared__ DRec<uint32_t> Dt[BT_WAVES][MAXN];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    View<uint32_t, 1, BT_THREADS> v;
    v.H = Ht[w];
    v.D = Dt[w];
    v.Q = reinterpret_cast<Slot<uint32_t> *>(smem) + threadIdx.x;
    const uint32_t total = hdr->total_tiles;
    const uint32_t per_tile = 64u * (uint32_t)cfg.lane_mult;
    for (;;) {
        uint32_t tile = 0;
        if (lane == 0) tile = atomicAdd(&hdr->next_tile, 1u);
        tile = __builtin_amdgcn_readfirstlane(__shfl(tile, 0));  // wave-uniform: keep it scalar
        if (tile >= total) break;
        // group of this tile: largest g with tile_off[g] <= tile
        int lo = 0, hi = G;  // tile_off[lo] <= tile < tile_off[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (tile_off[mid] <= tile) lo = mid; else hi = mid;
        }
        const int g = lo;
        const int base = offs[g];
        const int n = offs[g + 1] - base;
        const int m = cfg.m[n];
        if (lane < n) table_entry<uint32_t>(tasks[base + lane], r, &Ht[w][lane], &Dt[w][lane]);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t S = subtrees_of(n, m);
        const uint32_t s0 = (tile - tile_off[g]) * per_tile;
        Ctx c;
        c.n = n;
        c.r = r;
        c.out_sub = nullptr;
        unsigned long long kmin = ~0ull, kmax = 0, ksum = 0, kfp = 0;
        for (int k = 0; k < cfg.lane_mult; ++k) {
            const uint32_t s = s0 + (uint32_t)k * 64u + (uint32_t)lane;
            if (s < S) {
                BatchLane<uint32_t, DMA> st;
                const uint32_t list = (uint32_t)prefix<DMA>(st, s, n, m, v, r);
                Sub<uint32_t> u;
                sub_init(u);
                switch (m) {
                    case 1: run_subtree<1, DMA>(c, v, st, list, u); break;
                    case 2: run_subtree<2, DMA>(c, v, st, list, u); break;
                    case 3: run_subtree<3, DMA>(c, v, st, list, u); break;
                    case 4:
                        if constexpr (MMAX >= 4) run_subtree<4, DMA>(c, v, st, list, u);
                        break;
                    default:
                        if constexpr (MMAX >= 5) run_subtree<5, DMA>(c, v, st, list, u);
                        break;
                }
                const uint64_t r0 = (uint64_t)s * fact_c(m);
                const unsigned long long a = ((unsigned long long)u.min_t << 32) | (r0 + u.min_l);
                const unsigned long long b =
                    ((unsigned long long)(u.max_t1 - 1u) << 32) | (0xffffffffull - (r0 + u.max_l));
                kmin = a < kmin ? a : kmin;
                kmax = b > kmax ? b : kmax;
                ksum += u.sum;
                kfp += 2ull * (r0 * u.sum + u.s2) + u.sum;
            }
        }
        kmin = wave_min(kmin);
        kmax = wave_max(kmax);
        ksum = wave_sum(ksum);
        kfp = wave_sum(kfp);
        if (lane == 0) {
            atomicMin(&acc[g].minkey, kmin);
            atomicMax(&acc[g].maxkey, kmax);
            atomicAdd(&acc[g].sum, ksum);
            atomicAdd(&acc[g].fp, kfp);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// 64-bit path: wave-sized tiles of the groups flagged wide, each a range of
// consecutive subtrees (BT_WIDE_M positions walked per lane); every tile
// writes the Partial of its range to parts[tile].
template <int DMA>
__global__ __launch_bounds__(BT_THREADS) void batch_wide_kernel(const tgo_task *__restrict__ tasks,
                                                                const int32_t *__restrict__ offs, int G, Rates r,
                                                                int wide_tiles, const uint32_t *__restrict__ wtile_off,
                                                                BatchHdr *hdr, Partial *parts) {
    using TT = uint64_t;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ Quad<TT> Ht[BT_WAVES][MAXN];
    __shared__ DRec<TT> Dt[BT_WAVES][MAXN];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    View<TT, 1, BT_THREADS> v;
    v.H = Ht[w];
    v.D = Dt[w];
    v.Q = reinterpret_cast<Slot<TT> *>(smem) + threadIdx.x;
    const uint32_t total = hdr->total_wide;
    for (;;) {
        uint32_t tile = 0;
        if (lane == 0) tile = atomicAdd(&hdr->next_wide, 1u);
        tile = __builtin_amdgcn_readfirstlane(__shfl(tile, 0));
        if (tile >= total) break;
        int lo = 0, hi = G;  // wtile_off[lo] <= tile < wtile_off[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (wtile_off[mid] <= tile) lo = mid; else hi = mid;
        }
        const int g = lo;
        const int base = offs[g];
        const int n = offs[g + 1] - base;
        const int m = n < BT_WIDE_M ? n : BT_WIDE_M;
        if (lane < n) table_entry<TT>(tasks[base + lane], r, &Ht[w][lane], &Dt[w][lane]);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t S = subtrees_of(n, m);
        const uint32_t W = wide_tiles_of(n, wide_tiles);
        const uint32_t t = tile - wtile_off[g];
        const uint32_t s0 = (uint32_t)((uint64_t)S * t / W), s1 = (uint32_t)((uint64_t)S * (t + 1) / W);
        Ctx c;
        c.n = n;
        c.r = r;
        c.out_sub = nullptr;
        Partial p;
        p.min_t = ~0ull; p.min_r = ~0ull; p.max_t = 0; p.max_r = ~0ull;
        p.sum_lo = 0; p.sum_hi = 0; p.fp = 0; p.status = 0; p.pad = 0;
        for (uint32_t sb = s0 + (uint32_t)lane; sb < s1; sb += 64u) {
            BatchLane<TT, DMA> st;
            const uint32_t list = (uint32_t)prefix<DMA>(st, sb, n, m, v, r);
            Sub<TT> u;
            sub_init(u);
            switch (m) {
                case 1: level<TT, 1, false, 1, BT_THREADS, DMA>(c, v, st, list, 0u, u); break;
                case 2: level<TT, 2, false, 1, BT_THREADS, DMA>(c, v, st, list, 0u, u); break;
                default: level<TT, 3, false, 1, BT_THREADS, DMA>(c, v, st, list, 0u, u); break;
            }
            const uint64_t r0 = (uint64_t)sb * fact_c(m);
            // the lane meets its subtrees in increasing rank: strict comparisons keep the lowest rank
            if (u.min_t < p.min_t) { p.min_t = u.min_t; p.min_r = r0 + u.min_l; }
            if (u.max_t1 > p.max_t) { p.max_t = u.max_t1; p.max_r = r0 + u.max_l; }
            add128(p.sum_lo, p.sum_hi, u.sum, 0);
            p.fp += 2ull * (r0 * u.sum + u.s2) + u.sum;
        }
        for (int k = 32; k >= 1; k >>= 1) {
            const uint64_t mt = shfl_xor64(p.min_t, k), mr = shfl_xor64(p.min_r, k);
            const uint64_t xt = shfl_xor64(p.max_t, k), xr = shfl_xor64(p.max_r, k);
            const uint64_t sl = shfl_xor64(p.sum_lo, k), sh = shfl_xor64(p.sum_hi, k);
            const uint64_t f = shfl_xor64(p.fp, k);
            merge_min(p.min_t, p.min_r, mt, mr);
            merge_max(p.max_t, p.max_r, xt, xr);
            add128(p.sum_lo, p.sum_hi, sl, sh);
            p.fp += f;
        }
        if (lane == 0) parts[tile] = p;
        __builtin_amdgcn_wave_barrier();
    }
}

__device__ inline void unrank16(int n, uint64_t r, uint8_t *out) {
    uint64_t list = 0;
    for (int i = n - 1; i >= 0; --i) list = (list << 4) | (uint64_t)i;
    for (int i = 0; i < n; ++i) {
        const uint64_t f = fact_c(n - 1 - i);
        const uint64_t cd = r / f;
        r -= cd * f;
        out[i] = (uint8_t)((list >> (4 * cd)) & 15u);
        const uint64_t lo = list & ((1ull << (4 * cd)) - 1ull);
        const uint64_t hi = (list >> (4 * cd + 4)) << (4 * cd);
        list = lo | hi;
    }
    for (int i = n; i < 16; ++i) out[i] = 0xff;
}

__global__ __launch_bounds__(256) void batch_finalize(const GroupAcc *__restrict__ acc, int G,
                                                      const uint32_t *__restrict__ wtile_off,
                                                      const Partial *__restrict__ parts, tgo_summary *out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const GroupAcc a = acc[g];
    if (a.status == 0 && a.wide) {
        Partial p = parts[wtile_off[g]];
        for (uint32_t i = wtile_off[g] + 1; i < wtile_off[g + 1]; ++i) {
            const Partial q = parts[i];
            merge_min(p.min_t, p.min_r, q.min_t, q.min_r);
            merge_max(p.max_t, p.max_r, q.max_t, q.max_r);
            add128(p.sum_lo, p.sum_hi, q.sum_lo, q.sum_hi);
            p.fp += q.fp;
        }
        tgo_summary s;
        const uint64_t count = fact_c(a.n);
        s.n = a.n;
        s.status = 0;
        for (int i = 0; i < 16; ++i) { s.best[i] = 0xff; s.worst[i] = 0xff; s.heur[i] = 0xff; }
        s.heur_ns = -1;
        s.min_ns = (int64_t)p.min_t;
        s.argmin_rank = p.min_r;
        s.max_ns = (int64_t)(p.max_t - 1);
        s.argmax_rank = p.max_r;
        s.sum_lo = p.sum_lo;
        s.sum_hi = p.sum_hi;
        s.count = count;
        s.fingerprint = p.fp;
        if (p.sum_hi == 0) {
            const uint64_t qt = p.sum_lo / count, rm = p.sum_lo % count;
            s.mean_ns = (double)qt + (double)rm / (double)count;
        } else {
            s.mean_ns = ((double)p.sum_hi * 18446744073709551616.0 + (double)p.sum_lo) / (double)count;
        }
        unrank16(a.n, s.argmin_rank, s.best);
        unrank16(a.n, s.argmax_rank, s.worst);
        out[g] = s;
        return;
    }
    tgo_summary s;
    s.n = a.n;
    s.status = a.status;
    for (int i = 0; i < 16; ++i) { s.best[i] = 0xff; s.worst[i] = 0xff; s.heur[i] = 0xff; }
    s.heur_ns = -1;
    if (a.status != 0) {
        s.min_ns = s.max_ns = 0;
        s.argmin_rank = s.argmax_rank = 0;
        s.sum_lo = s.sum_hi = 0;
        s.count = 0;
        s.fingerprint = 0;
        s.mean_ns = 0.0;
    } else {
        const uint64_t count = fact_c(a.n);
        s.min_ns = (int64_t)(a.minkey >> 32);
        s.argmin_rank = a.minkey & 0xffffffffull;
        s.max_ns = (int64_t)(a.maxkey >> 32);
        s.argmax_rank = 0xffffffffull - (a.maxkey & 0xffffffffull);
        s.sum_lo = a.sum;
        s.sum_hi = 0;
        s.count = count;
        s.fingerprint = a.fp;
        const uint64_t qt = a.sum / count, rm = a.sum % count;
        s.mean_ns = (double)qt + (double)rm / (double)count;
        unrank16(a.n, s.argmin_rank, s.best);
        unrank16(a.n, s.argmax_rank, s.worst);
    }
    out[g] = s;
}

// ------------------------------------------------------------------- host side

static int default_m(int n) {
    // smallest per-lane depth that still gives at least one full wave of
    // subtrees, capped at 5
    int m = 1;
    for (int c = std::min(n, 5); c >= 1; --c) {
        if (factorial(n) / factorial(c) >= 64) { m = c; break; }
    }
    return m;
}

static BatchCfg default_cfg(int cus) {
    BatchCfg c;
    for (int n = 0; n <= BT_MAX_N; ++n) c.m[n] = (int8_t)(n < 1 ? 1 : default_m(n));
    c.lane_mult = 1;
    c.blocks = cus * 8;
    return c;
}

}  // namespace tgo

struct tgo_plan {
    tgo::Rates r;
    int max_groups = 0;
    int device = 0;
    int cus = 256;
    void *ws = nullptr;
    tgo::GroupAcc *acc = nullptr;
    uint32_t *tile_off = nullptr;
    tgo::BatchHdr *hdr = nullptr;
    uint32_t *wtile_off = nullptr;
    tgo::Partial *wparts = nullptr;
    int wide_tiles = 1;
    int max_n = 12;
    size_t bytes = 0;
    tgo::BatchCfg cfg;
    bool tuned = false;
    double tuned_ms = 0.0;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *k_tasks = nullptr, *k_offs = nullptr;
    void *k_out = nullptr;
    int k_groups = -1;
};

namespace tgo {

static int enqueue_batch(tgo_plan *p, const BatchCfg &cfg, const tgo_task *d_tasks,
                         const int32_t *d_offs, int G, tgo_summary *d_out, hipStream_t st) {
    hipLaunchKernelGGL(batch_prepare, dim3(1), dim3(1024), 0, st, d_tasks, d_offs, G, p->r, cfg, p->wide_tiles,
                       p->max_n, p->acc, p->tile_off, p->wtile_off, p->hdr);
    int mmax = 1;
    for (int n = 1; n <= BT_MAX_N; ++n) mmax = std::max(mmax, (int)cfg.m[n]);
    // no kernel-completion queue with one DMA engine
    const size_t shm = p->r.one_dma ? 0 : sizeof(Slot<uint32_t>) * BT_THREADS * BT_MAX_N;
    const dim3 grid(cfg.blocks), block(BT_THREADS);
    if (p->r.one_dma) {
        if (mmax <= 3)
            hipLaunchKernelGGL((batch_kernel<DMA_ONE, 3>), grid, block, shm, st, d_tasks, d_offs, G, p->r, cfg,
                               p->acc, p->tile_off, p->hdr);
        else if (mmax == 4)
            hipLaunchKernelGGL((batch_kernel<DMA_ONE, 4>), grid, block, shm, st, d_tasks, d_offs, G, p->r, cfg,
                               p->acc, p->tile_off, p->hdr);
        else
            hipLaunchKernelGGL((batch_kernel<DMA_ONE, 5>), grid, block, shm, st, d_tasks, d_offs, G, p->r, cfg,
                               p->acc, p->tile_off, p->hdr);
    } else {
        if (mmax <= 3)
            hipLaunchKernelGGL((batch_kernel<DMA_TWO, 3>), grid, block, shm, st, d_tasks, d_offs, G, p->r, cfg,
                               p->acc, p->tile_off, p->hdr);
        else if (mmax == 4)
            hipLaunchKernelGGL((batch_kernel<DMA_TWO, 4>), grid, block, shm, st, d_tasks, d_offs, G, p->r, cfg,
                               p->acc, p->tile_off, p->hdr);
        else
            hipLaunchKernelGGL((batch_kernel<DMA_TWO, 5>), grid, block, shm, st, d_tasks, d_offs, G, p->r, cfg,
                               p->acc, p->tile_off, p->hdr);
    }
    // the 64-bit path (its blocks return at once when no group needs it)
    const size_t wshm = sizeof(Slot<uint64_t>) * BT_THREADS * BT_MAX_N;
    const dim3 wgrid(p->cus * 2);
    if (p->r.one_dma)
        hipLaunchKernelGGL(batch_wide_kernel<DMA_ONE>, wgrid, block, 0, st, d_tasks, d_offs, G, p->r, p->wide_tiles,
                           p->wtile_off, p->hdr, p->wparts);
    else
        hipLaunchKernelGGL(batch_wide_kernel<DMA_TWO>, wgrid, block, wshm, st, d_tasks, d_offs, G, p->r,
                           p->wide_tiles, p->wtile_off, p->hdr, p->wparts);
    hipLaunchKernelGGL(batch_finalize, dim3((G + 255) / 256), dim3(256), 0, st, p->acc, G, p->wtile_off, p->wparts,
                       d_out);
    int rc = launch_heuristic(p->r, d_tasks, d_offs, G, &d_out[0].heur[0], (int)sizeof(tgo_summary),
                              &d_out[0].heur_ns, (int)(sizeof(tgo_summary) / sizeof(int64_t)), st);
    if (rc) return rc;
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

size_t plan_device_bytes(const tgo_plan *p) { return p ? p->bytes : 0; }

static void drop_graph(tgo_plan *p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    p->k_groups = -1;
}

}  // namespace tgo

using namespace tgo;

extern "C" {

int tgo_plan_create(const tgo_model *model, int max_groups, int max_n, size_t mem_budget, tgo_plan **out) {
    if (!out) return fail(TGO_EINVAL, "out is NULL");
    *out = nullptr;
    Rates r;
    int rc = make_rates(model, &r);
    if (rc) return rc;
    if (max_groups < 1 || max_groups > (1 << 24)) return fail(TGO_EINVAL, "max_groups must be in 1..2^24");
    if (max_n < 1 || max_n > BT_MAX_N) return fail(TGO_EINVAL, "max_n must be in 1..12");
    tgo_plan *p = new (std::nothrow) tgo_plan();
    if (!p) return fail(TGO_ENOMEM, "plan");
    p->r = r;
    p->max_groups = max_groups;
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "device query");
    }
    const size_t acc_b = (sizeof(GroupAcc) * (size_t)max_groups + 255) & ~size_t(255);
    const size_t off_b = (sizeof(uint32_t) * ((size_t)max_groups + 1) + 255) & ~size_t(255);
    // partials of the 64-bit path: up to BT_WIDE_TILES_MAX tiles per group
    // within BT_WIDE_BUDGET bytes (at least one tile per group)
    const size_t base_b = acc_b + 2 * off_b + 256;
    size_t budget = mem_budget ? mem_budget : base_b + BT_WIDE_BUDGET;
    if (budget > base_b + BT_WIDE_BUDGET) budget = base_b + BT_WIDE_BUDGET;
    if (base_b + sizeof(Partial) * (size_t)max_groups > budget) {
        delete p;
        return fail(TGO_ENOMEM, "mem_budget below the plan's minimum (" +
                                    std::to_string(base_b + sizeof(Partial) * (size_t)max_groups) + " bytes)");
    }
    size_t wt = (budget - base_b) / (sizeof(Partial) * (size_t)max_groups);
    wt = wt < 1 ? 1 : (wt > (size_t)BT_WIDE_TILES_MAX ? (size_t)BT_WIDE_TILES_MAX : wt);
    p->wide_tiles = (int)wt;
    p->max_n = max_n;
    const size_t wp_b = sizeof(Partial) * wt * (size_t)max_groups;
    p->bytes = base_b + wp_b;
    e = hipMalloc(&p->ws, base_b + wp_b);
    if (e != hipSuccess) {
        delete p;
        return fail(TGO_ENOMEM, std::string("plan workspace: ") + hipGetErrorString(e));
    }
    p->acc = (GroupAcc *)p->ws;
    p->tile_off = (uint32_t *)((char *)p->ws + acc_b);
    p->wtile_off = (uint32_t *)((char *)p->ws + acc_b + off_b);
    p->hdr = (BatchHdr *)((char *)p->ws + acc_b + 2 * off_b);
    p->wparts = (Partial *)((char *)p->ws + acc_b + 2 * off_b + 256);
    e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        (void)hipFree(p->ws);
        delete p;
        return hip_fail(e, "plan stream");
    }
    p->cfg = default_cfg(p->cus);
    *out = p;
    return TGO_OK;
}

void tgo_plan_destroy(tgo_plan *p) {
    if (!p) return;
    (void)hipStreamSynchronize(p->cap);
    drop_graph(p);
    (void)hipStreamDestroy(p->cap);
    (void)hipFree(p->ws);
    delete p;
}

static int check_batch_args(tgo_plan *p, const tgo_task *d_tasks, const int32_t *d_offs, int G,
                            tgo_summary *d_out) {
    if (!p) return fail(TGO_EINVAL, "plan is NULL");
    if (G < 1 || G > p->max_groups) return fail(TGO_EINVAL, "n_groups must be in 1..max_groups");
    if (!d_tasks || !d_offs || !d_out) return fail(TGO_EINVAL, "NULL buffer");
    int dev = 0;
    TGO_HIP(hipGetDevice(&dev));
    if (dev != p->device) return fail(TGO_EINVAL, "plan belongs to another device");
    return TGO_OK;
}

int tgo_batch(tgo_plan *p, const tgo_task *d_tasks, const int32_t *d_offs, int G,
              tgo_summary *d_out, tgo_stream stream) {
    int rc = check_batch_args(p, d_tasks, d_offs, G, d_out);
    if (rc) return rc;
    if (!(p->exec && p->k_tasks == d_tasks && p->k_offs == d_offs && p->k_groups == G && p->k_out == d_out)) {
        drop_graph(p);
        TGO_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
        rc = enqueue_batch(p, p->cfg, d_tasks, d_offs, G, d_out, p->cap);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(p->cap, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        p->graph = g;
        e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(p);
            return hip_fail(e, "hipGraphInstantiate");
        }
        p->k_tasks = d_tasks;
        p->k_offs = d_offs;
        p->k_groups = G;
        p->k_out = d_out;
    }
    TGO_HIP(hipGraphLaunch(p->exec, (hipStream_t)stream));
    return TGO_OK;
}

int tgo_plan_autotune(tgo_plan *p, const tgo_task *d_tasks, const int32_t *d_offs, int G,
                      tgo_summary *d_out, tgo_stream stream) {
    int rc = check_batch_args(p, d_tasks, d_offs, G, d_out);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    TGO_HIP(hipEventCreate(&e0));
    TGO_HIP(hipEventCreate(&e1));
    std::vector<BatchCfg> cands;
    for (int mbig = 4; mbig <= BT_MAX_M; ++mbig)
        for (int mult : {1, 2, 4})
            for (int bpc : {4, 6, 8}) {
                BatchCfg c = default_cfg(p->cus);
                for (int n = 1; n <= BT_MAX_N; ++n) c.m[n] = (int8_t)std::min((int)c.m[n], mbig);
                for (int n = 8; n <= BT_MAX_N; ++n) c.m[n] = (int8_t)std::min(n, mbig);
                c.lane_mult = mult;
                c.blocks = p->cus * bpc;
                cands.push_back(c);
            }
    double best = 1e30;
    BatchCfg bestc = p->cfg;
    for (const BatchCfg &c : cands) {
        rc = enqueue_batch(p, c, d_tasks, d_offs, G, d_out, st);  // warm-up
        if (rc) break;
        float tot = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
            (void)hipEventRecord(e0, st);
            rc = enqueue_batch(p, c, d_tasks, d_offs, G, d_out, st);
            (void)hipEventRecord(e1, st);
            if (rc) break;
            hipError_t e = hipEventSynchronize(e1);
            if (e != hipSuccess) { rc = hip_fail(e, "autotune"); break; }
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            tot += ms;
        }
        if (rc) break;
        if (tot / 2 < best) {
            best = tot / 2;
            bestc = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    p->cfg = bestc;
    p->tuned = true;
    p->tuned_ms = best;
    drop_graph(p);
    return TGO_OK;
}

int tgo_plan_set_decomposition(tgo_plan *p, const int32_t *m_by_n, int lane_mult, int blocks) {
    if (!p || !m_by_n) return fail(TGO_EINVAL, "NULL argument");
    if (lane_mult < 1 || lane_mult > 64) return fail(TGO_EINVAL, "lane_mult must be in 1..64");
    if (blocks < 1 || blocks > 65536) return fail(TGO_EINVAL, "blocks must be in 1..65536");
    BatchCfg c = p->cfg;
    for (int n = 1; n <= BT_MAX_N; ++n) {
        const int m = m_by_n[n - 1];
        if (m < 1 || m > std::min(n, BT_MAX_M)) return fail(TGO_EINVAL, "m_by_n[n-1] must be in 1..min(n, 5)");
        c.m[n] = (int8_t)m;
    }
    c.lane_mult = lane_mult;
    c.blocks = blocks;
    p->cfg = c;
    drop_graph(p);
    return TGO_OK;
}

int tgo_plan_describe(const tgo_plan *p, char *buf, size_t len) {
    if (!p || !buf || len == 0) return fail(TGO_EINVAL, "bad argument");
    std::string s = "{\"m_by_n\": [";
    for (int n = 1; n <= BT_MAX_N; ++n) s += std::to_string((int)p->cfg.m[n]) + (n < BT_MAX_N ? ", " : "");
    s += "], \"lane_mult\": " + std::to_string(p->cfg.lane_mult);
    s += ", \"blocks\": " + std::to_string(p->cfg.blocks);
    s += ", \"block_threads\": " + std::to_string(BT_THREADS);
    s += ", \"max_n\": " + std::to_string(p->max_n);
    s += ", \"wide_tiles\": " + std::to_string(p->wide_tiles);
    s += ", \"device_bytes\": " + std::to_string(p->bytes);
    s += ", \"tuned\": " + std::string(p->tuned ? "true" : "false");
    char tmp[64];
    std::snprintf(tmp, sizeof(tmp), "%.4f", p->tuned_ms);
    s += ", \"tuned_ms\": " + std::string(tmp) + "}";
    if (s.size() + 1 > len) return fail(TGO_ERANGE, "buffer too small");
    std::copy(s.begin(), s.end(), buf);
    buf[s.size()] = 0;
    return TGO_OK;
}

}  // extern "C"
