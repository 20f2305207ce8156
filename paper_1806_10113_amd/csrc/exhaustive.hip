// Exhaustive evaluation of every launch ordering of one task group.
//
// Brute force over all n! orderings (the search that Section 1 and
// Section 5.1 rule out at runtime on a CPU), reduced to the best, worst and
// average ordering (the quantities plotted in Section 6).
//
// Each lane walks subtrees (see enum_dev.h), striding over the grid in the
// set-major order of prefix_by_set; every merge prefers the lower rank on
// equal times, so the reduction keeps the lowest rank on ties.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <mutex>
#include <type_traits>

#include "enum_dev.h"
#include "tables_dev.h"
#include "tgo_internal.h"

namespace tgo {

constexpr int EX_THREADS = 256;

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
// lane meets its subtrees in set-major order, not in rank order, so ties
// between subtrees go to the lower rank explicitly (inside a subtree the
// leaves come in rank order).  fingerprint: sum of (2r+1) T with r = r0 + l
// is 2 (r0 sum T + sum l T) + sum T.
// On the 32-bit time path every T is below 2^31 and a group has at most
// 13! < 2^33 orderings, so even the sum over all of them stays below 2^64:
// the lane keeps no carry word there (two fewer live registers).
template <typename TT>
__device__ __forceinline__ void fold(Acc<TT> &a, const Sub<TT> &u, uint64_t r0) {
    const uint64_t rmin = r0 + u.min_l, rmax = r0 + u.max_l;
    if (u.min_t < a.min_t || (u.min_t == a.min_t && rmin < a.min_r)) { a.min_t = u.min_t; a.min_r = rmin; }
    if (u.max_t1 > a.max_t1 || (u.max_t1 == a.max_t1 && rmax < a.max_r)) { a.max_t1 = u.max_t1; a.max_r = rmax; }
    const uint64_t lo = a.sum_lo + u.sum;
    if constexpr (sizeof(TT) == 8) a.sum_hi += lo < a.sum_lo ? 1ull : 0ull;
    a.sum_lo = lo;
    a.fp += 2ull * (r0 * u.sum + u.s2) + u.sum;
}

template <typename TT>
using ExView = View<TT, 1, EX_THREADS>;

// Reduce a block's lane accumulators into one Partial, returned to thread 0.
// wsum: LDS for one Partial per wave; it may alias memory the block used
// before (every thread has left its loop once the barrier below is passed).
__device__ Partial block_reduce(Partial p, Partial *wsum) {
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
    __syncthreads();
    if ((threadIdx.x & 63) == 0) wsum[w] = p;
    __syncthreads();
    Partial o = wsum[0];
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x / 64); ++i) {
            merge_min(o.min_t, o.min_r, wsum[i].min_t, wsum[i].min_r);
            merge_max(o.max_t, o.max_r, wsum[i].max_t, wsum[i].max_r);
            add128(o.sum_lo, o.sum_hi, wsum[i].sum_lo, wsum[i].sum_hi);
            o.fp += wsum[i].fp;
        }
        o.status = 0;
        o.pad = 0;
    }
    return o;
}

// Whole-group accumulator of the 32-bit time path, folded into by every
// block with 64-bit atomics.  There T < 2^31 and a rank < 13! < 2^33, so
// (T << 33) | rank orders by time and then by rank: the smallest key is the
// best ordering with the lowest rank, and with the rank complemented the
// largest key is the worst ordering with the lowest rank.  The sum over all
// orderings stays below 13! * 2^31 < 2^64; the fingerprint wraps.
struct ExAcc {
    unsigned long long minkey, maxkey, sum, fp;
};
constexpr uint64_t EX_RANK_MASK = (1ull << 33) - 1;


// Dynamic LDS of the exhaustive kernel: the task tables (n entries each),
// then the per-lane kernel-completion queue, n - 1 slots (the last position's
// slot is never read; none with one DMA engine).  The block reduction reuses
// the queue's memory at the end.
template <typename TT>
__host__ __device__ constexpr size_t ex_tables_bytes(int n) {
    return (size_t)n * (sizeof(Quad<TT>) + sizeof(DRec<TT>));
}
template <typename TT>
__host__ __device__ constexpr int ex_queue_slots(int n, bool one_dma) {
    return one_dma ? 0 : (n > 1 ? n - 1 : 1);
}
template <typename TT>
inline size_t ex_shm_bytes(int n, bool one_dma) {
    const size_t q = sizeof(Slot<TT>) * EX_THREADS * (size_t)ex_queue_slots<TT>(n, one_dma);
    const size_t red = sizeof(Partial) * (EX_THREADS / 64);
    return ex_tables_bytes<TT>(n) + (q > red ? q : red);
}

// 32-bit time path: at most 72 VGPRs so that 7 waves fit per SIMD (with the
// n - 1 slot queue, 7 blocks also fit in LDS at n = 12).
template <typename TT>
constexpr int ex_min_waves() { return sizeof(TT) == 4 ? 7 : 1; }

// The group's time path, decided once before the enumeration: 0 = 32-bit,
// 1 = 64-bit, or a negative error code (classify_group).
__global__ void exhaustive_classify(const tgo_task *__restrict__ tasks, int n, Rates r, int *mode,
                                    ExAcc *acc) {
    if (threadIdx.x == 0) {
        *mode = classify_group(tasks, n, r);
        acc->minkey = ~0ull;
        acc->maxkey = 0;
        acc->sum = 0;
        acc->fp = 0;
    }
}

// MODE: 0 = 32-bit time path, 1 = 64-bit.  Both instantiations are launched;
// every block of the one that does not match the group's path (or of both,
// on an error) returns after reading one word.  DMA is the launch scheme
// (DMA_TWO or DMA_ONE, fixed per instantiation).
template <typename TT, int M, bool STORE, int DMA>
__global__ __launch_bounds__(EX_THREADS) __attribute__((amdgpu_waves_per_eu(ex_min_waves<TT>())))
void exhaustive_kernel(const tgo_task *__restrict__ tasks, int n, Rates r, uint32_t n_sub, int64_t *out,
                       Partial *partials, ExAcc *acc, const int *__restrict__ modep) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int MODE = sizeof(TT) == 4 ? 0 : 1;
    if (*modep != MODE) return;
    Quad<TT> *Ht = reinterpret_cast<Quad<TT> *>(smem);
    DRec<TT> *Dt = reinterpret_cast<DRec<TT> *>(smem + (size_t)n * sizeof(Quad<TT>));
    unsigned char *qbase = smem + ex_tables_bytes<TT>(n);
    if ((int)threadIdx.x < n) table_entry<TT>(tasks[threadIdx.x], r, &Ht[threadIdx.x], &Dt[threadIdx.x]);
    __syncthreads();

    ExView<TT> v;
    v.H = Ht;
    v.D = Dt;
    v.Q = reinterpret_cast<Slot<TT> *>(qbase) + threadIdx.x;
    Ctx c;
    c.n = n;
    c.r = r;
    c.out_sub = nullptr;

    Acc<TT> a;
    acc_init(a);
    const uint32_t stride = gridDim.x * blockDim.x;
    // two DMA engines: the chain form; one engine: windows without DtH events
    using LaneT = std::conditional_t<DMA == DMA_TWO, CLane<TT>, Lane<TT>>;
    for (uint32_t s = blockIdx.x * blockDim.x + threadIdx.x; s < n_sub; s += stride) {
        LaneT st;
        uint32_t lex;
        const uint64_t list = prefix_by_set<DMA>(st, s, n, M, v, r, &lex);
        const uint64_t r0 = (uint64_t)lex * factorial(M);
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
    const Partial o = block_reduce(p, reinterpret_cast<Partial *>(qbase));
    if (threadIdx.x == 0) {
        if constexpr (sizeof(TT) == 4) {
            // every block owns at least one subtree, so o holds an ordering
            atomicMin(&acc->minkey, (unsigned long long)((o.min_t << 33) | o.min_r));
            atomicMax(&acc->maxkey, (unsigned long long)(((o.max_t - 1) << 33) | (EX_RANK_MASK - o.max_r)));
            atomicAdd(&acc->sum, (unsigned long long)o.sum_lo);
            atomicAdd(&acc->fp, (unsigned long long)o.fp);
        } else {
            partials[blockIdx.x] = o;
        }
    }
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

constexpr int EX_FIN_THREADS = 1024;

__global__ __launch_bounds__(EX_FIN_THREADS) void exhaustive_finalize(const Partial *__restrict__ parts,
                                                                      int nparts, int n, uint64_t count,
                                                                      const ExAcc *__restrict__ acc,
                                                                      const int *__restrict__ modep,
                                                                      tgo_summary *out) {
    __shared__ Partial red[EX_FIN_THREADS / 64];
    const int mode = *modep;
    const int status = mode < 0 ? mode : 0;
    Partial p;
    p.min_t = ~0ull; p.min_r = ~0ull; p.max_t = 0; p.max_r = ~0ull;
    p.sum_lo = 0; p.sum_hi = 0; p.fp = 0; p.status = 0; p.pad = 0;
    auto take = [&p](const Partial &q) {
        merge_min(p.min_t, p.min_r, q.min_t, q.min_r);
        merge_max(p.max_t, p.max_r, q.max_t, q.max_r);
        add128(p.sum_lo, p.sum_hi, q.sum_lo, q.sum_hi);
        p.fp += q.fp;
    };
    if (mode == 1) {
        // four partials in flight per thread: the loads, not the merges, set the time
        const int b = (int)blockDim.x;
        int i = (int)threadIdx.x;
        for (; i + 3 * b < nparts; i += 4 * b) {
            const Partial q0 = parts[i], q1 = parts[i + b], q2 = parts[i + 2 * b], q3 = parts[i + 3 * b];
            take(q0);
            take(q1);
            take(q2);
            take(q3);
        }
        for (; i < nparts; i += b) take(parts[i]);
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
    if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = p;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x / 64); ++i) {
            const Partial &q = red[i];
            merge_min(red[0].min_t, red[0].min_r, q.min_t, q.min_r);
            merge_max(red[0].max_t, red[0].max_r, q.max_t, q.max_r);
            add128(red[0].sum_lo, red[0].sum_hi, q.sum_lo, q.sum_hi);
            red[0].fp += q.fp;
        }
        if (mode == 0) {
            red[0].min_t = acc->minkey >> 33;
            red[0].min_r = acc->minkey & EX_RANK_MASK;
            red[0].max_t = (acc->maxkey >> 33) + 1;
            red[0].max_r = EX_RANK_MASK - (acc->maxkey & EX_RANK_MASK);
            red[0].sum_lo = acc->sum;
            red[0].sum_hi = 0;
            red[0].fp = acc->fp;
        }
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
    // two engines: with the three innermost levels unrolled, 5 levels beat 4
    // at n = 12 on MI355X (1.81 vs 1.99 ms: fewer windows per ordering, 2.77
    // vs 3.0).  One engine: a window is a handful of operations, so the
    // per-subtree prefix decode is worth amortising over 6 levels.
    const int top = one_dma ? 6 : 5;
    int m = 1;
    for (int c = top; c >= 1; --c) {
        if (c > n) continue;
        const uint64_t sub = factorial(n) / factorial(c);
        if (sub >= 32768 || c == 1) { m = c; break; }
    }
    if (n <= 5) m = n < 1 ? 1 : n;
    return m;
}

// Blocks that fit on the device at once for a kernel and its dynamic LDS.
static uint32_t resident_blocks(const void *kern, size_t shm) {
    struct Entry { int dev; const void *k; size_t shm; uint32_t blocks; };
    static std::mutex mu;
    static Entry cache[64];
    static int used = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    std::lock_guard<std::mutex> lk(mu);
    for (int i = 0; i < used; ++i)
        if (cache[i].dev == dev && cache[i].k == kern && cache[i].shm == shm) return cache[i].blocks;
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, EX_THREADS, shm) != hipSuccess || per_cu <= 0)
        per_cu = 1;
    const uint32_t b = (uint32_t)cus * (uint32_t)per_cu;
    if (used < 64) cache[used++] = Entry{dev, kern, shm, b};
    return b;
}

// Blocks per launch, in units of the blocks the 32-bit kernel keeps resident
// at once.  A subtree's cost varies with its DtH events, so blocks finish at
// different times: one resident round leaves SIMDs idle at the end, many
// short blocks let the dispatcher fill them.  Measured at N = 12 on MI355X
// with 6 waves per SIMD (1,536 resident blocks) and block partials: 8 rounds
// gave 3.06-3.11 ms per launch against 3.82 ms for one round and 3.30 ms for
// 20 subtrees per lane.  With 7 waves (1,792 resident blocks) and the
// accumulator atomics: 6 / 8 / 10 / 12 / 14 / 16 / 20 rounds took 2.85-2.87 /
// 2.80 / 2.81-2.82 / 2.78-2.80 / 2.80-2.82 / 2.77-2.78 / 2.83 ms, and grids
// that are not a multiple of the resident count were slower; 12 rounds,
// 21,504 blocks.
constexpr uint32_t EX_ROUNDS = 12;

// Launch the 32-bit and 64-bit instantiations (the one that does not match
// the group returns at once) and the finalize.  The grid is sized from the
// 32-bit kernel (the fast path), capped at one subtree per lane;
// TGO_EXHAUSTIVE_BLOCKS overrides it for tuning experiments.
// Scratch of one call: caller-provided (ptr, bytes), or the library's
// per-(device, stream) workspace when ptr is NULL.
struct ExScratch {
    void *ptr = nullptr;
    size_t bytes = 0;
};

template <int M, bool STORE, int DMA>
static int launch_pair(size_t shm32, size_t shm64, hipStream_t st, const tgo_task *t, int n,
                       const Rates &r, uint32_t n_sub, int64_t *out, tgo_summary *d_out, ExScratch ws) {
    const void *k32 = reinterpret_cast<const void *>(&exhaustive_kernel<uint32_t, M, STORE, DMA>);
    const uint64_t want = ((uint64_t)n_sub + EX_THREADS - 1) / EX_THREADS;
    uint32_t blocks = resident_blocks(k32, shm32);
    blocks = blocks == 0 ? 8192u : blocks * EX_ROUNDS;
    if (const char *e = std::getenv("TGO_EXHAUSTIVE_BLOCKS")) {
        const long v = std::atol(e);
        if (v >= 1 && v <= (1l << 20)) blocks = (uint32_t)v;
    }
    if ((uint64_t)blocks > want) blocks = (uint32_t)want;
    // workspace: the block partials (64-bit path), the 32-bit path's
    // accumulator, then the group's time path.  A fixed scratch bounds the
    // grid instead (any grid gives the same result: lanes stride over the
    // subtrees).
    const size_t fixed = sizeof(ExAcc) + sizeof(Partial);
    Partial *parts = nullptr;
    if (ws.ptr) {
        if (ws.bytes < fixed + sizeof(Partial))
            return fail(TGO_ENOMEM, "scratch too small for one block");
        const size_t fit = (ws.bytes - fixed) / sizeof(Partial);
        if ((size_t)blocks > fit) blocks = (uint32_t)fit;
        parts = reinterpret_cast<Partial *>(ws.ptr);
    } else {
        int rc = workspace(sizeof(Partial) * (blocks + 1) + sizeof(ExAcc), (void **)&parts, st);
        if (rc) return rc;
    }
    ExAcc *acc = reinterpret_cast<ExAcc *>(parts + blocks);
    int *mode = reinterpret_cast<int *>(acc + 1);
    hipLaunchKernelGGL(exhaustive_classify, dim3(1), dim3(64), 0, st, t, n, r, mode, acc);
    const dim3 grid(blocks);
    hipLaunchKernelGGL((exhaustive_kernel<uint32_t, M, STORE, DMA>), grid, dim3(EX_THREADS), shm32, st, t, n, r,
                       n_sub, out, parts, acc, mode);
    hipLaunchKernelGGL((exhaustive_kernel<uint64_t, M, STORE, DMA>), grid, dim3(EX_THREADS), shm64, st, t, n, r,
                       n_sub, out, parts, acc, mode);
    TGO_HIP(hipGetLastError());
    hipLaunchKernelGGL(exhaustive_finalize, dim3(1), dim3(EX_FIN_THREADS), 0, st, parts, (int)blocks, n,
                       factorial(n), acc, mode, d_out);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

template <bool STORE, int DMA>
static int launch_m(int m, size_t shm32, size_t shm64, hipStream_t st, const tgo_task *t, int n,
                    const Rates &r, uint32_t n_sub, int64_t *out, tgo_summary *d_out, ExScratch ws) {
    switch (m) {
        case 1: return launch_pair<1, STORE, DMA>(shm32, shm64, st, t, n, r, n_sub, out, d_out, ws);
        case 2: return launch_pair<2, STORE, DMA>(shm32, shm64, st, t, n, r, n_sub, out, d_out, ws);
        case 3: return launch_pair<3, STORE, DMA>(shm32, shm64, st, t, n, r, n_sub, out, d_out, ws);
        case 4: return launch_pair<4, STORE, DMA>(shm32, shm64, st, t, n, r, n_sub, out, d_out, ws);
        case 5: return launch_pair<5, STORE, DMA>(shm32, shm64, st, t, n, r, n_sub, out, d_out, ws);
        default:
            if constexpr (DMA == DMA_ONE)
                return launch_pair<6, STORE, DMA>(shm32, shm64, st, t, n, r, n_sub, out, d_out, ws);
            else
                return launch_pair<5, STORE, DMA>(shm32, shm64, st, t, n, r, n_sub, out, d_out, ws);
    }
}

static int launch_exhaustive_ws(const Rates &r, const tgo_task *d_tasks, int n, int64_t *d_per_order,
                                tgo_summary *d_out, hipStream_t st, ExScratch ws) {
    const bool one = r.one_dma != 0;
    const int m = choose_m(n, one);
    const uint64_t n_sub64 = factorial(n) / factorial(m);
    if (n_sub64 >= (1ull << 32)) return fail(TGO_EINVAL, "group too large to enumerate");
    const uint32_t n_sub = (uint32_t)n_sub64;
    const size_t shm32 = ex_shm_bytes<uint32_t>(n, one);
    const size_t shm64 = ex_shm_bytes<uint64_t>(n, one);
    if (one) {
        return d_per_order
                   ? launch_m<true, DMA_ONE>(m, shm32, shm64, st, d_tasks, n, r, n_sub, d_per_order, d_out, ws)
                   : launch_m<false, DMA_ONE>(m, shm32, shm64, st, d_tasks, n, r, n_sub, nullptr, d_out, ws);
    }
    return d_per_order
               ? launch_m<true, DMA_TWO>(m, shm32, shm64, st, d_tasks, n, r, n_sub, d_per_order, d_out, ws)
               : launch_m<false, DMA_TWO>(m, shm32, shm64, st, d_tasks, n, r, n_sub, nullptr, d_out, ws);
}

int launch_exhaustive(const Rates &r, const tgo_task *d_tasks, int n, int64_t *d_per_order,
                      tgo_summary *d_out, hipStream_t st) {
    return launch_exhaustive_ws(r, d_tasks, n, d_per_order, d_out, st, ExScratch{});
}

// Fixed scratch of the allocation-free enumeration: block partials, the
// 32-bit accumulator and the time-path word of one call.  Each device holds
// its own copy for the life of the process.  On the host the array's name is
// only a stand-in: its device address comes from hipGetSymbolAddress, taken
// once per device with that device current.
static __device__ __align__(256) unsigned char scratch[TGO_NOALLOC_SCRATCH_BYTES];

constexpr int EX_MAX_DEVICES = 64;

static int scratch_address(void **ptr) {
    static std::mutex mu;
    static void *addr[EX_MAX_DEVICES] = {};
    int dev = 0;
    TGO_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= EX_MAX_DEVICES) return fail(TGO_EDEVICE, "device index above 63");
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(TGO_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return TGO_OK;
}

int launch_exhaustive_noalloc(const Rates &r, const tgo_task *d_tasks, int n, int64_t *d_per_order,
                              tgo_summary *d_out, hipStream_t st) {
    ExScratch ws;
    int rc = scratch_address(&ws.ptr);
    if (rc) return rc;
    ws.bytes = TGO_NOALLOC_SCRATCH_BYTES;
    return launch_exhaustive_ws(r, d_tasks, n, d_per_order, d_out, st, ws);
}

}  // namespace tgo
