// Multi-round task groups (Section 6.2): T workers, each offloading R
// dependent tasks; a worker hands over its next task only when the previous
// one has completely finished (its DtH has ended).
//
// Task (w, r) is index w * R + r of the task table.  Two setups:
//   NoReorder: all T*R tasks queued at t = 0, round by round, round r in a
//     worker order pi_r; every (pi_0, ..., pi_{R-1}) is an ordering, ranked
//     with pi_0 most significant and each pi_r lexicographic.  The HtD of
//     (w, r) waits for the DtH of (w, r - 1), and the in-order queue behind it
//     waits too.  One lane per ordering, reduced like the single-group
//     enumeration.
//   Heuristic: a proxy takes every task waiting in the shared buffer as a
//     task group, orders it with Algorithm 1 and queues it; it looks at the
//     buffer again when the HtD of the group's last task starts (HtDs handed
//     to the engine just in time), or at the next arrival if the buffer is
//     empty then.  One lane per experiment.
//
// The window formulation of the single-group kernels assumes an HtD engine
// busy without gaps; dependencies break that, so this path steps events
// directly: at each instant every finished command retires, then every ready
// queue head starts, then the proxy looks, until nothing changes; time then
// advances to the earliest completion estimate (remaining transfer work is
// exact in 1/q solo-ns, estimates rounded up to whole ns, overlapped HtD and
// DtH at p_htd/q and p_dth/q).  Launch schemes of Section 3.2: two DMA
// engines = three FIFO queues in submission order; one DMA engine = one
// transfer queue holding, per submitted group, its HtDs then its DtHs.
#include <hip/hip_runtime.h>

#include "enum_dev.h"
#include "heur_dev.h"
#include "tables_dev.h"
#include "tgo_internal.h"

namespace tgo {

constexpr int RD_THREADS = 256;
constexpr int RD_MAX_BLOCKS = 4096;

__device__ __forceinline__ uint32_t nib(uint64_t v, int i) { return (uint32_t)(v >> (4 * i)) & 15u; }
__device__ __forceinline__ uint64_t set_nib(uint64_t v, int i, uint32_t x) {
    return (v & ~(15ull << (4 * i))) | ((uint64_t)x << (4 * i));
}

struct Dur {
    int64_t h, k, d;
};

// Event-stepping state of one simulation.
struct RSim {
    int64_t t;
    uint64_t seq;    // nibble j: task at submitted position j
    uint64_t posof;  // nibble x: position of task x (once submitted)
    uint32_t gend;   // bit j: position j closes a submitted group
    int nsub;        // positions submitted so far
    // completed commands: positions < *_done have finished (every queue is
    // served in position order)
    int h_done, k_done, d_done;
    // two engines: next position to start per queue; one engine: the
    // transfer queue's current group [xb, xe) and offset xo in [0, 2 (xe - xb))
    int hc, kc, dc;
    int xb, xe, xo;
    bool hrun, krun, drun;  // one engine: hrun/drun say which transfer runs
    int hpos, dpos;         // position of the running transfer(s)
    int64_t uh, ud, kend;   // remaining transfer work (1/q ns), kernel end
};

__device__ __forceinline__ void rsim_init(RSim &s) {
    s.t = 0;
    s.seq = 0;
    s.posof = 0;
    s.gend = 0;
    s.nsub = 0;
    s.h_done = s.k_done = s.d_done = 0;
    s.hc = s.kc = s.dc = 0;
    s.xb = s.xe = s.xo = 0;
    s.hrun = s.krun = s.drun = false;
    s.hpos = s.dpos = 0;
    s.uh = s.ud = s.kend = 0;
}

// Append a group of tasks (in launch order) at the current instant.
__device__ __forceinline__ void rsim_submit(RSim &s, const uint8_t *order, int g) {
    for (int i = 0; i < g; ++i) {
        const int j = s.nsub + i;
        s.seq = set_nib(s.seq, j, order[i]);
        s.posof = set_nib(s.posof, order[i], (uint32_t)j);
    }
    s.nsub += g;
    s.gend |= 1u << (s.nsub - 1);
}

__device__ __forceinline__ uint64_t ceil_div_u64(uint64_t u, uint64_t p) { return (u + p - 1) / p; }

// The HtD at position j may start once the DtH of the same worker's previous
// task has ended.
__device__ __forceinline__ bool dep_ok(const RSim &s, int j, int R) {
    const uint32_t x = nib(s.seq, j);
    if (x % (uint32_t)R == 0) return true;
    return (uint32_t)s.d_done > nib(s.posof, x - 1);
}

// One pass at the current instant: retire finished commands, then start every
// ready head.  Returns whether anything changed; finished DtHs are reported
// in *arrived (bit x: the worker's next task x became available), the start
// of the HtD at position trig in *trig_started.
template <bool ONE>
__device__ __forceinline__ bool rsim_pass(RSim &s, const Dur *tab, int R, const Rates &r, int trig,
                                          uint32_t *arrived, bool *trig_started) {
    bool changed = false;
    const int64_t q = int64_t(1) << r.q_log2;
    // retire
    if (s.hrun && s.uh == 0) { s.hrun = false; ++s.h_done; changed = true; }
    if (s.krun && s.kend == s.t) { s.krun = false; ++s.k_done; changed = true; }
    if (s.drun && s.ud == 0) {
        s.drun = false;
        ++s.d_done;
        changed = true;
        const uint32_t x = nib(s.seq, s.dpos);
        if (x % (uint32_t)R + 1 < (uint32_t)R) *arrived |= 1u << (x + 1);
    }
    // start ready heads
    if constexpr (!ONE) {
        if (!s.hrun && s.hc < s.nsub && dep_ok(s, s.hc, R)) {
            s.hpos = s.hc++;
            s.uh = q * tab[nib(s.seq, s.hpos)].h;
            s.hrun = true;
            changed = true;
            if (s.hpos == trig) *trig_started = true;
        }
        if (!s.drun && s.dc < s.nsub && s.dc < s.k_done) {
            s.dpos = s.dc++;
            s.ud = q * tab[nib(s.seq, s.dpos)].d;
            s.drun = true;
            changed = true;
        }
    } else {
        if (!s.hrun && !s.drun) {
            if (s.xo == 2 * (s.xe - s.xb) && s.xe < s.nsub) {
                // next submitted group: [xe, end of that group)
                s.xb = s.xe;
                const uint32_t rest = s.gend >> s.xb;
                s.xe = s.xb + __ffs(rest);
                s.xo = 0;
            }
            const int len = s.xe - s.xb;
            if (s.xo < len) {
                const int j = s.xb + s.xo;
                if (dep_ok(s, j, R)) {
                    s.hpos = j;
                    s.uh = q * tab[nib(s.seq, j)].h;
                    s.hrun = true;
                    ++s.xo;
                    changed = true;
                    if (j == trig) *trig_started = true;
                }
            } else if (s.xo < 2 * len) {
                const int j = s.xb + s.xo - len;
                if (s.k_done > j) {
                    s.dpos = j;
                    s.ud = q * tab[nib(s.seq, j)].d;
                    s.drun = true;
                    ++s.xo;
                    changed = true;
                }
            }
        }
    }
    if (!s.krun && s.kc < s.nsub && s.kc < s.h_done) {
        const int j = s.kc++;
        s.kend = s.t + tab[nib(s.seq, j)].k;
        s.krun = true;
        changed = true;
    }
    return changed;
}

// Advance to the earliest completion estimate.  Returns false when nothing runs.
template <bool ONE>
__device__ __forceinline__ bool rsim_advance(RSim &s, const Rates &r) {
    if (!s.hrun && !s.krun && !s.drun) return false;
    const uint64_t q = 1ull << r.q_log2;
    const bool both = !ONE && s.hrun && s.drun;
    const uint64_t rh = both ? r.p_h : q, rd = both ? r.p_d : q;
    const int64_t INF = INT64_MAX;
    const int64_t eh = s.hrun ? (int64_t)ceil_div_u64((uint64_t)s.uh, rh) : INF;
    const int64_t ed = s.drun ? (int64_t)ceil_div_u64((uint64_t)s.ud, rd) : INF;
    const int64_t ek = s.krun ? s.kend - s.t : INF;
    int64_t dt = eh < ed ? eh : ed;
    dt = ek < dt ? ek : dt;
    if (s.hrun) s.uh = eh == dt ? 0 : s.uh - (int64_t)rh * dt;
    if (s.drun) s.ud = ed == dt ? 0 : s.ud - (int64_t)rd * dt;
    s.t += dt;
    return true;
}

// NoReorder: simulate one fully queued launch sequence (groups are rounds).
template <bool ONE>
__device__ int64_t rsim_noreorder(RSim &s, const Dur *tab, int R, const Rates &r) {
    for (;;) {
        uint32_t arrived = 0;
        bool trig = false;
        while (rsim_pass<ONE>(s, tab, R, r, -1, &arrived, &trig)) {}
        if (!rsim_advance<ONE>(s, r)) break;
    }
    return s.t;
}

__device__ __forceinline__ bool valid_task(const tgo_task &t) {
    return t.htd_ns >= 0 && t.kern_ns >= 0 && t.dth_ns >= 0 && t.htd_ns < MAX_DURATION &&
           t.kern_ns < MAX_DURATION && t.dth_ns < MAX_DURATION;
}

// Per-lane accumulators over the ranks the lane owns (in increasing order).
struct RAcc {
    uint64_t min_t, min_r, max_t, max_r, sum_lo, sum_hi, fp;
};

template <bool ONE, bool STORE>
__global__ __launch_bounds__(RD_THREADS) void rounds_kernel(const tgo_task *__restrict__ tasks, int T,
                                                            int R, Rates r, uint32_t count,
                                                            uint32_t tfact, int64_t *out,
                                                            Partial *partials) {
    __shared__ Dur tab[MAXN];
    __shared__ int bad;
    const int n = T * R;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    if ((int)threadIdx.x < n) {
        const tgo_task t = tasks[threadIdx.x];
        if (!valid_task(t)) atomicOr(&bad, 1);
        tab[threadIdx.x] = Dur{t.htd_ns, t.kern_ns, t.dth_ns};
    }
    __syncthreads();
    if (bad) {
        if (threadIdx.x == 0) {
            Partial p = {};
            p.status = TGO_ERANGE;
            partials[blockIdx.x] = p;
        }
        return;
    }
    RAcc a;
    a.min_t = ~0ull; a.min_r = ~0ull; a.max_t = 0; a.max_r = ~0ull;
    a.sum_lo = 0; a.sum_hi = 0; a.fp = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t rk64 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; rk64 < count; rk64 += stride) {
        const uint32_t rk = (uint32_t)rk64;
        // rank -> one worker order per round (pi_0 most significant)
        uint8_t order[MAXN];
        uint32_t rem = rk;
        for (int rr = R - 1; rr >= 0; --rr) {
            uint32_t d = rem % tfact;
            rem /= tfact;
            uint64_t list = 0;  // remaining workers, ascending, one per nibble (T <= 12)
            for (int i = T - 1; i >= 0; --i) list = (list << 4) | (uint64_t)i;
            uint32_t f = tfact;
            for (int i = 0; i < T; ++i) {
                f /= (uint32_t)(T - i);
                const uint32_t c = d / f;
                d -= c * f;
                const uint32_t w = (uint32_t)(list >> (4 * c)) & 15u;
                const uint64_t lo = list & ((1ull << (4 * c)) - 1ull);
                const uint64_t hi = (list >> (4 * c + 4)) << (4 * c);
                list = lo | hi;
                order[rr * T + i] = (uint8_t)(w * R + rr);
            }
        }
        RSim s;
        rsim_init(s);
        for (int rr = 0; rr < R; ++rr) rsim_submit(s, order + rr * T, T);
        const uint64_t Tt = (uint64_t)rsim_noreorder<ONE>(s, tab, R, r);
        if constexpr (STORE) out[rk] = (int64_t)Tt;
        if (Tt < a.min_t) { a.min_t = Tt; a.min_r = rk; }
        if (Tt + 1 > a.max_t) { a.max_t = Tt + 1; a.max_r = rk; }
        add128(a.sum_lo, a.sum_hi, Tt, 0);
        a.fp += (2ull * rk + 1ull) * Tt;
    }
    Partial p;
    p.min_t = a.min_t; p.min_r = a.min_r; p.max_t = a.max_t; p.max_r = a.max_r;
    p.sum_lo = a.sum_lo; p.sum_hi = a.sum_hi; p.fp = a.fp; p.status = 0; p.pad = 0;
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
    __shared__ Partial wsum[RD_THREADS / 64];
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x / 64] = p;
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial o = wsum[0];
        for (int i = 1; i < RD_THREADS / 64; ++i) {
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

// Launch sequence (task per position) of NoReorder rank rk.
__device__ inline void rounds_unrank(int T, int R, uint64_t rk, uint64_t tfact, uint8_t *out) {
    for (int rr = R - 1; rr >= 0; --rr) {
        uint64_t d = rk % tfact;
        rk /= tfact;
        uint64_t list = 0;
        for (int i = T - 1; i >= 0; --i) list = (list << 4) | (uint64_t)i;
        uint64_t f = tfact;
        for (int i = 0; i < T; ++i) {
            f /= (uint64_t)(T - i);
            const uint64_t c = d / f;
            d -= c * f;
            const uint64_t w = (list >> (4 * c)) & 15u;
            const uint64_t lo = list & ((1ull << (4 * c)) - 1ull);
            const uint64_t hi = (list >> (4 * c + 4)) << (4 * c);
            list = lo | hi;
            out[rr * T + i] = (uint8_t)(w * R + rr);
        }
    }
    for (int i = T * R; i < 16; ++i) out[i] = 0xff;
}

__global__ __launch_bounds__(256) void rounds_finalize(const Partial *__restrict__ parts, int nparts,
                                                       int T, int R, uint64_t count, uint64_t tfact,
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
            const Partial q = red[threadIdx.x + s];
            Partial &o = red[threadIdx.x];
            merge_min(o.min_t, o.min_r, q.min_t, q.min_r);
            merge_max(o.max_t, o.max_r, q.max_t, q.max_r);
            add128(o.sum_lo, o.sum_hi, q.sum_lo, q.sum_hi);
            o.fp += q.fp;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const Partial &o = red[0];
        tgo_summary s;
        s.n = T * R;
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
            if (o.sum_hi == 0) {
                const uint64_t qt = o.sum_lo / count, rm = o.sum_lo % count;
                s.mean_ns = (double)qt + (double)rm / (double)count;
            } else {
                s.mean_ns = ((double)o.sum_hi * 18446744073709551616.0 + (double)o.sum_lo) / (double)count;
            }
            rounds_unrank(T, R, o.min_r, tfact, s.best);
            rounds_unrank(T, R, o.max_r, tfact, s.worst);
        }
        *out = s;
    }
}

// Heuristic setup: one thread drives the proxy and the device model.
template <bool ONE>
__global__ __launch_bounds__(64) void rounds_heuristic_kernel(const tgo_task *__restrict__ tasks, int T,
                                                              int R, Rates r, tgo_summary *out,
                                                              uint16_t *groups) {
    __shared__ Dur tab[MAXN];
    __shared__ Quad<uint64_t> Ht[MAXN];
    __shared__ DRec<uint64_t> Dt[MAXN];
    __shared__ Slot<uint64_t> Qs[MAXN];
    if (threadIdx.x != 0) return;
    const int n = T * R;
    for (int x = 0; x < n; ++x) {
        const tgo_task t = tasks[x];
        if (!valid_task(t)) {
            out->heur_ns = TGO_ERANGE;
            if (groups) *groups = 0;
            return;
        }
        tab[x] = Dur{t.htd_ns, t.kern_ns, t.dth_ns};
    }
    View<uint64_t, 1, 1> v;
    v.H = Ht;
    v.D = Dt;
    v.Q = Qs;
    RSim s;
    rsim_init(s);
    uint32_t buffer = 0;
    for (int w = 0; w < T; ++w) buffer |= 1u << (w * R);
    bool armed = true;
    int trig = -1;
    for (;;) {
        bool changed = true;
        while (changed) {
            uint32_t arrived = 0;
            bool started = false;
            changed = rsim_pass<ONE>(s, tab, R, r, trig, &arrived, &started);
            buffer |= arrived;
            armed = armed || started;
            if (armed && buffer) {
                // the group: waiting tasks in ascending index, ordered by Algorithm 1
                uint8_t mem[MAXN];
                int g = 0;
                for (int x = 0; x < n; ++x)
                    if ((buffer >> x) & 1u) mem[g++] = (uint8_t)x;
                for (int i = 0; i < g; ++i) table_entry<uint64_t>(tasks[mem[i]], r, &Ht[i], &Dt[i]);
                uint8_t ord[MAXN];
                heuristic_order(g, v, r, ord);
                uint8_t launch[MAXN];
                for (int i = 0; i < g; ++i) launch[i] = mem[ord[i]];
                rsim_submit(s, launch, g);
                trig = s.nsub - 1;
                buffer = 0;
                armed = false;
                changed = true;
            }
        }
        if (!rsim_advance<ONE>(s, r)) break;
    }
    uint8_t seq[16];
    for (int j = 0; j < 16; ++j) seq[j] = j < n ? (uint8_t)nib(s.seq, j) : (uint8_t)0xff;
    for (int j = 0; j < 16; ++j) out->heur[j] = seq[j];
    out->heur_ns = s.t;
    if (groups) *groups = (uint16_t)s.gend;
}

int launch_summary_finalize(const Partial *d_parts, int nparts, int T, int R, uint64_t count, uint64_t tfact,
                            tgo_summary *d_out, hipStream_t st) {
    hipLaunchKernelGGL(rounds_finalize, dim3(1), dim3(256), 0, st, d_parts, nparts, T, R, count, tfact, d_out);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

int launch_rounds(const Rates &r, const tgo_task *d_tasks, int T, int R, int64_t *d_per_order,
                  tgo_summary *d_out, uint16_t *d_groups, hipStream_t st) {
    const uint64_t tf = factorial(T);
    uint64_t count = 1;
    for (int i = 0; i < R; ++i) count *= tf;
    const uint64_t want = (count + RD_THREADS - 1) / RD_THREADS;
    const uint32_t blocks = (uint32_t)(want < RD_MAX_BLOCKS ? want : RD_MAX_BLOCKS);
    Partial *parts = nullptr;
    int rc = workspace(sizeof(Partial) * blocks, (void **)&parts, st);
    if (rc) return rc;
    const bool one = r.one_dma != 0;
    const uint32_t c32 = (uint32_t)count, t32 = (uint32_t)tf;
    if (one) {
        if (d_per_order)
            hipLaunchKernelGGL((rounds_kernel<true, true>), dim3(blocks), dim3(RD_THREADS), 0, st, d_tasks, T,
                               R, r, c32, t32, d_per_order, parts);
        else
            hipLaunchKernelGGL((rounds_kernel<true, false>), dim3(blocks), dim3(RD_THREADS), 0, st, d_tasks, T,
                               R, r, c32, t32, nullptr, parts);
    } else {
        if (d_per_order)
            hipLaunchKernelGGL((rounds_kernel<false, true>), dim3(blocks), dim3(RD_THREADS), 0, st, d_tasks, T,
                               R, r, c32, t32, d_per_order, parts);
        else
            hipLaunchKernelGGL((rounds_kernel<false, false>), dim3(blocks), dim3(RD_THREADS), 0, st, d_tasks,
                               T, R, r, c32, t32, nullptr, parts);
    }
    TGO_HIP(hipGetLastError());
    hipLaunchKernelGGL(rounds_finalize, dim3(1), dim3(256), 0, st, parts, (int)blocks, T, R, count, tf, d_out);
    TGO_HIP(hipGetLastError());
    if (one)
        hipLaunchKernelGGL(rounds_heuristic_kernel<true>, dim3(1), dim3(64), 0, st, d_tasks, T, R, r, d_out,
                           d_groups);
    else
        hipLaunchKernelGGL(rounds_heuristic_kernel<false>, dim3(1), dim3(64), 0, st, d_tasks, T, R, r, d_out,
                           d_groups);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

}  // namespace tgo
