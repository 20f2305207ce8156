// Task groups under a device-memory limit: lane-level simulators.
//
// Section 5 observes that tasks running at the same time hold their input and
// output buffers at once, so the device memory can restrict which tasks may
// run together; the paper assumes enough memory.  Reading: task x holds
// mem[x] bytes from the start of its HtD to the end of its DtH, at most `cap`
// bytes at once.
//
// Two DMA engines (GSim): the HtD at the head of its queue starts only when
// its bytes fit beside those held; the HtDs behind it wait too.  The engine
// can then sit idle while a DtH finishes, which breaks the premise of the
// window formulation (an HtD engine busy without gaps), so the simulation
// steps events: at each instant finished commands retire and ready heads
// start until nothing changes, then time advances to the earliest
// completion estimate.  Remaining transfer work is exact in 1/q solo-ns;
// estimates round up to whole ns; an HtD and a DtH moving data together
// advance at p_htd/q and p_dth/q.  DtHs end in launch order, so the bytes
// held are those of positions [DtHs done, HtDs started).
//
// One DMA engine (Chain): the ordering is cut greedily into consecutive
// sub-groups whose bytes fit together, each launched as its HtDs and then its
// DtHs on the one transfer engine.  Transfers never overlap, so no rate
// applies and the schedule is the closed-form chain: HtDs back to back,
// K_i = max(HtD_i end, K_{i-1} end) + k_i, and after the sub-group's last HtD
// its DtHs in order, D_i = max(K_i, D_{i-1}) + d_i (kept as a running max, so
// each position costs O(1)); the next sub-group's HtDs follow its last DtH.
//
// Both expose push (place the next task; for GSim the simulation then runs
// to the instant that task's HtD ends, after which nothing depends on later
// positions) and finish (the rest in closed form, return T).  An enumeration can thus
// keep the state after a common prefix and extend it per suffix.
#pragma once

#include "model_dev.h"

namespace tgo {

template <typename TT>
struct MemTab {
    TT qh[MAXN], k[MAXN], qd[MAXN];  // q * h, k, q * d
    TT h[MAXN], d[MAXN];
    uint64_t m[MAXN];
};

__device__ __forceinline__ uint32_t mnib(uint64_t v, int i) { return (uint32_t)(v >> (4 * i)) & 15u; }

// Per-lane queue of kernel end times (LDS, one slot per position, slots of a
// wave's lanes adjacent): the end of K_i is fixed once HtD_i has ended.
template <typename TT>
struct KQ {
    TT *base;
    int stride;
    __device__ __forceinline__ TT get(int i) const { return base[i * stride]; }
    __device__ __forceinline__ void put(int i, TT v) const { base[i * stride] = v; }
};

template <typename TT>
struct GSim {
    TT t, uh, ud;   // now; HtD and DtH work left (1/q solo-ns)
    TT kp;          // end of the kernel of the last position whose HtD ended
    uint64_t held;
    uint64_t seq;   // nibble j: task at position j
    int n;          // positions placed
    int hc, dc;     // next position to start on the HtD / DtH engine
    int hd, dd;     // positions finished on the HtD / DtH engine
};

template <typename TT>
__device__ __forceinline__ void gsim_init(GSim<TT> &s) {
    s.t = s.uh = s.ud = s.kp = 0;
    s.held = 0;
    s.seq = 0;
    s.n = s.hc = s.dc = s.hd = s.dd = 0;
}

// All retirements and starts at the current instant.  The kernel engine
// needs no events: K_i = max(HtD_i end, K_{i-1} end) + k_i is fixed when
// HtD_i ends and kept in the queue; the DtH of position i starts once the
// engine is free and t has reached K_i.  One sweep (retire HtD, DtH, then
// start HtD, DtH) follows every chain of causes within the instant; only a
// command that starts with zero duration needs another sweep.
template <typename TT>
__device__ __forceinline__ void gsim_pass(GSim<TT> &s, const MemTab<TT> &tb, uint64_t cap, const KQ<TT> &kq) {
    for (;;) {
        if (s.hc > s.hd && s.uh == 0) {
            s.kp = tmax(s.t, s.kp) + tb.k[mnib(s.seq, s.hd)];
            kq.put(s.hd, s.kp);
            ++s.hd;
        }
        if (s.dc > s.dd && s.ud == 0) {
            s.held -= tb.m[mnib(s.seq, s.dd)];
            ++s.dd;
        }
        bool again = false;
        if (s.hc == s.hd && s.hc < s.n) {
            const uint32_t x = mnib(s.seq, s.hc);
            if (s.held + tb.m[x] <= cap) {
                s.held += tb.m[x];
                s.uh = tb.qh[x];
                ++s.hc;
                again = again || s.uh == 0;
            }
        }
        if (s.dc == s.dd && s.dc < s.hd && kq.get(s.dc) <= s.t) {
            s.ud = tb.qd[mnib(s.seq, s.dc)];
            ++s.dc;
            again = again || s.ud == 0;
        }
        if (!again) break;
    }
}

// Advance to the earliest completion estimate (a transfer's end, or the end
// of the kernel an idle DtH engine waits for); false when nothing is pending.
template <typename TT>
__device__ __forceinline__ bool gsim_advance(GSim<TT> &s, const Rates &r, const KQ<TT> &kq) {
    const bool hrun = s.hc > s.hd, drun = s.dc > s.dd;
    const bool dwait = !drun && s.dc < s.hd;
    if (!hrun && !drun && !dwait) return false;
    const bool both = hrun && drun;
    const TT INF = inf_time<TT>();
    const TT eh = hrun ? (both ? (TT)ceil_p(s.uh, r.p_h, r.inv_ph, r.c_ph) : ceil_q(s.uh, r.q_log2)) : INF;
    const TT ed = drun ? (both ? (TT)ceil_p(s.ud, r.p_d, r.inv_pd, r.c_pd) : ceil_q(s.ud, r.q_log2)) : INF;
    const TT ek = dwait ? kq.get(s.dc) - s.t : INF;
    TT dt = eh < ed ? eh : ed;
    dt = ek < dt ? ek : dt;
    const TT q = TT(1) << r.q_log2;
    if (hrun) s.uh = eh == dt ? TT(0) : s.uh - (both ? TT(r.p_h) : q) * dt;
    if (drun) s.ud = ed == dt ? TT(0) : s.ud - (both ? TT(r.p_d) : q) * dt;
    s.t += dt;
    return true;
}

// Place task x at the next position and run to the instant its HtD ends.
template <typename TT>
__device__ __forceinline__ void gsim_push(GSim<TT> &s, uint32_t x, const MemTab<TT> &tb, uint64_t cap,
                                          const Rates &r, const KQ<TT> &kq) {
    s.seq |= (uint64_t)x << (4 * s.n);
    ++s.n;
    for (;;) {
        gsim_pass(s, tb, cap, kq);
        if (s.hd == s.n) break;
        if (!gsim_advance(s, r, kq)) break;
    }
}

// Total time once every HtD has ended (the state gsim_push leaves after the
// last position): no transfer overlaps any more, so the running DtH ends
// ceil(ud / q) later and each later DtH takes its solo time, starting when
// both its kernel and the previous DtH have ended.
template <typename TT>
__device__ __forceinline__ TT gsim_finish(const GSim<TT> &s, const MemTab<TT> &tb, const Rates &r,
                                          const KQ<TT> &kq) {
    TT D = s.dc > s.dd ? s.t + ceil_q(s.ud, r.q_log2) : s.t;
    for (int i = s.dc; i < s.n; ++i) D = tmax(kq.get(i), D) + tb.d[mnib(s.seq, i)];
    return D;
}

template <typename TT>
struct Chain {
    using ST = typename Signed<TT>::type;
    TT x;      // transfer engine: end of the open sub-group's last HtD (or of
               // the previous sub-group's last DtH while none is open)
    TT kp;     // end of the last kernel
    ST emax;   // open sub-group: max over its positions p of
               // (K_p end - its DtH time before p)
    TT dsum;   // open sub-group: its DtH time so far
    uint64_t held;
    int open;  // positions in the open sub-group
};

template <typename TT>
__device__ __forceinline__ void chain_init(Chain<TT> &c) {
    using ST = typename Signed<TT>::type;
    c.x = c.kp = 0;
    c.emax = (ST)(((TT)1) << (8 * sizeof(TT) - 1));  // most negative
    c.dsum = 0;
    c.held = 0;
    c.open = 0;
}

// The open sub-group's DtHs: after its last HtD they run in order, each when
// its kernel has ended, so the last one ends at
// max(x, max_p (K_p - sum_{s<p} d_s)) + sum d (the recurrence
// D_p = max(K_p, D_{p-1}) + d_p unrolled).
template <typename TT>
__device__ __forceinline__ void chain_close(Chain<TT> &c) {
    using ST = typename Signed<TT>::type;
    const ST e = (ST)c.x > c.emax ? (ST)c.x : c.emax;
    c.x = (TT)(e + (ST)c.dsum);
    c.emax = (ST)(((TT)1) << (8 * sizeof(TT) - 1));
    c.dsum = 0;
    c.held = 0;
    c.open = 0;
}

template <typename TT>
__device__ __forceinline__ void chain_push(Chain<TT> &c, uint32_t x, const MemTab<TT> &tb, uint64_t cap) {
    using ST = typename Signed<TT>::type;
    if (c.open > 0 && c.held + tb.m[x] > cap) chain_close(c);
    c.x += tb.h[x];
    c.kp = tmax(c.x, c.kp) + tb.k[x];
    const ST e = (ST)c.kp - (ST)c.dsum;
    c.emax = e > c.emax ? e : c.emax;
    c.dsum += tb.d[x];
    c.held += tb.m[x];
    ++c.open;
}

template <typename TT>
__device__ __forceinline__ TT chain_finish(Chain<TT> &c, const MemTab<TT> &) {
    if (c.open > 0) chain_close(c);
    return c.x;
}

}  // namespace tgo
