// Device-side temporal execution model (gfx950).
//
// The model is the FIFO simulator of Section 4.1 for a two-DMA device
// (launch scheme of Section 3.2 with three command queues), with the
// overlapped-transfer slowdown of Section 4.2.1 read as constant rates p/q.
// Integer nanoseconds; remaining transfer work exact in 1/q solo-ns units; a
// completion estimate is rounded up to a whole nanosecond.
//
// GPU formulation (same results as stepping every event):
//   * The HtD engine is busy without a gap from t = 0 until the last HtD
//     completes, so the DtH rate is p_dth/q for every DtH that starts before
//     that instant and q/q afterwards.  The HtD rate changes only when the
//     DtH engine goes idle or starts from idle.
//   * Between rate changes an end estimate stays valid, because
//     ceil((U - r*D)/r) = ceil(U/r) - D for a whole number of ns D.  So each
//     running transfer carries its absolute end time, and the remaining work is
//     recomputed (one multiply) only when its rate changes.
//   * The kernel engine needs no events of its own: K_j = max(HtD_j end,
//     K_{j-1} end) + k.  A kernel completion matters only to the DtH engine,
//     which reads it from a per-lane queue in LDS (slot j = K_j end and the
//     overlapped duration of DtH j, so one read serves each DtH event).
//   * The simulation is cut into "windows": window j runs from the start to
//     the end of HtD at position j and processes the DtH events inside it.
//     The state at the start of window j depends only on positions < j, which
//     lets an enumeration share the windows of a common prefix.
//   * Chain form (CLane below): since every DtH that starts before the last
//     HtD ends runs at the overlapped rate, its start and end follow from the
//     previous DtH's end and its own kernel's end alone:
//     S_j = max(E_{j-1}, K_j), E_j = S_j + ceil(q d_j / p_dth).  Window j
//     appends DtH j to this chain once K_j is known, and a window only walks
//     the DtHs that end inside it; a start from idle is handled in the same
//     step as the completion before it, and a DtH that follows the previous
//     one without a gap leaves the HtD estimate as it is.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tgo {

constexpr int MAXN = 16;

// Host-prepared model constants.
struct Rates {
    int32_t q_log2;
    uint32_t p_h, p_d;
    int32_t one_dma;  // 1: device with one DMA engine (launch scheme of Section 3.2)
    // ceil(u / p) for u < 2^32 as trunc(fma(u, 1/p, (p - 1/2)/p)).  The exact
    // value (u + p - 1/2)/p lies at least 1/(2p) away from the integers that
    // bound ceil(u/p); the double rounding error is below 2^-19 for u < 2^32,
    // so for p <= 1024 the truncation is exact.
    double inv_ph, c_ph;
    double inv_pd, c_pd;
};

template <typename TT>
struct alignas(4 * sizeof(TT)) DRec {
    TT d;      // DtH solo duration
    TT dp;     // duration when fully overlapped: ceil(q d / p_dth)
    TT slack;  // p_dth dp - q d, in [0, p_dth)
    TT pad;
};

template <typename TT>
struct alignas(4 * sizeof(TT)) Quad {
    TT h, hp, k, d;  // HtD solo, HtD fully overlapped, kernel, DtH solo
};

template <typename TT>
struct alignas(2 * sizeof(TT)) Slot {
    TT ck;  // completion time of the kernel at this position
    TT dp;  // its DtH while overlapped: ceil(q d / p_dth).  p_dth dp = q d + slack
            // with slack < p_dth <= q, so d and slack follow from p_dth dp
};

// Chain entry of DtH j: start and end while the HtD engine is busy.
template <typename TT>
struct alignas(2 * sizeof(TT)) Span {
    TT s, e;
};
static_assert(sizeof(Span<uint32_t>) == sizeof(Slot<uint32_t>), "chain entries reuse the queue slots");
static_assert(sizeof(Span<uint64_t>) == sizeof(Slot<uint64_t>), "chain entries reuse the queue slots");

template <typename TT> struct Signed;
template <> struct Signed<uint32_t> { using type = int32_t; };
template <> struct Signed<uint64_t> { using type = int64_t; };

template <typename TT>
__device__ __forceinline__ TT ceil_q(TT u, int q_log2) {
    return (u + ((TT(1) << q_log2) - 1)) >> q_log2;
}

__device__ __forceinline__ uint32_t ceil_p(uint32_t u, uint32_t, double inv, double c) {
    return (uint32_t)__builtin_fma((double)u, inv, c);
}
__device__ __forceinline__ uint64_t ceil_p(uint64_t u, uint32_t p, double, double) {
    return (u + p - 1) / p;
}

template <typename TT>
__device__ __forceinline__ TT tmax(TT a, TT b) { return a > b ? a : b; }

template <typename TT>
__device__ __forceinline__ TT inf_time() { return ~TT(0); }

// Launch scheme a function is compiled for: read from Rates at run time, or
// fixed at compile time (kernels specialised for one scheme).
enum DmaMode : int { DMA_RUNTIME = 0, DMA_ONE = 1, DMA_TWO = 2 };

template <int DMA>
__device__ __forceinline__ bool is_one_dma(const Rates &r) {
    if constexpr (DMA == DMA_ONE) return true;
    else if constexpr (DMA == DMA_TWO) return false;
    else return r.one_dma != 0;
}

// Task tables and the per-lane kernel-completion queue.  Entry x of a table
// is at [x * TS], slot j of the queue at [j * QS] (compile-time strides);
// shared tables use TS = 1, per-lane tables interleave lanes so that a
// wave's accesses fall into distinct banks.
template <typename TT, int TS, int QS>
struct View {
    const Quad<TT> *H;  // (h, ceil(q h / p_h), k, d)
    const DRec<TT> *D;  // (d, ceil(q d / p_d), slack)
    Slot<TT> *Q;
    __device__ __forceinline__ Quad<TT> task(uint32_t x) const { return H[x * TS]; }
    __device__ __forceinline__ DRec<TT> d(uint32_t x) const { return D[x * TS]; }
    __device__ __forceinline__ Slot<TT> q(int j) const { return Q[j * QS]; }
    __device__ __forceinline__ void put(int j, Slot<TT> s) const { Q[j * QS] = s; }
    // the same queue memory holding chain entries (start, end) of DtH j
    __device__ __forceinline__ Span<TT> span(int j) const { return reinterpret_cast<const Span<TT> *>(Q)[j * QS]; }
    __device__ __forceinline__ void put_span(int j, Span<TT> e) const { reinterpret_cast<Span<TT> *>(Q)[j * QS] = e; }
};

// Simulation state at the start of a window (an HtD about to start).
template <typename TT>
struct Lane {
    using ST = typename Signed<TT>::type;
    TT t;        // now: end of the previous HtD (0 before the first)
    TT ck;       // end of the previous kernel
    TT dev;      // next DtH event: end of the running DtH, or (idle) end of
                 // the kernel it waits for; inf while that is not known yet
    TT slack;    // running DtH: p_dth dp - q d of its task; with end estimate
                 // dev its work left at time t <= dev is p_dth (dev - t) - slack
    TT dpre;     // sum of solo DtH durations of the positions placed so far
    TT dthru;    // sum of solo DtH durations up to the cursor (running included)
    ST emax;     // max over placed positions p of (K_p end - sum_{s<p} d_s)
    int i;       // DtH cursor (position of the running or next DtH)
    bool drun;   // DtH engine busy
};

template <typename TT>
__device__ __forceinline__ Lane<TT> lane_init() {
    using ST = typename Signed<TT>::type;
    Lane<TT> s;
    s.t = 0; s.ck = 0; s.dev = inf_time<TT>(); s.slack = 0;
    s.dpre = 0; s.dthru = 0;
    s.emax = (ST)(((TT)1) << (8 * sizeof(TT) - 1));  // most negative
    s.i = 0; s.drun = false;
    return s;
}

template <typename TT>
__device__ __forceinline__ void lane_reset(Lane<TT> &s) { s = lane_init<TT>(); }

// One DMA engine (Section 3.2, scheme for such devices): every HtD is queued
// on the one transfer engine before every DtH, so the HtDs run back to back
// at solo speed (two transfers never move data at the same time), kernels
// follow K_j = max(HtD_j end, K_{j-1} end) + k, and every DtH waits for the
// last HtD.  A window is the HtD alone; the DtHs are left to the tail.
template <typename TT, int TS, int QS>
__device__ __forceinline__ void window_one(Lane<TT> &s, uint32_t x, const View<TT, TS, QS> &v) {
    using ST = typename Signed<TT>::type;
    const Quad<TT> tx = v.task(x);
    s.t += tx.h;
    s.ck = tmax(s.t, s.ck) + tx.k;
    const ST e = (ST)s.ck - (ST)s.dpre;
    s.emax = e > s.emax ? e : s.emax;
    s.dpre += tx.d;
}

// Window j: HtD of task x starts at s.t; process DtH events until it ends,
// then derive the kernel of position j and record it in the queue.
//
// A DtH event is either a completion (engine busy) or a start from idle.  A
// completion followed at once by the next DtH leaves both rates unchanged, so
// the HtD end estimate stays valid; only a change of the DtH engine between
// busy and idle changes the HtD rate and forces a new estimate from the exact
// remaining work.
// PUT = false skips writing the position's queue slot (the last position of
// an ordering: no later window reads it).
template <int DMA = DMA_RUNTIME, bool PUT = true, typename TT, int TS, int QS>
__device__ __forceinline__ void window(Lane<TT> &s, int j, uint32_t x, const View<TT, TS, QS> &v,
                                       const Rates &r) {
    using ST = typename Signed<TT>::type;
    if (is_one_dma<DMA>(r)) {
        window_one(s, x, v);
        return;
    }
    const TT q = TT(1) << r.q_log2;
    const Quad<TT> tx = v.task(x);
    // an idle DtH waiting for the previous position's kernel now knows its time
    if (!s.drun && s.i == j - 1) s.dev = s.ck;
    const int jlast = j > 0 ? j - 1 : 0;
    TT uh = tx.h << r.q_log2;  // remaining HtD work at th0
    TT th0 = s.t;
    TT eh = s.t + (s.drun ? tx.hp : tx.h);
    for (;;) {
        const TT ev = s.dev;
        if (!(ev < eh)) break;
        const int inew = s.i + (s.drun ? 1 : 0);
        // slot inew is only used if inew < j.  The last position's window
        // (PUT = false) reads slot min(inew, j - 1) so that a queue of n - 1
        // slots suffices; other windows read slots <= j < n - 1
        const Slot<TT> nx = v.q(PUT ? inew : (inew < jlast ? inew : jlast));
        const bool start = inew < j && nx.ck <= ev;
        if (start != s.drun) {
            // the HtD rate changes at ev: exact remaining work, new estimate
            // (both roundings computed and selected: no nested branch)
            uh -= (s.drun ? TT(r.p_h) : q) * (ev - th0);
            th0 = ev;
            const TT cp = (TT)ceil_p(uh, r.p_h, r.inv_ph, r.c_ph);
            const TT cq = ceil_q(uh, r.q_log2);
            eh = ev + (start ? cp : cq);
        }
        // the DtH that starts (or not): computed on every lane and selected,
        // which measured faster than a second divergent branch.  Its solo time
        // and rounding slack come from w = p_dth dp = q d + slack (no further
        // LDS read on the loop's path)
        const TT w = TT(r.p_d) * nx.dp;
        s.dthru += start ? (w >> r.q_log2) : TT(0);
        s.slack = start ? (w & (q - 1)) : s.slack;
        s.dev = start ? ev + nx.dp : (inew < j ? nx.ck : inf_time<TT>());
        s.drun = start;
        s.i = inew;
    }
    s.t = eh;
    s.ck = tmax(eh, s.ck) + tx.k;
    const ST e = (ST)s.ck - (ST)s.dpre;
    s.emax = e > s.emax ? e : s.emax;
    s.dpre += tx.d;
    if constexpr (PUT) {
        Slot<TT> sl;
        sl.ck = s.ck;
        sl.dp = v.d(x).dp;
        v.put(j, sl);
    }
}

// Total time once the last placed HtD has ended at s.t (used for the whole
// group, and for a prefix simulated on its own).  After that instant every
// DtH runs at full speed, so the rest is the two-machine recurrence
// D = max(D, K_p end) + d_p over the remaining positions, whose value is
//   max(end of the running DtH + sum of the solo DtH left after it,
//       max_p (K_p end + sum_{s >= p} d_s)).
// Terms of positions whose DtH already started are lower bounds of the total
// (every DtH takes at least its solo time after its kernel), so the second max
// may run over every placed position: it is emax + dpre, kept per window.
//
// With one DMA engine the DtH recurrence starts when the last HtD ends (the
// engine is busy with HtDs until s.t), so the total is
// max(s.t + sum d, max_p (K_p end + sum_{s >= p} d_s)) = max(s.t, emax) + dpre.
template <int DMA = DMA_RUNTIME, typename TT>
__device__ __forceinline__ TT tail(const Lane<TT> &s, const Rates &r) {
    using ST = typename Signed<TT>::type;
    if (is_one_dma<DMA>(r)) {
        const ST e = (ST)s.t > s.emax ? (ST)s.t : s.emax;
        return (TT)(e + (ST)s.dpre);
    }
    TT T = (TT)(s.emax + (ST)s.dpre);
    if (s.drun) {
        // work left on the running DtH (it ran at p_dth since its start;
        // s.dev >= s.t): q d - p_dth (t - start) = p_dth (dev - t) - slack
        const TT pw = TT(r.p_d) * (s.dev - s.t);
        const TT ud = pw > s.slack ? pw - s.slack : TT(0);
        const TT dend = s.t + ceil_q(ud, r.q_log2) + (s.dpre - s.dthru);
        T = tmax(T, dend);
    }
    return T;
}

// ------------------------------------------------------------ chain form
// Simulation state at the start of a window, two DMA engines.  The DtHs of
// positions < j are on the chain (entries in the queue); c is the first of
// them that may still run at t, and its entry is kept in registers.
template <typename TT>
struct CLane {
    using ST = typename Signed<TT>::type;
    TT t;       // now: end of the previous HtD (0 before the first)
    TT ck;      // end of the previous kernel
    ST emax;    // max over placed positions p of (K_p end - sum_{s<p} d_s)
    TT dpre;    // sum of solo DtH durations of the positions placed so far
    TT elast;   // end of the last DtH on the chain (0 while it is empty)
    TT cs, ce;  // start and end of DtH c (when c is on the chain)
    TT dcross;  // sum of solo DtH durations of the DtHs before c
    int c;      // chain cursor: every DtH before c ends by t
    bool run;   // the last window's HtD ended while DtH c ran
};

template <typename TT>
__device__ __forceinline__ void lane_reset(CLane<TT> &s) {
    using ST = typename Signed<TT>::type;
    s.t = 0; s.ck = 0;
    s.emax = (ST)(((TT)1) << (8 * sizeof(TT) - 1));  // most negative
    s.dpre = 0; s.elast = 0; s.cs = 0; s.ce = 0; s.dcross = 0;
    s.c = 0; s.run = false;
}

// Window j of the chain form: HtD of task x from s.t, against the DtHs on the
// chain.  The loop visits only DtHs that end before the HtD: in the busy state
// the HtD end estimate stays valid while DtHs follow each other without a gap;
// at a gap the exact remaining work gives the idle estimate, and a DtH that
// starts before it gives a new busy estimate.  Event order and roundings are
// those of the event-by-event window (an event at ev is processed when ev is
// before the current estimate).  PUT = false skips appending DtH j (the last
// position: no later window reads it).
template <int DMA = DMA_TWO, bool PUT = true, typename TT, int TS, int QS>
__device__ __forceinline__ void window(CLane<TT> &s, int j, uint32_t x, const View<TT, TS, QS> &v,
                                       const Rates &r) {
    static_assert(DMA == DMA_TWO, "the chain form models two DMA engines");
    using ST = typename Signed<TT>::type;
    const Quad<TT> tx = v.task(x);
    int i = s.c;
    TT S = s.cs, E = s.ce, dsum = s.dcross;
    TT rc = s.t;                  // last rate change
    TT u = tx.h << r.q_log2;      // HtD work left at rc, 1/q solo-ns
    TT eb;                        // HtD end estimate
    TT ecmp = E;                  // end of the running DtH; inf once the HtD end is final
    if (!(i < j)) {
        eb = s.t + tx.h;          // no DtH on the chain (first position)
        ecmp = inf_time<TT>();
    } else if (S < s.t) {
        eb = s.t + tx.hp;         // DtH c runs at t
    } else {
        const TT ei = s.t + tx.h;
        if (S < ei) {             // DtH c starts inside the window
            u -= (S - s.t) << r.q_log2;
            rc = S;
            eb = S + (TT)ceil_p(u, r.p_h, r.inv_ph, r.c_ph);
        } else {
            eb = ei;
            ecmp = inf_time<TT>();
        }
    }
    // One exit: while the running DtH ends before the estimate, it completes
    // and the next one on the chain follows, after a gap or without one.
    while (ecmp < eb) {
        // its solo time joins the crossed sum (p_dth dp = q d + slack, slack < q)
        dsum += (TT(r.p_d) * (E - S)) >> r.q_log2;
        const TT ep = E;
        ++i;
        const Span<TT> nx = v.span(i < j ? i : j - 1);  // slot j - 1 exists: i >= 1
        S = nx.s;
        E = nx.e;
        ecmp = E;
        if (!(i < j) || S != ep) {
            // the DtH engine goes idle at ep: exact work left, idle estimate;
            // the next DtH starts from idle if it begins before that estimate
            u -= TT(r.p_h) * (ep - rc);
            rc = ep;
            const TT ei = rc + ceil_q(u, r.q_log2);
            const bool start = i < j && S < ei;
            const TT us = u - ((S - rc) << r.q_log2);
            const TT ebs = S + (TT)ceil_p(us, r.p_h, r.inv_ph, r.c_ph);
            u = start ? us : u;
            rc = start ? S : rc;
            eb = start ? ebs : ei;
            ecmp = start ? ecmp : inf_time<TT>();
        }
    }
    const TT eh = eb;
    const bool run = ecmp != inf_time<TT>();
    s.c = i;
    s.cs = S;
    s.ce = E;
    s.dcross = dsum;
    s.run = run;
    s.t = eh;
    s.ck = tmax(eh, s.ck) + tx.k;
    const ST e = (ST)s.ck - (ST)s.dpre;
    s.emax = e > s.emax ? e : s.emax;
    s.dpre += tx.d;
    if constexpr (PUT) {
        // DtH j joins the chain: it starts once the engine and its kernel are done
        Span<TT> sp;
        sp.s = tmax(s.elast, s.ck);
        sp.e = sp.s + v.d(x).dp;
        v.put_span(j, sp);
        s.elast = sp.e;
        if (s.c == j) {
            s.cs = sp.s;
            s.ce = sp.e;
        }
    }
}

// Total time of the chain form once the last HtD has ended at s.t: the
// two-machine recurrence of the event form's tail.  A DtH running at s.t has
// moved p_dth (s.t - start) of its q d work, so it needs
// d - floor(p_dth (s.t - start) / q) more ns at full speed, followed by the
// solo times of the DtHs after it.
template <int DMA = DMA_TWO, typename TT>
__device__ __forceinline__ TT tail(const CLane<TT> &s, const Rates &r) {
    static_assert(DMA == DMA_TWO, "the chain form models two DMA engines");
    using ST = typename Signed<TT>::type;
    TT T = (TT)(s.emax + (ST)s.dpre);
    if (s.run) {
        const TT dend = s.t + (s.dpre - s.dcross) - ((TT(r.p_d) * (s.t - s.cs)) >> r.q_log2);
        T = tmax(T, dend);
    }
    return T;
}

// T of one whole ordering o[0..n) (o(j) gives the task at position j): the
// chain form with two DMA engines, the event form's windows with one.  The
// queue needs n - 1 slots.
template <typename TT, int TS, int QS, typename Order>
__device__ __forceinline__ TT simulate_order(int n, Order o, const View<TT, TS, QS> &v, const Rates &r) {
    if (is_one_dma<DMA_RUNTIME>(r)) {
        Lane<TT> st = lane_init<TT>();
        for (int j = 0; j < n; ++j) window<DMA_ONE>(st, j, o(j), v, r);
        return tail<DMA_ONE>(st, r);
    }
    CLane<TT> st;
    lane_reset(st);
    for (int j = 0; j + 1 < n; ++j) window<DMA_TWO, true>(st, j, o(j), v, r);
    if (n > 0) window<DMA_TWO, false>(st, n - 1, o(n - 1), v, r);
    return tail<DMA_TWO>(st, r);
}

// Host-side validity bound for the 32-bit time path (checked on the device
// from the task table): every work amount fits 31 bits and every instant of
// the simulation fits 31 bits.  T never exceeds the sum of each command's
// slowest duration plus one ns of rounding per rate change per command.
__host__ __device__ inline uint64_t time_bound_slack(int n) { return 3ull * n * (2ull * n + 2ull); }

}  // namespace tgo
