// The ordering heuristic of Section 5.1 (Algorithm 1) as a per-lane device
// function, shared by the per-group heuristic kernel and the proxy of the
// multi-round evaluator.
//
// The three selection functions are described in words only; the readings:
//   select_first: largest K - HtD (short HtD, long kernel); ties to the longer
//                 DtH, then the lower index.
//   select_next:  smallest |h_c - (t_K - t_HtD)| + |k_c - (t_DtH - max(t_HtD + h_c, t_K))|,
//                 i.e. the HtD that best fills the kernel engine's remaining
//                 busy time and the kernel that best fills the DtH engine's;
//                 ties to the lower index.
//   select_last:  both orders (x, y) of the last two tasks scored
//                 fit(x | OT) + fit(y | OT + x) + d_y; ties to the shorter
//                 final DtH, then to x with the lower index.
// t_HtD, t_K, t_DtH come from simulating the ordered set OT alone (update).
#pragma once

#include "../../include/tgo.h"
#include "model_dev.h"

namespace tgo {

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

template <typename TT, int TS, int QS>
__device__ __forceinline__ Fit3 fit_state(const Lane<TT> &st, const Rates &r) {
    Fit3 u;
    u.th = (int64_t)st.t;
    u.tk = (int64_t)st.ck;
    u.td = (int64_t)tail(st, r);
    return u;
}

// Algorithm 1 on n tasks: v holds the lane's tables of tasks 0..n-1 (built
// by the caller) and its queue; the candidates' durations are read from those
// LDS tables, not from global memory, since every selection step scans all of
// them.  Writes the ordering to ord[0..n-1] and returns its total time.
template <int TS, int QS>
__device__ int64_t heuristic_order(int n, const View<uint64_t, TS, QS> &v, const Rates &r, uint8_t *ord) {
    using TT = uint64_t;
    auto task = [&v](int x) {
        const Quad<TT> q = v.task((uint32_t)x);
        tgo_task t;
        t.htd_ns = (int64_t)q.h;
        t.kern_ns = (int64_t)q.k;
        t.dth_ns = (int64_t)q.d;
        return t;
    };
    uint32_t rt = (1u << n) - 1u;
    int first = -1;
    int64_t bkh = 0, bd = 0;
    for (int x = 0; x < n; ++x) {
        const tgo_task tx = task(x);
        const int64_t kh = tx.kern_ns - tx.htd_ns, d = tx.dth_ns;
        if (first < 0 || kh > bkh || (kh == bkh && d > bd)) { first = x; bkh = kh; bd = d; }
    }
    ord[0] = (uint8_t)first;
    rt &= ~(1u << first);
    Lane<TT> st = lane_init<TT>();
    window(st, 0, (uint32_t)first, v, r);
    int pos = 1;
    while (__popc(rt) > 2) {
        const Fit3 u = fit_state<TT, TS, QS>(st, r);
        int best = -1;
        int64_t bf = 0;
        for (int c = 0; c < n; ++c) {
            if (!((rt >> c) & 1u)) continue;
            const tgo_task tc = task(c);
            const int64_t f = fit(tc.htd_ns, tc.kern_ns, u);
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
        const Fit3 u = fit_state<TT, TS, QS>(st, r);
        int bx = -1, by = -1;
        int64_t bs = 0, bdy = 0;
        for (int o = 0; o < 2; ++o) {
            const int x = o == 0 ? a : b, y = o == 0 ? b : a;
            const tgo_task tx = task(x), ty = task(y);
            const int64_t s1 = fit(tx.htd_ns, tx.kern_ns, u);
            Lane<TT> s2 = st;
            window(s2, pos, (uint32_t)x, v, r);
            const Fit3 w = fit_state<TT, TS, QS>(s2, r);
            const int64_t sc = s1 + fit(ty.htd_ns, ty.kern_ns, w) + ty.dth_ns;
            const int64_t dy = ty.dth_ns;
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
    return (int64_t)tail(st, r);
}

}  // namespace tgo
