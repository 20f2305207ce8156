// Task-table loading and validation on the device.
#pragma once

#include "../../include/tgo.h"
#include "model_dev.h"

namespace tgo {

// 0 = every instant and work amount fits the 32-bit path, 1 = 64-bit path,
// TGO_ERANGE = a duration is negative or >= 2^40 ns.
__device__ inline int classify_group(const tgo_task *t, int n, const Rates &r) {
    const uint64_t q = 1ull << r.q_log2;
    uint64_t mx = 0, sum = 0;
    for (int i = 0; i < n; ++i) {
        const int64_t h = t[i].htd_ns, k = t[i].kern_ns, d = t[i].dth_ns;
        const int64_t lim = int64_t(1) << 40;
        if (h < 0 || k < 0 || d < 0 || h >= lim || k >= lim || d >= lim) return TGO_ERANGE;
        const uint64_t qh = q * (uint64_t)h, qd = q * (uint64_t)d;
        mx = qh > mx ? qh : mx;
        mx = qd > mx ? qd : mx;
        sum += (qh + r.p_h - 1) / r.p_h + (uint64_t)k + (qd + r.p_d - 1) / r.p_d;
    }
    const uint64_t lim32 = 1ull << 31;
    return (mx < lim32 && sum + time_bound_slack(n) < lim32) ? 0 : 1;
}

// Entry x of the tables from task t: (h, ceil(q h/p_h), k, d) and
// (d, ceil(q d/p_d), p_d ceil(q d/p_d) - q d).
template <typename TT>
__device__ inline void table_entry(const tgo_task &t, const Rates &r, Quad<TT> *H, DRec<TT> *D) {
    const uint64_t q = 1ull << r.q_log2;
    const uint64_t h = (uint64_t)t.htd_ns, k = (uint64_t)t.kern_ns, d = (uint64_t)t.dth_ns;
    Quad<TT> e;
    e.h = (TT)h;
    e.hp = (TT)((q * h + r.p_h - 1) / r.p_h);
    e.k = (TT)k;
    e.d = (TT)d;
    DRec<TT> pd;
    const uint64_t dp = (q * d + r.p_d - 1) / r.p_d;
    pd.d = (TT)d;
    pd.dp = (TT)dp;
    pd.slack = (TT)(r.p_d * dp - q * d);
    pd.pad = 0;
    *H = e;
    *D = pd;
}

}  // namespace tgo
