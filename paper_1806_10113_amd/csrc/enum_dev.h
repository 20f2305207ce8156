// Depth-first enumeration of the last positions of a group, shared by the
// single-group and the batched exhaustive kernels.
//
// Ranks are lexicographic, so the orderings that share a prefix of length
// n - M form a contiguous block of M! ranks (a "subtree").  A lane that owns a
// subtree simulates the prefix windows once, then walks the last M positions
// in lexicographic order, re-simulating only the windows below the position
// that changed: per ordering sum_{L=1..M} 1/(L-1)! (about 2.7) windows plus the
// tail instead of n windows.
#pragma once

#include "model_dev.h"

namespace tgo {

constexpr uint64_t fact_c(int n) { return n <= 1 ? 1ull : (uint64_t)n * fact_c(n - 1); }

// Accumulators over one subtree; l is the leaf index inside the subtree
// (rank - first rank of the subtree), the same for every lane of a wave at
// the same point of the walk.
template <typename TT>
struct Sub {
    TT min_t, max_t1;
    uint32_t min_l, max_l;
    uint64_t sum;  // sum of T over the subtree (exact: M! * 2^50 < 2^64)
    uint64_t s2;   // sum of l * T, modulo 2^64
};

template <typename TT>
__device__ __forceinline__ void sub_init(Sub<TT> &u) {
    u.min_t = inf_time<TT>();
    u.max_t1 = 0;
    u.min_l = 0;
    u.max_l = 0;
    u.sum = 0;
    u.s2 = 0;
}

template <typename TT, bool STORE>
__device__ __forceinline__ void leaf(TT T, uint32_t l, Sub<TT> &u, int64_t *out_sub) {
    if (T < u.min_t) { u.min_t = T; u.min_l = l; }
    if (T >= u.max_t1) { u.max_t1 = T + 1; u.max_l = l; }
    u.sum += (uint64_t)T;
    u.s2 += (uint64_t)l * (uint64_t)T;
    if constexpr (STORE) out_sub[l] = (int64_t)T;
}

struct Ctx {
    int n;
    Rates r;
    int64_t *out_sub;  // per-ordering output at the subtree's first rank (or null)
};

// Level with L positions left (position n - L is being chosen).  list holds
// the remaining tasks in increasing order, one per nibble.  LaneT is the
// simulation state (Lane: event form, CLane: chain form).
template <typename TT, int L, bool STORE, int TS, int QS, int DMA, typename LaneT>
__device__ __forceinline__ void level(const Ctx &c, const View<TT, TS, QS> &v, const LaneT &s,
                                      uint32_t list, uint32_t l, Sub<TT> &u) {
    const int j = c.n - L;
#pragma unroll 1
    for (int ci = 0; ci < L; ++ci) {
        const uint32_t x = (list >> (4 * ci)) & 15u;
        LaneT s2 = s;
        window<DMA, (L > 1)>(s2, j, x, v, c.r);
        const uint32_t l2 = l + (uint32_t)ci * (uint32_t)fact_c(L - 1);
        if constexpr (L == 1) {
            leaf<TT, STORE>(tail<DMA>(s2, c.r), l2, u, c.out_sub);
        } else {
            const uint32_t lo = list & ((1u << (4 * ci)) - 1u);
            const uint32_t hi = (list >> (4 * ci + 4)) << (4 * ci);
            level<TT, L - 1, STORE, TS, QS, DMA>(c, v, s2, lo | hi, l2, u);
        }
    }
}

// Decode the prefix of subtree s (positions 0 .. n-M-1 of rank s*M!) and
// simulate its windows.  Returns the remaining tasks, ascending, one per nibble.
template <int DMA, typename LaneT, typename TT, int TS, int QS>
__device__ __forceinline__ uint64_t prefix(LaneT &st, uint32_t s, int n, int m,
                                           const View<TT, TS, QS> &v, const Rates &r) {
    uint64_t list = 0;
    for (int i = n - 1; i >= 0; --i) list = (list << 4) | (uint64_t)i;
    lane_reset(st);
    const int plen = n - m;
    uint32_t rem = s;
    // block size of position i in subtree units: (n-1-i)!/m!
    uint32_t blk = 1;
    for (int i = m + 1; i <= n - 1; ++i) blk *= (uint32_t)i;
    for (int i = 0; i < plen; ++i) {
        const uint32_t cdig = rem / blk;
        rem -= cdig * blk;
        if (i + 1 < plen) blk /= (uint32_t)(n - 1 - i);
        const uint32_t x = (uint32_t)(list >> (4 * cdig)) & 15u;
        const uint64_t lo = list & ((1ull << (4 * cdig)) - 1ull);
        const uint64_t hi = (list >> (4 * cdig + 4)) << (4 * cdig);
        list = lo | hi;
        window<DMA>(st, i, x, v, r);
    }
    return list;
}

template <typename T>
__device__ __forceinline__ T shfl_xor64(T v, int m) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = __shfl_xor((uint32_t)u, m);
    const uint32_t hi = __shfl_xor((uint32_t)(u >> 32), m);
    return (T)(((uint64_t)hi << 32) | lo);
}

// (t, r) pairs: smaller t wins, ties to smaller r.
__device__ __forceinline__ void merge_min(uint64_t &t, uint64_t &r, uint64_t t2, uint64_t r2) {
    if (t2 < t || (t2 == t && r2 < r)) { t = t2; r = r2; }
}
// larger t wins (t is max+1, 0 = none), ties to smaller r.
__device__ __forceinline__ void merge_max(uint64_t &t, uint64_t &r, uint64_t t2, uint64_t r2) {
    if (t2 > t || (t2 == t && r2 < r)) { t = t2; r = r2; }
}

__device__ __forceinline__ void add128(uint64_t &lo, uint64_t &hi, uint64_t lo2, uint64_t hi2) {
    const uint64_t s = lo + lo2;
    hi += hi2 + (s < lo ? 1ull : 0ull);
    lo = s;
}

}  // namespace tgo
