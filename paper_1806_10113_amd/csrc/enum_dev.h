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
    auto child = [&](int ci) {
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
    };
    // the three innermost levels are unrolled (each child's state is then
    // derived from the parent's registers without loop-carried copies)
    if constexpr (L <= 3) {
#pragma unroll
        for (int ci = 0; ci < L; ++ci) child(ci);
    } else {
#pragma unroll 1
        for (int ci = 0; ci < L; ++ci) child(ci);
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

// Binomial coefficients C(a, b) for a, b <= MAXN.
struct Binom {
    uint32_t c[MAXN + 1][MAXN + 1];
    constexpr Binom() : c() {
        for (int a = 0; a <= MAXN; ++a) {
            c[a][0] = 1;
            for (int b = 1; b <= a; ++b) c[a][b] = c[a - 1][b - 1] + (b <= a - 1 ? c[a - 1][b] : 0u);
        }
    }
};
__constant__ constexpr Binom BINOM{};

// Set-major order of the subtrees: index s' = c * plen! + p, where c ranks
// (lexicographically) the set of tasks in the prefix of length plen = n - m
// and p ranks their order.  Consecutive indices share the set, so the lanes
// of a wave walk the same remaining tasks in the same order (their walked
// windows place the same task at every step) and differ only in the order of
// their prefixes, which makes their DtH work alike.  Decodes s', simulates the
// prefix windows and returns the remaining tasks (ascending, one per nibble);
// *lex receives the subtree's lexicographic index (its first rank / m!).
template <int DMA, typename LaneT, typename TT, int TS, int QS>
__device__ __forceinline__ uint64_t prefix_by_set(LaneT &st, uint32_t sp, int n, int m,
                                                  const View<TT, TS, QS> &v, const Rates &r, uint32_t *lex) {
    lane_reset(st);
    const int plen = n - m;
    uint32_t pf = 1;  // plen! < 2^32: n!/m! = C(n, plen) * plen! fits 32 bits
    for (int i = 2; i <= plen; ++i) pf *= (uint32_t)i;
    const uint32_t cset = sp / pf;
    uint32_t p = sp - cset * pf;
    // the set: the cset-th plen-subset of {0..n-1} in lexicographic order
    uint64_t sub = 0, rest = 0;  // ascending nibble lists of the set and of the rest
    int ns = 0, nr = 0;
    uint32_t cc = cset;
    int k = plen;
    for (int x = 0; x < n; ++x) {
        const uint32_t w = k > 0 ? BINOM.c[n - 1 - x][k - 1] : 0u;  // subsets whose next element is x
        if (k > 0 && cc < w) {
            sub |= (uint64_t)x << (4 * ns++);
            --k;
        } else {
            cc -= k > 0 ? w : 0u;
            rest |= (uint64_t)x << (4 * nr++);
        }
    }
    // the order: factorial digits of p over the set; the lexicographic index
    // of the prefix counts, at each position, the unused tasks below it
    uint32_t f = pf / (plen > 0 ? (uint32_t)plen : 1u);  // (plen - 1)!
    uint32_t blk = 1;  // (n-1-i)!/m! at position i
    for (int i = m + 1; i <= n - 1; ++i) blk *= (uint32_t)i;
    uint32_t avail = (1u << n) - 1u;
    uint32_t s = 0;
    for (int i = 0; i < plen; ++i) {
        const uint32_t d = p / f;
        p -= d * f;
        const uint32_t x = (uint32_t)(sub >> (4 * d)) & 15u;
        const uint64_t lo = sub & ((1ull << (4 * d)) - 1ull);
        const uint64_t hi = (sub >> (4 * d + 4)) << (4 * d);
        sub = lo | hi;
        s += (uint32_t)__popc(avail & ((1u << x) - 1u)) * blk;
        avail &= ~(1u << x);
        if (i + 1 < plen) {
            f /= (uint32_t)(plen - 1 - i);
            blk /= (uint32_t)(n - 1 - i);
        }
        window<DMA>(st, i, x, v, r);
    }
    *lex = s;
    return rest;
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
