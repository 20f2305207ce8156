// Learned proposal for groups too large to enumerate (n up to 16).
//
// A multilayer perceptron 48 -> 256 -> 256 -> 256 -> 1 scores orderings from
// per-position task features; bfloat16 weights and activations, float32
// accumulation on the matrix cores (v_mfma_f32_16x16x32_bf16).  It is trained
// on (ordering, exact predicted time) pairs that the exact evaluator
// generates, with float32 master weights and Adam.  The search samples
// orderings with a counter-based generator, scores them, keeps the best
// scored per group and re-scores those exactly; the exact model decides the
// answer, and the heuristic of Section 5.1 is always a candidate too.
#include <algorithm>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>

#include <cmath>
#include <cstdlib>
#include <string>
#include <vector>

#include "enum_dev.h"
#include "surrogate_dev.h"
#include "tables_dev.h"
#include "tgo_internal.h"

namespace tgo {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int SG_THREADS = 256;
constexpr int GK = 32;  // K per MFMA instruction (16 x 16 x 32 bf16)

// ------------------------------------------------------------- exact lanes
// Exact evaluation of (group, ordering) items, one wave per group tile: the
// wave loads the group's task table into its own LDS area and each lane
// evaluates one ordering with simulate_order.  A group runs the 32-bit time
// path when its times stay below 2^31 ns (group mode 0) and the 64-bit path
// otherwise (mode 1); every kernel below exists in both widths and takes the
// groups of its own mode.

template <typename TT>
struct WaveTables {
    Quad<TT> H[4][MAXN];
    DRec<TT> D[4][MAXN];
};

template <typename TT, int NT>
__device__ __forceinline__ TT eval_perm(uint64_t perm, int n, const View<TT, 1, NT> &v, const Rates &r) {
    return simulate_order(n, [perm](int j) { return (uint32_t)((perm >> (4 * j)) & 15u); }, v, r);
}

template <typename TT>
__device__ __forceinline__ void load_group(WaveTables<TT> &wt, int w, int lane, const tgo_task *t, int n,
                                           const Rates &r) {
    if (lane < n) table_entry<TT>(t[lane], r, &wt.H[w][lane], &wt.D[w][lane]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename TT>
constexpr int mode_of() { return sizeof(TT) == 4 ? 0 : 1; }

// dynamic LDS of the exact-lane kernels: the per-lane kernel queue
// (the 64-bit kernels run blocks of 128 lanes: their queue stays at 32 KB)
template <typename TT>
constexpr int lane_threads() { return sizeof(TT) == 4 ? SG_THREADS : SG_THREADS / 2; }
template <typename TT>
constexpr size_t lane_queue_bytes() { return sizeof(Slot<TT>) * lane_threads<TT>() * SG_POS; }

// per group: 0 (32-bit path), 1 (64-bit path) or a TGO_E* code (size out of
// range, a duration outside [0, 2^40))
__global__ void group_status_kernel(const tgo_task *__restrict__ tasks, const int32_t *__restrict__ offs,
                                    int G, Rates r, int32_t *mode, int32_t *status) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const int n = offs[g + 1] - offs[g];
    const int c = (n < 1 || n > SG_POS) ? TGO_EINVAL : classify_group(tasks + offs[g], n, r);
    if (mode) mode[g] = c;
    if (status) status[g] = c < 0 ? c : 0;
}

// Training pairs: per group `per` sampled orderings (per is a multiple of 64)
// and their exact T.  The 32-bit instantiation also fills the rows of groups
// with an error status.
template <typename TT, int NT = lane_threads<TT>()>
__global__ __launch_bounds__(NT) void pairs_kernel(const tgo_task *__restrict__ tasks,
                                                           const int32_t *__restrict__ offs, int G,
                                                           Rates r, int64_t per, uint64_t seed,
                                                           const int32_t *__restrict__ mode,
                                                           uint8_t *orders, int32_t *gid, int64_t *T) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ WaveTables<TT> wt;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    View<TT, 1, NT> v;
    v.H = wt.H[w];
    v.D = wt.D[w];
    v.Q = reinterpret_cast<Slot<TT> *>(smem) + threadIdx.x;
    const int64_t tiles_per_group = per / 64;
    const int64_t total = tiles_per_group * G;
    const int64_t wstride = (int64_t)gridDim.x * (NT / 64);
    for (int64_t tile = (int64_t)blockIdx.x * (NT / 64) + w; tile < total; tile += wstride) {
        const int g = (int)(tile / tiles_per_group);
        const int md = mode[g];
        if (md >= 0 && md != mode_of<TT>()) continue;
        const int64_t s = (tile % tiles_per_group) * 64 + lane;
        const int64_t row = (int64_t)g * per + s;
        const int n = offs[g + 1] - offs[g];
        uint8_t *o = orders + row * SG_POS;
        if (md < 0) {
            if constexpr (sizeof(TT) == 4) {
                gid[row] = g;
                T[row] = md;
                for (int p = 0; p < SG_POS; ++p) o[p] = 0xff;
            }
            continue;
        }
        gid[row] = g;
        load_group(wt, w, lane, tasks + offs[g], n, r);
        const uint64_t perm = sample_ordering(n, (uint32_t)g, (uint64_t)s, seed);
        T[row] = (int64_t)eval_perm<TT, NT>(perm, n, v, r);
        for (int p = 0; p < SG_POS; ++p) o[p] = p < n ? (uint8_t)((perm >> (4 * p)) & 15u) : 0xff;
        __builtin_amdgcn_wave_barrier();
    }
}

// Best (T, sample) of a group, for the groups of the 64-bit path (T may need
// more than 32 bits, so it is not packed with the sample into one key).
struct BestPair {
    uint64_t t;  // ~0: none
    uint64_t s;
};

__device__ __forceinline__ void pair_min(uint64_t &t, uint64_t &s, uint64_t t2, uint64_t s2) {
    if (t2 < t || (t2 == t && s2 < s)) { t = t2; s = s2; }
}

// Plain exact search: `per` sampled orderings per group (a multiple of 64).
// Each wave takes chunks of `chunk` consecutive 64-sample tiles of one group,
// so the group's table is loaded and the wave's minimum published once per
// chunk; wave-uniform values are kept in scalar registers.  32-bit path: the
// smallest (T << 32 | sample) per group by one 64-bit atomic per chunk.
// 64-bit path: chunk c of group g writes its (T, sample) to wpart[g][c]
// (chunks of wchunk tiles, at most RS_WIDE_CHUNKS per group).
constexpr int RS_WIDE_CHUNKS = 256;

template <typename TT, int NT = lane_threads<TT>()>
__global__ __launch_bounds__(NT) void random_search_kernel(const tgo_task *__restrict__ tasks,
                                                                   const int32_t *__restrict__ offs,
                                                                   int G, Rates r, int64_t per,
                                                                   uint64_t seed, int64_t chunk_tiles,
                                                                   const int32_t *__restrict__ mode,
                                                                   unsigned long long *best, BestPair *wpart) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ WaveTables<TT> wt;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    View<TT, 1, NT> v;
    v.H = wt.H[w];
    v.D = wt.D[w];
    v.Q = reinterpret_cast<Slot<TT> *>(smem) + threadIdx.x;
    const int64_t tiles_per_group = per / 64;
    const int64_t chunks_per_group = (tiles_per_group + chunk_tiles - 1) / chunk_tiles;
    const int64_t total = chunks_per_group * G;
    const int64_t wstride = (int64_t)gridDim.x * (NT / 64);
    for (int64_t chunk = (int64_t)blockIdx.x * (NT / 64) + w; chunk < total; chunk += wstride) {
        const int g = (int)(chunk / chunks_per_group);
        if (mode[g] != mode_of<TT>()) continue;
        const int n = offs[g + 1] - offs[g];
        load_group(wt, w, lane, tasks + offs[g], n, r);
        const int64_t t0 = (chunk % chunks_per_group) * chunk_tiles;
        const int64_t t1 = t0 + chunk_tiles < tiles_per_group ? t0 + chunk_tiles : tiles_per_group;
        uint64_t bt = ~0ull, bs = ~0ull;
        for (int64_t tile = t0; tile < t1; ++tile) {
            const int64_t s = tile * 64 + lane;
            const uint64_t perm = sample_ordering(n, (uint32_t)g, (uint64_t)s, seed);
            pair_min(bt, bs, (uint64_t)eval_perm<TT, NT>(perm, n, v, r), (uint64_t)s);
        }
        for (int m = 32; m >= 1; m >>= 1) {
            const uint64_t t2 = shfl_xor64(bt, m), s2 = shfl_xor64(bs, m);
            pair_min(bt, bs, t2, s2);
        }
        if (lane == 0) {
            if constexpr (sizeof(TT) == 4) {
                atomicMin(&best[g], (unsigned long long)((bt << 32) | bs));
            } else {
                BestPair bp;
                bp.t = bt;
                bp.s = bs;
                wpart[(int64_t)g * RS_WIDE_CHUNKS + chunk % chunks_per_group] = bp;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Exact re-score of the k best-scored candidates of every group (k <= 64,
// one wave per group): keys hold the sample index in the low 32 bits.  The
// group's best (T, sample) goes to out[g] (T = ~0: no candidate).
template <typename TT, int NT = lane_threads<TT>()>
__global__ __launch_bounds__(NT) void rescore_kernel(const tgo_task *__restrict__ tasks,
                                                             const int32_t *__restrict__ offs, int G,
                                                             Rates r, int k, uint64_t seed,
                                                             const int32_t *__restrict__ mode,
                                                             const uint32_t *__restrict__ gkeys,
                                                             const unsigned long long *__restrict__ keys,
                                                             int key_stride, BestPair *out) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ WaveTables<TT> wt;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    View<TT, 1, NT> v;
    v.H = wt.H[w];
    v.D = wt.D[w];
    v.Q = reinterpret_cast<Slot<TT> *>(smem) + threadIdx.x;
    for (int g = blockIdx.x * (NT / 64) + w; g < G; g += gridDim.x * (NT / 64)) {
        const int md = mode[g];
        if (md >= 0 && md != mode_of<TT>()) continue;
        if (md < 0) {
            if (sizeof(TT) == 4 && lane == 0) out[g] = BestPair{~0ull, ~0ull};
            continue;
        }
        const int n = offs[g + 1] - offs[g];
        load_group(wt, w, lane, tasks + offs[g], n, r);
        uint64_t bt = ~0ull, bs = ~0ull;
        const unsigned long long kk = lane < k ? keys[(int64_t)g * key_stride + lane] : ~0ull;
        if (kk != ~0ull) {
            const uint64_t s = kk & 0xffffffffull;
            const uint64_t perm = sample_ordering(n, gkeys ? gkeys[g] : (uint32_t)g, s, seed);
            bt = (uint64_t)eval_perm<TT, NT>(perm, n, v, r);
            bs = s;
        }
        for (int m = 32; m >= 1; m >>= 1) {
            const uint64_t t2 = shfl_xor64(bt, m), s2 = shfl_xor64(bs, m);
            pair_min(bt, bs, t2, s2);
        }
        if (lane == 0) out[g] = BestPair{bt, bs};
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------- features

// per group: feature values of its (up to 16) tasks, float [G][16][3]
__global__ void group_features_kernel(const tgo_task *__restrict__ tasks, const int32_t *__restrict__ offs,
                                      int G, float *F) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= G * SG_POS) return;
    const int g = i / SG_POS, x = i % SG_POS;
    const int n = offs[g + 1] - offs[g];
    float *f = F + (int64_t)i * 3;
    if (x < n && n <= SG_POS) {
        const tgo_task t = tasks[offs[g] + x];
        f[0] = feature_value(t.htd_ns);
        f[1] = feature_value(t.kern_ns);
        f[2] = feature_value(t.dth_ns);
    } else {
        f[0] = f[1] = f[2] = 0.f;
    }
}

// Group, size and ordering of row i: orders[i] (orders != null, group
// gid[i]) or sample (row mod spad) of group (row div spad) for row = row0 + i
// (samples >= S are padding: *ok = false, and the row's input is all zero).
__device__ __forceinline__ void row_order(const int32_t *__restrict__ offs, const uint32_t *__restrict__ gkeys,
                                          const uint8_t *__restrict__ orders, const int32_t *__restrict__ gid,
                                          int64_t i, int64_t row0, int64_t spad, int64_t S, uint64_t seed,
                                          int *gp, int *np, uint64_t *permp, bool *okp) {
    int g;
    uint64_t perm;
    int n;
    bool ok = true;
    if (orders) {
        g = gid[i];
        n = offs[g + 1] - offs[g];
        perm = 0;
        for (int p = SG_POS - 1; p >= 0; --p) perm = (perm << 4) | (uint64_t)(orders[i * SG_POS + p] & 15u);
    } else {
        const int64_t row = row0 + i;
        g = (int)(row / spad);
        const int64_t s = row % spad;
        n = offs[g + 1] - offs[g];
        ok = s < S && n >= 1 && n <= SG_POS;
        perm = ok ? sample_ordering(n, gkeys ? gkeys[g] : (uint32_t)g, (uint64_t)s, seed) : 0;
    }
    *gp = g;
    *np = n;
    *permp = perm;
    *okp = ok;
}

// float -> uint32 with the same order (top-k keys compare as integers)
__device__ __forceinline__ uint32_t orderable(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// --------------------------------------------------------- fused inference
// Wave-level sorting of 64-bit keys, lane i holding element i (64 lanes).
__device__ __forceinline__ unsigned long long shfl64(unsigned long long v, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return ((unsigned long long)hi << 32) | lo;
}
// Bitonic sort network, ascending.
__device__ __forceinline__ unsigned long long wave_sort64(unsigned long long v, int lane) {
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const unsigned long long o = shfl_xor64(v, j);
            const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
            v = keep_min ? (o < v ? o : v) : (o > v ? o : v);
        }
    return v;
}
// The 64 smallest of two ascending lists a and b, ascending: min(a[i],
// b[63 - i]) is a bitonic sequence holding them, which a half-cleaner
// cascade sorts.
__device__ __forceinline__ unsigned long long wave_merge_low64(unsigned long long a, unsigned long long b, int lane) {
    const unsigned long long br = shfl64(b, 63 - lane);
    unsigned long long v = a < br ? a : br;
#pragma unroll
    for (int j = 32; j > 0; j >>= 1) {
        const unsigned long long o = shfl_xor64(v, j);
        v = (lane & j) == 0 ? (o < v ? o : v) : (o > v ? o : v);
    }
    return v;
}

// One block scores FM_ROWS rows end to end: it builds their first-layer
// inputs in LDS, runs the three hidden layers on MFMA with the activations
// kept in LDS (rounded to bf16, as the layer-by-layer path stores them) and
// applies the head, so only the scores (or top-k keys) leave the block.  Each
// of the 8 waves computes 32 output columns of each layer for all rows as
// FM_RT x FM_CT MFMA tiles; weights (bf16, in the fragment order that
// pack_frag_kernel writes) come from global memory, where every block reads
// the same 282 KB.  The tiles are computed transposed
// (weights as the A operand, activations as B), so a lane's accumulator holds
// four consecutive output columns of one row: a layer's outputs leave in
// 8-byte LDS stores and the head reduces over four lanes per row.
constexpr int FM_ROWS = 128;
constexpr int FM_RT = FM_ROWS / 16;    // row tiles per block
constexpr int FM_LD = SG_H + 8;        // LDS row pitch in bf16
constexpr int FM_WAVES = 8;            // wave w owns output columns FM_CT * 16 * w ..
constexpr int FM_CT = SG_H / 16 / FM_WAVES;  // column tiles per wave
constexpr int FM_THREADS = 64 * FM_WAVES;
constexpr int FM_TPR = FM_THREADS / FM_ROWS;  // threads building one row's input
constexpr int FM_PPT = SG_POS / FM_TPR;       // positions per thread (3 features each)
static_assert(FM_TPR * FM_ROWS == FM_THREADS && FM_PPT * FM_TPR == SG_POS && FM_PPT % 2 == 0 &&
                  (SG_K0 / 2 - 3 * SG_POS / 2) % FM_TPR == 0 && FM_ROWS % 64 == 0,
              "input build: whole positions and padding words per thread, whole waves of rows");

template <int K>
__device__ __forceinline__ void fm_layer(const uint16_t (*Hs)[FM_LD], const uint16_t *__restrict__ W, int w, int l,
                                         f32x4 (&acc)[FM_RT][FM_CT]) {
#pragma unroll
    for (int a = 0; a < FM_RT; ++a)
#pragma unroll
        for (int b = 0; b < FM_CT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    // W in fragment order (pack_frag_kernel): fragment (column tile
    // FM_CT w + t, K step ks) of this lane at wf + (t KS + ks) 512
    constexpr int KS = K / GK;
    const uint16_t *wf = W + ((int64_t)FM_CT * w * KS * 64 + l) * 8;
    bf16x8 fb[FM_CT], nb[FM_CT];
#pragma unroll
    for (int t = 0; t < FM_CT; ++t) fb[t] = *reinterpret_cast<const bf16x8 *>(wf + (int64_t)t * KS * 512);
#pragma unroll 1
    for (int k0 = 0; k0 < K; k0 += GK) {
        if (k0 + GK < K) {
#pragma unroll
            for (int t = 0; t < FM_CT; ++t)
                nb[t] = *reinterpret_cast<const bf16x8 *>(wf + ((int64_t)t * KS + (k0 + GK) / GK) * 512);
        }
        bf16x8 fa[FM_RT];
#pragma unroll
        for (int t = 0; t < FM_RT; ++t)
            fa[t] = *reinterpret_cast<const bf16x8 *>(&Hs[16 * t + (l & 15)][k0 + (l >> 4) * 8]);
#pragma unroll
        for (int a = 0; a < FM_RT; ++a)
#pragma unroll
            for (int b = 0; b < FM_CT; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[b], fa[a], acc[a][b], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < FM_CT; ++t) fb[t] = nb[t];
    }
}

// relu(acc + bias) as bf16 into Hs (lane l holds columns
// 16 (FM_CT w + b) + 4(l/16) + i of row 16a + l%16)
__device__ __forceinline__ void fm_store(uint16_t (*Hs)[FM_LD], const float *__restrict__ bias, int w, int l,
                                         const f32x4 (&acc)[FM_RT][FM_CT]) {
#pragma unroll
    for (int b = 0; b < FM_CT; ++b) {
        const int c0 = 16 * (FM_CT * w + b) + 4 * (l >> 4);
        float bb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) bb[i] = bias[c0 + i];
#pragma unroll
        for (int a = 0; a < FM_RT; ++a) {
            uint32_t h[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float v = acc[a][b][i] + bb[i];
                h[i] = f2bf(v > 0.f ? v : 0.f);
            }
            *reinterpret_cast<uint2 *>(&Hs[16 * a + (l & 15)][c0]) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
        }
    }
}

// The three layers' bf16 weights ([out][in], W1 padded to SG_K0 inputs) in
// the fragment order mlp_fused_kernel reads: the B fragment of column tile ct
// and K step ks (16 output columns x GK inputs) is 64 lanes x 8 bf16 at
// ((ct K/GK + ks) 64 + lane) 8, lane l holding W[16 ct + l%16][GK ks +
// 8 (l/16) ..], so each of a wave's fragment loads reads 1 KB contiguously.
// Layers at 0, FM_WF1 and FM_WF1 + SG_H^2 of Wf.
constexpr int FM_WF1 = SG_H * SG_K0;
constexpr int FM_WF = FM_WF1 + 2 * SG_H * SG_H;
__global__ void pack_frag_kernel(const uint16_t *__restrict__ W1, const uint16_t *__restrict__ W2,
                                 const uint16_t *__restrict__ W3, uint16_t *__restrict__ Wf) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= FM_WF) return;
    const uint16_t *W = W3;
    int K = SG_H, q = e - FM_WF1 - SG_H * SG_H;
    if (e < FM_WF1) {
        W = W1;
        K = SG_K0;
        q = e;
    } else if (e < FM_WF1 + SG_H * SG_H) {
        W = W2;
        q = e - FM_WF1;
    }
    const int j = q & 7, lane = (q >> 3) & 63, frag = q >> 9;
    const int ks = frag % (K / GK), ct = frag / (K / GK);
    Wf[e] = W[(16 * ct + (lane & 15)) * K + GK * ks + 8 * (lane >> 4) + j];
}

// Rows are chosen as in features_kernel.  Output: score[i] (keys == null) or
// the top-k key of row i (keys != null: orderable score bits << 32 | sample
// index, ~0 for padding rows).
__global__ __launch_bounds__(FM_THREADS) void mlp_fused_kernel(const float *__restrict__ F,
                                                               const int32_t *__restrict__ offs,
                                                               const uint32_t *__restrict__ gkeys,
                                                               const uint8_t *__restrict__ orders,
                                                               const int32_t *__restrict__ gid, int64_t row0,
                                                               int64_t rows, int64_t spad, int64_t S, uint64_t seed,
                                                               const uint16_t *__restrict__ W1,
                                                               const uint16_t *__restrict__ W2,
                                                               const uint16_t *__restrict__ W3,
                                                               const float *__restrict__ p, float *score,
                                                               unsigned long long *keys) {
    __shared__ __align__(16) uint16_t Hs[FM_ROWS][FM_LD];
    __shared__ float part[FM_WAVES][FM_ROWS];
    __shared__ uint8_t okrow[FM_ROWS];
    __shared__ unsigned long long sperm[FM_ROWS];
    __shared__ int sgn[FM_ROWS];  // group << 5 | size, or -1: the row has no ordering
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int64_t base = (int64_t)blockIdx.x * FM_ROWS;
    // inputs: the first FM_ROWS threads draw each row's ordering, then
    // FM_TPR threads per row gather the features of FM_PPT positions each
    if (tid < FM_ROWS) {
        const int64_t i = base + tid;
        int g = 0, n = 0;
        uint64_t perm = 0;
        bool ok = false;
        if (i < rows) row_order(offs, gkeys, orders, gid, i, row0, spad, S, seed, &g, &n, &perm, &ok);
        okrow[tid] = ok ? 1 : 0;
        sperm[tid] = perm;
        sgn[tid] = ok ? (g << 5) | n : -1;
    }
    __syncthreads();
    {
        const int r = tid % FM_ROWS, q = tid / FM_ROWS;
        const int gn = sgn[r];
        uint32_t f[3 * FM_PPT];
#pragma unroll
        for (int c = 0; c < 3 * FM_PPT; ++c) f[c] = 0u;
        if (gn >= 0) {
            const int g = gn >> 5, n = gn & 31;
            const uint64_t perm = sperm[r];
            const float *Fg = F + (int64_t)g * SG_POS * 3;
#pragma unroll
            for (int h = 0; h < FM_PPT; ++h) {
                const int p = FM_PPT * q + h;
                if (p < n) {
                    const int t = (int)((perm >> (4 * p)) & 15u);
                    f[3 * h] = f2bf(Fg[t * 3]);
                    f[3 * h + 1] = f2bf(Fg[t * 3 + 1]);
                    f[3 * h + 2] = f2bf(Fg[t * 3 + 2]);
                }
            }
        }
        // features 3 FM_PPT q .. are words 3 FM_PPT q / 2 .. of the row; the
        // words after the 48 features are padding (a 64-wide first layer)
        uint32_t *row = reinterpret_cast<uint32_t *>(&Hs[r][0]);
#pragma unroll
        for (int c = 0; c < 3 * FM_PPT / 2; ++c) row[3 * FM_PPT / 2 * q + c] = f[2 * c] | (f[2 * c + 1] << 16);
        constexpr int PAD = (SG_K0 / 2 - 3 * SG_POS / 2) / FM_TPR;
#pragma unroll
        for (int c = 0; c < PAD; ++c) row[3 * SG_POS / 2 + PAD * q + c] = 0u;
    }
    __syncthreads();
    f32x4 acc[FM_RT][FM_CT];
    fm_layer<SG_K0>(Hs, W1, w, l, acc);
    __syncthreads();
    fm_store(Hs, p + SG_OFF_B1, w, l, acc);
    __syncthreads();
    fm_layer<SG_H>(Hs, W2, w, l, acc);
    __syncthreads();
    fm_store(Hs, p + SG_OFF_B2, w, l, acc);
    __syncthreads();
    fm_layer<SG_H>(Hs, W3, w, l, acc);
    // head on the bf16-rounded third layer: per-row partial sums over this
    // wave's columns, reduced across the 4 lanes that share a row
    float sum[FM_RT];
#pragma unroll
    for (int a = 0; a < FM_RT; ++a) sum[a] = 0.f;
#pragma unroll
    for (int b = 0; b < FM_CT; ++b) {
        const int c0 = 16 * (FM_CT * w + b) + 4 * (l >> 4);
        float bb[4], w4[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            bb[i] = p[SG_OFF_B3 + c0 + i];
            w4[i] = p[SG_OFF_W4 + c0 + i];
        }
#pragma unroll
        for (int a = 0; a < FM_RT; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float v = acc[a][b][i] + bb[i];
                sum[a] += bf2f(f2bf(v > 0.f ? v : 0.f)) * w4[i];
            }
    }
#pragma unroll
    for (int a = 0; a < FM_RT; ++a) {
        float v = sum[a];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (l < 16) part[w][16 * a + l] = v;
    }
    __syncthreads();
    if (tid < FM_ROWS) {  // one row per lane
        const int64_t i = base + tid;
        float sc = p[SG_OFF_B4];
#pragma unroll
        for (int v = 0; v < FM_WAVES; ++v) sc += part[v][tid];
        if (keys) {
            // each wave's 64 keys, sorted: the top-k passes take every 64
            // consecutive keys as an ascending list (rows past the end are
            // ~0, so the valid keys come first)
            unsigned long long key = ~0ull;
            if (i < rows && okrow[tid]) key = ((unsigned long long)orderable(sc) << 32) | (uint64_t)((row0 + i) % spad);
            key = wave_sort64(key, l);
            if (i < rows) keys[i] = key;
        } else if (i < rows) {
            score[i] = okrow[tid] ? sc : INFINITY;
        }
    }
}

// ---------------------------------------------------------------- training
// One training step is three kernels:
//   train_fwd_bwd_kernel  128 rows per block: features, the three hidden
//                         layers and the head on MFMA with the activations in
//                         LDS, the loss gradient, and back-propagation through
//                         layers 3 and 2, all without leaving the block.  It
//                         stores the bf16 activations and activation gradients
//                         transposed ([feature][row]) for the weight gradients,
//                         and per-block sums for the bias, head and loss terms.
//   train_wgrad_kernel    weight gradients G^T A of the three layers as one
//                         split-K launch (128 x 128 output tiles staged
//                         through LDS), plus the per-chunk sums of the
//                         per-block vectors; partials per K chunk in
//                         parameter order, no atomics (the sum order is fixed).
//   train_update_kernel   sums the K-chunk partials into the gradient and
//                         (optionally) applies Adam and refreshes the bf16
//                         weight copies.
// Every wave keeps the B operands of its 32 output columns of a whole layer
// in registers (64 VGPRs for K = 256), the next layer's loaded while the
// current one runs, so the MFMA loop reads only LDS.  Every weight a CU
// fetches serves the block's 128 rows (the weights are the kernel's largest
// memory stream).  Two LDS activation buffers of 128 rows suffice: the ReLU
// masks of layers 1 and 2, needed again by the backward pass, stay in
// registers as bits, because a lane owns the same (row, column) elements in
// every layer.
constexpr int TR_WAVES = 8;
constexpr int TR_THREADS = 64 * TR_WAVES;   // wave w owns output columns 32w .. 32w+31
constexpr int TR_RT = 8;                    // row tiles of 16
constexpr int TR_ROWS = 16 * TR_RT;         // rows per block
constexpr int TR_HALF = TR_RT / 2;          // row tiles per MFMA pass (two passes per layer)
constexpr int TR_LD = SG_H + 8;             // LDS pitch (bf16) of a 256-wide activation
constexpr int TR_LD0 = SG_K0 + 8;           // LDS pitch of the 64-wide input
// per-block vector: sums over the block's rows of the bias gradients of
// layers 1..3, the head weight and bias gradients, and the loss
constexpr int TR_V_B1 = 0, TR_V_B2 = 256, TR_V_B3 = 512, TR_V_W4 = 768, TR_V_B4 = 1024, TR_V_LOSS = 1025;
constexpr int TR_VLEN = 1026, TR_VSTRIDE = 1028;
constexpr int WG_BT = 128;                  // weight-gradient output tile: 128 x 128 (layer 1: 128 x 64)
constexpr int WG_TILES = 10;                // 4 (layer 3) + 4 (layer 2) + 2 (layer 1)
constexpr int WG_BK = 64;                   // rows (K) per LDS stage
constexpr int WG_LDK = WG_BK + 8;           // LDS pitch (bf16) of a staged operand row
constexpr int WG_VEC_BLOCKS = (TR_VLEN + 255) / 256;
constexpr int WG_KS_MAX = 64;               // K chunks (partials) at most
constexpr int WG_KC = 1024;                 // rows per K chunk (more for larger batches)
static_assert(TR_ROWS * SG_POS % TR_THREADS == 0, "features: whole passes of one thread per (row, position)");
static_assert(2 * TR_HALF * 2 * 4 == 64, "a lane's ReLU mask bits fill one 64-bit word");

// Block barrier that waits only for this wave's LDS accesses: __syncthreads()
// also waits for every outstanding global load and store, which would drain
// the next layer's weight loads and the activation stores at each layer.  The
// kernel below never reads global memory that it writes, so only LDS needs
// ordering here.
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Read for the tasks of an empty group (then masked), so that the feature
// loads need no branch.
__device__ const tgo_task ZERO_TASK = {0, 0, 0};

// A 64-bit value rotated right by R lanes within each row of 16 lanes (two
// DPP moves).
template <int R>
__device__ __forceinline__ int64_t row_ror64(int64_t v) {
    const uint64_t u = (uint64_t)v;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, 0x120 + R, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), 0x120 + R, 0xF, 0xF, false);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
// Sum / minimum over the 16 lanes of a row, left in every lane of the row.
__device__ __forceinline__ void row16_sum(int64_t &v) {
    v += row_ror64<8>(v);
    v += row_ror64<4>(v);
    v += row_ror64<2>(v);
    v += row_ror64<1>(v);
}
__device__ __forceinline__ void row16_min(int64_t &v) {
    int64_t t = row_ror64<8>(v);
    v = t < v ? t : v;
    t = row_ror64<4>(v);
    v = t < v ? t : v;
    t = row_ror64<2>(v);
    v = t < v ? t : v;
    t = row_ror64<1>(v);
    v = t < v ? t : v;
}

// Keeps the compiler from moving memory accesses across this point (no
// instruction): the next layer's weight loads stay behind the current layer,
// so that at most two layers' weights are live in registers.
__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

template <int K>
struct WRegs {
    bf16x8 v[K / GK][2];
};

// W: bf16 [256][K] output-major.  Wave w takes the B operands of output
// columns 32w + 16b + (l % 16), b = 0, 1, for every K step.
template <int K>
__device__ __forceinline__ void wload(WRegs<K> &t, const uint16_t *__restrict__ W, int w, int l) {
    const uint16_t *base = W + (int64_t)(32 * w + (l & 15)) * K + (l >> 4) * 8;
#pragma unroll
    for (int s = 0; s < K / GK; ++s)
#pragma unroll
        for (int b = 0; b < 2; ++b) t.v[s][b] = *reinterpret_cast<const bf16x8 *>(base + (int64_t)16 * b * K + GK * s);
}

// acc[a][b] = A[16(a0 + a) .. +15][0..K) x W[cols of tile b][0..K)^T; lane l
// ends with rows 16(a0 + a) + 4(l/16) + i, column 32w + 16b + l%16.
template <int K, int LD, int RA>
__device__ __forceinline__ void wmma_rows(const uint16_t (*A)[LD], int a0, const WRegs<K> &t, int l,
                                          f32x4 (&acc)[RA][2]) {
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < K / GK; ++s) {
        bf16x8 fa[RA];
#pragma unroll
        for (int a = 0; a < RA; ++a)
            fa[a] = *reinterpret_cast<const bf16x8 *>(&A[16 * (a0 + a) + (l & 15)][GK * s + (l >> 4) * 8]);
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], t.v[s][b], acc[a][b], 0, 0, 0);
    }
}

// Transposed store of an LDS activation block: dst[c][r0 + r] = S[r][c] for
// c < WIDTH, r < TR_ROWS (8 rows = 16 bytes per store).  The transposed
// arrays hold ld >= every row a block writes (see TR_LD_PAD), so no store
// needs a bounds test; stores without branches and with a fixed count let
// the compiler wait for exactly the loads it needs later, instead of for
// every outstanding memory operation.
template <int WIDTH, int LD>
__device__ __forceinline__ void store_t(const uint16_t (*S)[LD], uint16_t *dst, int64_t ld, int r0, int tid) {
    constexpr int chunks = WIDTH * (TR_ROWS / 8);
    static_assert(chunks % TR_THREADS == 0, "whole passes");
#pragma unroll
    for (int qq = 0; qq < chunks / TR_THREADS; ++qq) {
        const int q = tid + qq * TR_THREADS;
        const int c = q / (TR_ROWS / 8), r = (q % (TR_ROWS / 8)) * 8;
        uint4 v;
        v.x = S[r][c] | ((uint32_t)S[r + 1][c] << 16);
        v.y = S[r + 2][c] | ((uint32_t)S[r + 3][c] << 16);
        v.z = S[r + 4][c] | ((uint32_t)S[r + 5][c] << 16);
        v.w = S[r + 6][c] | ((uint32_t)S[r + 7][c] << 16);
        *reinterpret_cast<uint4 *>(dst + (int64_t)c * ld + r0 + r) = v;
    }
}

// The four values a lane holds for (row tile a, column col) are rows
// 16a + 4(l/16) + 0..3 of that column: one 8-byte store into the transposed
// layout dst[col][row] (every row a block writes lies below ld).
__device__ __forceinline__ void store4_t(uint16_t *dst, int64_t ld, int col, int row0, const uint16_t (&v)[4]) {
    uint2 q;
    q.x = v[0] | ((uint32_t)v[1] << 16);
    q.y = v[2] | ((uint32_t)v[3] << 16);
    *reinterpret_cast<uint2 *>(dst + (int64_t)col * ld + row0) = q;
}

// Sum over the rows a lane holds (4 per row tile) and over the lanes that
// share its column (l, l ^ 16, l ^ 32, l ^ 48); lanes l < 16 end with the
// column total.
__device__ __forceinline__ float col_total(float v) {
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    return v;
}

// Forward and backward of the rows [128 blockIdx.x, +128).  Rows >= `rows`
// carry zero features and zero loss gradient.  inv_rows = 1 / rows.
// LDS: bufA holds h1, then h3 and, in place, dL/dz3; bufB holds the input
// features, then h2, then dL/dz2.
__global__ __launch_bounds__(TR_THREADS) void train_fwd_bwd_kernel(
    const tgo_task *__restrict__ tasks, const int32_t *__restrict__ offs, const uint8_t *__restrict__ orders,
    const int32_t *__restrict__ gid, const int64_t *__restrict__ T, int rows, float inv_rows,
    const uint16_t *__restrict__ W1, const uint16_t *__restrict__ W2, const uint16_t *__restrict__ W3,
    const uint16_t *__restrict__ W2t, const uint16_t *__restrict__ W3t, const float *__restrict__ p, int64_t ld,
    uint16_t *Xt, uint16_t *H1t, uint16_t *H2t, uint16_t *G3t, uint16_t *G2t, uint16_t *G1t, float *vec,
    uint16_t *H3keep, float *score_keep) {
    __shared__ __align__(16) uint16_t bufA[TR_ROWS][TR_LD];
    __shared__ __align__(16) uint16_t bufB[TR_ROWS][TR_LD];
    __shared__ float part[TR_WAVES][TR_ROWS];
    __shared__ float ys[TR_ROWS], dss[TR_ROWS];
    uint16_t (*Xs)[TR_LD0] = reinterpret_cast<uint16_t (*)[TR_LD0]>(&bufB[0][0]);
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int r0 = blockIdx.x * TR_ROWS;
    float *vb = vec + (int64_t)blockIdx.x * TR_VSTRIDE;
    // the row a lane's element (pass h, row tile a, value i) belongs to, and
    // the bit of that element in the lane's ReLU masks
#define TR_ROW(h, a, i) (16 * ((h) * TR_HALF + (a)) + 4 * (l >> 4) + (i))
#define TR_BIT(h, a, b, i) ((((h) * TR_HALF + (a)) * 2 + (b)) * 4 + (i))

    // biases and head weights of this lane's two columns
    float bias1[2], bias2[2], bias3[2], w4c[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int col = 32 * w + 16 * b + (l & 15);
        bias1[b] = p[SG_OFF_B1 + col];
        bias2[b] = p[SG_OFF_B2 + col];
        bias3[b] = p[SG_OFF_B3 + col];
        w4c[b] = p[SG_OFF_W4 + col];
    }
    const float bias4 = p[SG_OFF_B4];

    // features of (row, position) and the target of each row, 32 rows per
    // pass.  The 16 lanes of a row also hold the group's tasks (lane x: task
    // x) for the target's lower bound, reduced across the row's lanes.  The
    // loads come at three dependent levels (row -> group -> tasks), each
    // issued for all passes at once and without branches (indices clamped
    // into range, results selected), so their latencies overlap.
    constexpr int FP = TR_ROWS * SG_POS / TR_THREADS;  // passes
    const int pos = tid & 15;
    int gv[FP], xv[FP], bv[FP], nv[FP];
    int64_t Tv[FP];
#pragma unroll
    for (int it = 0; it < FP; ++it) {
        const int i = r0 + 32 * it + (tid >> 4);
        const int ic = i < rows ? i : rows - 1;
        gv[it] = gid[ic];
        xv[it] = orders[(int64_t)ic * SG_POS + pos];
        Tv[it] = T[ic];
    }
#pragma unroll
    for (int it = 0; it < FP; ++it) {
        bv[it] = offs[gv[it]];
        nv[it] = offs[gv[it] + 1] - bv[it];
    }
    tgo_task tx[FP], tp[FP];
#pragma unroll
    for (int it = 0; it < FP; ++it) {
        // an index past the group reads its first task (an empty group: a
        // zero task), masked below
        const int n = nv[it];
        const tgo_task *g0 = n > 0 ? tasks + bv[it] : &ZERO_TASK;
        tx[it] = g0[xv[it] < n ? xv[it] : 0];
        tp[it] = g0[pos < n ? pos : 0];
    }
#pragma unroll
    for (int it = 0; it < FP; ++it) {
        const int rr = 32 * it + (tid >> 4);
        const bool live = r0 + rr < rows;
        const int n = live ? nv[it] : 0;
        const bool has = pos < n && xv[it] < n;
        const tgo_task t = tx[it];
        const uint16_t f0 = has ? f2bf(feature_value(t.htd_ns)) : (uint16_t)0;
        const uint16_t f1 = has ? f2bf(feature_value(t.kern_ns)) : (uint16_t)0;
        const uint16_t f2 = has ? f2bf(feature_value(t.dth_ns)) : (uint16_t)0;
        // y = T / LB - 1, LB the largest machine lower bound of the group
        const bool own = pos < n;
        const tgo_task u = tp[it];
        int64_t sh = own ? u.htd_ns : 0, sk = own ? u.kern_ns : 0, sd = own ? u.dth_ns : 0;
        int64_t mh = own ? u.htd_ns : INT64_MAX, md = own ? u.dth_ns : INT64_MAX;
        int64_t mkd = own ? u.kern_ns + u.dth_ns : INT64_MAX, mhk = own ? u.htd_ns + u.kern_ns : INT64_MAX;
        row16_sum(sh);
        row16_sum(sk);
        row16_sum(sd);
        row16_min(mh);
        row16_min(md);
        row16_min(mkd);
        row16_min(mhk);
        if (pos == 0) {
            int64_t lb = sh + mkd;
            lb = mh + sk + md > lb ? mh + sk + md : lb;
            lb = mhk + sd > lb ? mhk + sd : lb;
            lb = lb < 1 ? 1 : lb;
            ys[rr] = live ? (float)((double)Tv[it] / (double)lb - 1.0) : 0.f;
        }
        Xs[rr][3 * pos] = f0;
        Xs[rr][3 * pos + 1] = f1;
        Xs[rr][3 * pos + 2] = f2;
        Xs[rr][SG_FEAT + pos] = 0;
    }
    // the first two layers' weights are loaded once the features are built
    // (vector memory returns in order: loads issued before the features'
    // own would hold them up)
    compiler_fence();
    WRegs<SG_K0> w1r;
    wload(w1r, W1, w, l);
    WRegs<SG_H> w2r;
    wload(w2r, W2, w, l);
    lds_barrier();
    store_t<SG_K0>(Xs, Xt, ld, r0, tid);

    uint64_t m1 = 0, m2 = 0;  // ReLU masks of layers 1 and 2 (bit TR_BIT: h > 0)
    // layer 1: Xs -> bufA
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
        f32x4 acc[TR_HALF][2];
        wmma_rows<SG_K0, TR_LD0, TR_HALF>(Xs, h * TR_HALF, w1r, l, acc);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int col = 32 * w + 16 * b + (l & 15);
#pragma unroll
            for (int a = 0; a < TR_HALF; ++a) {
                uint16_t hv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float v = acc[a][b][i] + bias1[b];
                    hv[i] = f2bf(v > 0.f ? v : 0.f);
                    bufA[TR_ROW(h, a, i)][col] = hv[i];
                    m1 |= (uint64_t)(hv[i] != 0) << TR_BIT(h, a, b, i);
                }
                store4_t(H1t, ld, col, r0 + TR_ROW(h, a, 0), hv);
            }
        }
    }
    compiler_fence();  // the next layer's weights load only once this layer is done
    WRegs<SG_H> w3r;
    wload(w3r, W3, w, l);
    lds_barrier();
    // layer 2: bufA -> bufB (the input features are no longer read)
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
        f32x4 acc[TR_HALF][2];
        wmma_rows<SG_H, TR_LD, TR_HALF>(bufA, h * TR_HALF, w2r, l, acc);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int col = 32 * w + 16 * b + (l & 15);
#pragma unroll
            for (int a = 0; a < TR_HALF; ++a) {
                uint16_t hv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float v = acc[a][b][i] + bias2[b];
                    hv[i] = f2bf(v > 0.f ? v : 0.f);
                    bufB[TR_ROW(h, a, i)][col] = hv[i];
                    m2 |= (uint64_t)(hv[i] != 0) << TR_BIT(h, a, b, i);
                }
                store4_t(H2t, ld, col, r0 + TR_ROW(h, a, 0), hv);
            }
        }
    }
    compiler_fence();  // the next layer's weights load only once this layer is done
    WRegs<SG_H> w3tr;
    wload(w3tr, W3t, w, l);
    lds_barrier();
    // layer 3: bufB -> bufA (h1 is no longer read: its mask is in m1), and
    // the head's per-wave row sums
#pragma unroll 1
    for (int h = 0; h < 2; ++h) {
        f32x4 acc[TR_HALF][2];
        wmma_rows<SG_H, TR_LD, TR_HALF>(bufB, h * TR_HALF, w3r, l, acc);
#pragma unroll
        for (int a = 0; a < TR_HALF; ++a) {
            float sum[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int col = 32 * w + 16 * b + (l & 15);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float v = acc[a][b][i] + bias3[b];
                    const uint16_t hq = f2bf(v > 0.f ? v : 0.f);
                    bufA[TR_ROW(h, a, i)][col] = hq;
                    sum[i] += bf2f(hq) * w4c[b];
                    if (H3keep) {
                        const int row = r0 + TR_ROW(h, a, i);
                        if (row < rows) H3keep[(int64_t)row * SG_H + col] = hq;
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float v = sum[i];
                for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m);
                if ((l & 15) == 0) part[w][TR_ROW(h, a, i)] = v;
            }
        }
    }
    compiler_fence();  // the next layer's weights load only once this layer is done
    WRegs<SG_H> w2tr;
    wload(w2tr, W2t, w, l);
    lds_barrier();
    // scores, loss gradient and loss (wave 0: rows l and l + 64)
    if (w == 0) {
        float e = 0.f, dsum = 0.f;
#pragma unroll
        for (int q = 0; q < TR_ROWS / 64; ++q) {
            const int row = l + 64 * q, i = r0 + row;
            float sc = bias4;
#pragma unroll
            for (int v = 0; v < TR_WAVES; ++v) sc += part[v][row];
            float ds = 0.f;
            if (i < rows) {
                const float d = sc - ys[row];
                ds = 2.f * d * inv_rows;
                e += d * d * inv_rows;
                if (score_keep) score_keep[i] = sc;
            }
            dss[row] = ds;
            dsum += ds;
        }
        for (int m = 32; m >= 1; m >>= 1) {
            e += __shfl_xor(e, m);
            dsum += __shfl_xor(dsum, m);
        }
        if (l == 0) {
            vb[TR_V_LOSS] = e;
            vb[TR_V_B4] = dsum;
        }
    }
    lds_barrier();
    // dL/dz3 = ds w4 where h3 > 0, in place of h3 in bufA; head and layer-3 bias sums
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int col = 32 * w + 16 * b + (l & 15);
        float gw4 = 0.f, gb3 = 0.f;
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int a = 0; a < TR_HALF; ++a) {
                uint16_t gv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = TR_ROW(h, a, i);
                    const float ds = dss[row];
                    const float hf = bf2f(bufA[row][col]);
                    const uint16_t g = hf > 0.f ? f2bf(ds * w4c[b]) : (uint16_t)0;
                    gv[i] = g;
                    bufA[row][col] = g;
                    gw4 += ds * hf;
                    gb3 += bf2f(g);
                }
                store4_t(G3t, ld, col, r0 + TR_ROW(h, a, 0), gv);
            }
        gw4 = col_total(gw4);
        gb3 = col_total(gb3);
        if (l < 16) {
            vb[TR_V_W4 + col] = gw4;
            vb[TR_V_B3 + col] = gb3;
        }
    }
    lds_barrier();
    // dL/dz2 = (dL/dz3 W3) where h2 > 0: bufA -> bufB (h2 is no longer read)
    {
        float gb[2] = {0.f, 0.f};
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            f32x4 acc[TR_HALF][2];
            wmma_rows<SG_H, TR_LD, TR_HALF>(bufA, h * TR_HALF, w3tr, l, acc);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int col = 32 * w + 16 * b + (l & 15);
#pragma unroll
                for (int a = 0; a < TR_HALF; ++a) {
                    uint16_t gv[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const uint16_t g = (m2 >> TR_BIT(h, a, b, i)) & 1 ? f2bf(acc[a][b][i]) : (uint16_t)0;
                        gv[i] = g;
                        bufB[TR_ROW(h, a, i)][col] = g;
                        gb[b] += bf2f(g);
                    }
                    store4_t(G2t, ld, col, r0 + TR_ROW(h, a, 0), gv);
                }
            }
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const float t = col_total(gb[b]);
            if (l < 16) vb[TR_V_B2 + 32 * w + 16 * b + l] = t;
        }
    }
    lds_barrier();
    // dL/dz1 = (dL/dz2 W2) where h1 > 0, from bufB; stored only
    {
        float gb[2] = {0.f, 0.f};
#pragma unroll 1
        for (int h = 0; h < 2; ++h) {
            f32x4 acc[TR_HALF][2];
            wmma_rows<SG_H, TR_LD, TR_HALF>(bufB, h * TR_HALF, w2tr, l, acc);
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int col = 32 * w + 16 * b + (l & 15);
#pragma unroll
                for (int a = 0; a < TR_HALF; ++a) {
                    uint16_t gv[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const uint16_t g = (m1 >> TR_BIT(h, a, b, i)) & 1 ? f2bf(acc[a][b][i]) : (uint16_t)0;
                        gv[i] = g;
                        gb[b] += bf2f(g);
                    }
                    store4_t(G1t, ld, col, r0 + TR_ROW(h, a, 0), gv);
                }
            }
        }
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const float t = col_total(gb[b]);
            if (l < 16) vb[TR_V_B1 + 32 * w + 16 * b + l] = t;
        }
    }
#undef TR_ROW
#undef TR_BIT
}

// src[0] + src[stride] + ... + src[(ks - 1) stride], added in that order, with
// the loads issued eight at a time.
__device__ __forceinline__ float chunk_sum(const float *__restrict__ src, int64_t stride, int ks) {
    float s = 0.f;
    int c = 0;
    for (; c + 8 <= ks; c += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = src[(int64_t)(c + u) * stride];
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; c < ks; ++c) s += src[(int64_t)c * stride];
    return s;
}

// One LDS stage of the weight-gradient kernel: rows cr + 32q (q < 4) of the
// G and A feature blocks, 8 K values from k on, one 16-byte load each (A rows
// at or past na are zero).  The staging arrays use a native vector type: with
// HIP's uint4 (a struct) the compiler kept them in scratch memory.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void wg_fetch(u32x4 (&rg)[4], u32x4 (&ra)[4], const uint16_t *gsrc, const uint16_t *asrc,
                                         int64_t ld, int64_t k, int cr, int na) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        rg[q] = *reinterpret_cast<const u32x4 *>(gsrc + (int64_t)32 * q * ld + k);
        ra[q] = 32 * q + cr < na ? *reinterpret_cast<const u32x4 *>(asrc + (int64_t)32 * q * ld + k) : u32x4{0, 0, 0, 0};
    }
}
__device__ __forceinline__ void wg_stash(const u32x4 (&rg)[4], const u32x4 (&ra)[4], uint16_t (*sg)[WG_LDK],
                                         uint16_t (*sa)[WG_LDK], int cr, int ck) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        *reinterpret_cast<u32x4 *>(&sg[32 * q + cr][ck]) = rg[q];
        *reinterpret_cast<u32x4 *>(&sa[32 * q + cr][ck]) = ra[q];
    }
}

// The MFMAs of one LDS stage: this wave's 64 x 64 quarter (rows 64 wo.., columns
// 64 wi..) over the stage's 64 K values.
__device__ __forceinline__ void wg_mma(f32x4 (&acc)[4][4], const uint16_t (*sg)[WG_LDK], const uint16_t (*sa)[WG_LDK],
                                       int wo, int wi, int l) {
#pragma unroll
    for (int kk = 0; kk < WG_BK / GK; ++kk) {
        bf16x8 fg[4], fa[4];
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            fg[x] = *reinterpret_cast<const bf16x8 *>(&sg[64 * wo + 16 * x + (l & 15)][GK * kk + (l >> 4) * 8]);
            fa[x] = *reinterpret_cast<const bf16x8 *>(&sa[64 * wi + 16 * x + (l & 15)][GK * kk + (l >> 4) * 8]);
        }
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fg[x], fa[y], acc[x][y], 0, 0, 0);
    }
}

// Weight gradients dW[o][i] = sum over rows of G[r][o] A[r][i] for the three
// layers (A = X, h1, h2; G = dL/dz1..3), one 128 x 128 output tile (layer 1:
// 128 x 64) and one K chunk of kc rows per block, written as a partial in
// parameter order (wpart[chunk][parameter]); blockIdx maps to tile 0..3
// (layer 3), 4..7 (layer 2), 8..9 (layer 1) or WG_TILES + j for the
// per-block vectors (entries 256j .. 256j+255 summed over the chunk's row
// blocks into the bias, head and loss entries).  Work items (chunk, tile) map
// to blocks so that every item of a chunk runs on one XCD: blocks are handed
// to the 8 XCDs in turn (block b to XCD b % 8), and XCD x takes the chunks
// x, x + 8, ...; the chunk's rows of the six activation arrays are then
// fetched into that XCD's L2 once.
// Both operands are K-contiguous in HBM ([feature][row]); a stage of 64 rows
// of both is copied into LDS with whole 128-byte lines per feature (double
// buffered, with the loads two stages ahead in flight), and each of the four
// waves computes a 64 x 64 quarter of the tile from LDS.
__global__ __launch_bounds__(256) void train_wgrad_kernel(
    const uint16_t *__restrict__ Xt, const uint16_t *__restrict__ H1t, const uint16_t *__restrict__ H2t,
    const uint16_t *__restrict__ G1t, const uint16_t *__restrict__ G2t, const uint16_t *__restrict__ G3t,
    int64_t ld, int rows, int kc, const float *__restrict__ vec, float *wpart, float *vpart) {
    constexpr int ITEMS = WG_TILES + WG_VEC_BLOCKS;
    const int xcd = blockIdx.x % 8, j = blockIdx.x / 8;
    const int chunk = xcd + 8 * (j / ITEMS), tile = j % ITEMS;
    const int ks = (rows + kc - 1) / kc;
    if (chunk >= ks) return;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int k0 = chunk * kc, k1 = min(rows, k0 + kc);
    float *wp = wpart + (int64_t)chunk * SG_NPARAM;
    if (tile >= WG_TILES) {
        const int e = (tile - WG_TILES) * 256 + tid;
        if (e < TR_VLEN) {
            const int b0 = k0 / TR_ROWS, b1 = (k1 + TR_ROWS - 1) / TR_ROWS;
            const float v = chunk_sum(vec + (int64_t)b0 * TR_VSTRIDE + e, TR_VSTRIDE, b1 - b0);
            if (e == TR_V_LOSS) vpart[chunk] = v;
            else if (e == TR_V_B4) wp[SG_OFF_B4] = v;
            else if (e >= TR_V_W4) wp[SG_OFF_W4 + (e - TR_V_W4)] = v;
            else if (e >= TR_V_B3) wp[SG_OFF_B3 + (e - TR_V_B3)] = v;
            else if (e >= TR_V_B2) wp[SG_OFF_B2 + (e - TR_V_B2)] = v;
            else wp[SG_OFF_B1 + (e - TR_V_B1)] = v;
        }
        return;
    }
    __shared__ __align__(16) uint16_t sG[2][WG_BT][WG_LDK];
    __shared__ __align__(16) uint16_t sA[2][WG_BT][WG_LDK];
    const uint16_t *G, *A;
    int tm, tn, na;  // output rows 128 tm.., columns 128 tn.., na columns in the tile
    if (tile < 4) {
        G = G3t; A = H2t; tm = tile >> 1; tn = tile & 1; na = WG_BT;
    } else if (tile < 8) {
        G = G2t; A = H1t; tm = (tile - 4) >> 1; tn = (tile - 4) & 1; na = WG_BT;
    } else {
        G = G1t; A = Xt; tm = tile - 8; tn = 0; na = SG_K0;
    }
    // copy of one stage: 128 feature rows x 64 K of each operand, 16 bytes per
    // thread and step; thread t takes feature row t/8 + 32s, K offset 8 (t%8)
    const int cr = tid >> 3, ck = (tid & 7) * 8;
    const uint16_t *gsrc = G + (int64_t)(WG_BT * tm + cr) * ld + ck;
    const uint16_t *asrc = A + (int64_t)(WG_BT * tn + cr) * ld + ck;
    const int nstage = (k1 - k0 + WG_BK - 1) / WG_BK;
    u32x4 rg[4], ra[4];
    const int wo = w >> 1, wi = w & 1;  // this wave's 64 x 64 quarter
    const bool active = 64 * wi < na;
    f32x4 acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
    // a last partial stage reads rows up to the next multiple of 64, which
    // the forward kernel wrote (zero gradients) and which lie below ld.
    // Two register sets alternate: the loads of stage s + 2 are issued before
    // the MFMAs of stage s, and land in LDS after those of stage s + 1.
    u32x4 rg2[4], ra2[4];
    wg_fetch(rg, ra, gsrc, asrc, ld, k0, cr, na);
    wg_stash(rg, ra, sG[0], sA[0], cr, ck);
    if (1 < nstage) wg_fetch(rg2, ra2, gsrc, asrc, ld, k0 + WG_BK, cr, na);
    __syncthreads();
    for (int st = 0; st < nstage; st += 2) {
        if (st + 2 < nstage) wg_fetch(rg, ra, gsrc, asrc, ld, k0 + (int64_t)(st + 2) * WG_BK, cr, na);
        if (active) wg_mma(acc, sG[0], sA[0], wo, wi, l);
        if (st + 1 < nstage) wg_stash(rg2, ra2, sG[1], sA[1], cr, ck);
        __syncthreads();
        if (st + 1 >= nstage) break;
        if (st + 3 < nstage) wg_fetch(rg2, ra2, gsrc, asrc, ld, k0 + (int64_t)(st + 3) * WG_BK, cr, na);
        if (active) wg_mma(acc, sG[1], sA[1], wo, wi, l);
        if (st + 2 < nstage) wg_stash(rg, ra, sG[0], sA[0], cr, ck);
        __syncthreads();
    }
    if (!active) return;
    // lane l holds rows 4(l/16) + i, column l%16 of each 16 x 16 sub-tile
    float *dst = wp + (tile < 4 ? SG_OFF_W3 : tile < 8 ? SG_OFF_W2 : SG_OFF_W1);
    const int pitch = tile < 8 ? SG_H : SG_FEAT;
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int c = WG_BT * tn + 64 * wi + 16 * y + (l & 15);
            if (c < pitch) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int o = WG_BT * tm + 64 * wo + 16 * x + 4 * (l >> 4) + i;
                    dst[o * pitch + c] = acc[x][y][i];
                }
            }
        }
}

// Adam on the float32 masters (bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t)
// (omb1 = 1 - beta1 and omb2 = 1 - beta2 are rounded from double on the host:
// 1 - 0.999f in float32 would be 1.3e-5 off 0.001)
struct AdamArgs {
    float lr, beta1, beta2, eps, c1, c2, omb1, omb2;
};

// mode 0: gradient only (sum the chunk partials into g);
// mode 1: that, then Adam and the bf16 copies; mode 2: Adam on the given
// gradient gin.  Block 0 also writes the loss (modes 0, 1).
__global__ void train_update_kernel(int mode, const float *__restrict__ wpart, const float *__restrict__ vpart,
                                    int ks, const float *__restrict__ gin, float *p, float *g, float *m, float *v,
                                    AdamArgs a, float *loss, uint16_t *W1, uint16_t *W2, uint16_t *W2t,
                                    uint16_t *W3, uint16_t *W3t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (mode != 2 && i == 0) *loss = chunk_sum(vpart, 1, ks);
    if (i >= SG_NPARAM) return;
    float gi;
    if (mode == 2) {
        gi = gin[i];
    } else {
        gi = chunk_sum(wpart + i, SG_NPARAM, ks);
        g[i] = gi;
    }
    if (mode == 0) return;
    const float mi = a.beta1 * m[i] + a.omb1 * gi;
    const float vi = a.beta2 * v[i] + a.omb2 * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
    p[i] = pi;
    const uint16_t bb = f2bf(pi);
    if (i < SG_OFF_B1) {
        W1[(i / SG_FEAT) * SG_K0 + i % SG_FEAT] = bb;
    } else if (i >= SG_OFF_W2 && i < SG_OFF_B2) {
        const int j = i - SG_OFF_W2;
        W2[j] = bb;
        W2t[(j % SG_H) * SG_H + j / SG_H] = bb;
    } else if (i >= SG_OFF_W3 && i < SG_OFF_B3) {
        const int j = i - SG_OFF_W3;
        W3[j] = bb;
        W3t[(j % SG_H) * SG_H + j / SG_H] = bb;
    }
}

__global__ void refresh_bf16_kernel(const float *__restrict__ p, uint16_t *W1, uint16_t *W2, uint16_t *W2t,
                                    uint16_t *W3, uint16_t *W3t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < SG_H * SG_K0) {
        const int o = i / SG_K0, c = i % SG_K0;
        W1[o * SG_K0 + c] = c < SG_FEAT ? f2bf(p[SG_OFF_W1 + o * SG_FEAT + c]) : (uint16_t)0;
    }
    if (i < SG_H * SG_H) {
        const int o = i / SG_H, c = i % SG_H;
        const uint16_t b2 = f2bf(p[SG_OFF_W2 + i]);
        const uint16_t b3 = f2bf(p[SG_OFF_W3 + i]);
        W2[i] = b2;
        W2t[c * SG_H + o] = b2;
        W3[i] = b3;
        W3t[c * SG_H + o] = b3;
    }
}

// He-uniform initialisation from Philox(seed, parameter index)
__global__ void init_params_kernel(float *p, uint64_t seed) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= SG_NPARAM) return;
    float bound = 0.f;
    if (i < SG_OFF_B1) bound = sqrtf(6.f / SG_FEAT);
    else if (i >= SG_OFF_W2 && i < SG_OFF_B2) bound = sqrtf(6.f / SG_H);
    else if (i >= SG_OFF_W3 && i < SG_OFF_B3) bound = sqrtf(6.f / SG_H);
    else if (i >= SG_OFF_W4 && i < SG_OFF_B4) bound = sqrtf(6.f / SG_H);
    U4 c;
    c.x = (uint32_t)i;
    c.y = 0x5EEDu;
    c.z = 0;
    c.w = 0;
    const U4 u = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const float unit = (float)(u.x >> 8) * (1.0f / 16777216.0f);  // [0, 1)
    p[i] = bound * (2.f * unit - 1.f);
}

// ------------------------------------------------------------------ top-k
// Keys (orderable score bits << 32 | sample index) per group; each pass keeps
// the 64 smallest of every run of 1024 keys.  A run is 16 ascending lists of
// 64 keys (the scoring kernel sorts each block's 64 keys; a pass writes its
// 64 ascending); the 8 waves of a block merge pairs of lists in a tree
// (16 -> 8 -> 4 -> 2 -> 1), keeping the lower 64 at each merge.
constexpr int TK_RUN = 1024;
constexpr int TK_THREADS = 512;
constexpr int TK_KEEP = 64;
static_assert(TK_THREADS == 64 * (TK_RUN / 128), "one wave per pair of lists");

// in: [G][len] keys (group stride in_stride); out: [G][ceil(len/TK_RUN)*64]
__global__ __launch_bounds__(TK_THREADS) void topk_pass_kernel(const unsigned long long *__restrict__ in,
                                                         int64_t in_stride, int64_t len, int runs,
                                                         unsigned long long *out, int64_t out_stride) {
    __shared__ unsigned long long s[TK_RUN / 128][TK_KEEP];
    const int g = blockIdx.y, run = blockIdx.x;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const unsigned long long *src = in + (int64_t)g * in_stride;
    const int64_t ia = (int64_t)run * TK_RUN + 128 * w + lane, ib = ia + 64;
    const unsigned long long a = ia < len ? src[ia] : ~0ull;
    const unsigned long long b = ib < len ? src[ib] : ~0ull;
    unsigned long long v = wave_merge_low64(a, b, lane);
    s[w][lane] = v;
    __syncthreads();
#pragma unroll
    for (int nl = TK_RUN / 256; nl >= 1; nl >>= 1) {
        if (w < nl) v = wave_merge_low64(s[2 * w][lane], s[2 * w + 1][lane], lane);
        __syncthreads();
        if (w < nl) s[w][lane] = v;
        __syncthreads();
    }
    if (w == 0) out[(int64_t)g * out_stride + (int64_t)run * TK_KEEP + lane] = v;
}

__global__ void fill_u64_kernel(unsigned long long *p, int64_t n, unsigned long long v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// results: best of candidates (exact) and the heuristic
// Results: best of candidates (exact) and the heuristic.  The candidates'
// best (T, sample) of group g comes from pairs[g] (re-score), or, for the
// plain search, from the packed key best[g] (32-bit path) or the chunk
// partials wpart[g][0 .. wchunks) (64-bit path).
__global__ void search_finish_kernel(const int32_t *__restrict__ offs, int G, uint64_t seed,
                                     const uint32_t *__restrict__ gkeys,
                                     const int32_t *__restrict__ mode,
                                     const BestPair *__restrict__ pairs,
                                     const unsigned long long *__restrict__ best,
                                     const BestPair *__restrict__ wpart, int wchunks,
                                     const uint8_t *__restrict__ horders, const int64_t *__restrict__ hns,
                                     tgo_search_result *out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    tgo_search_result r;
    const int n = offs[g + 1] - offs[g];
    const int md = mode[g];
    r.n = n;
    r.status = md < 0 ? md : 0;
    r.pad = 0;
    for (int i = 0; i < 16; ++i) r.best[i] = 0xff;
    r.heur_ns = hns[g];
    uint64_t ct = ~0ull, cs = ~0ull;
    if (md >= 0) {
        if (pairs) {
            ct = pairs[g].t;
            cs = pairs[g].s;
        } else if (md == 0) {
            if (best[g] != ~0ull) {
                ct = best[g] >> 32;
                cs = best[g] & 0xffffffffull;
            }
        } else {
            for (int c = 0; c < wchunks; ++c) {
                const BestPair q = wpart[(int64_t)g * RS_WIDE_CHUNKS + c];
                pair_min(ct, cs, q.t, q.s);
            }
        }
    }
    if (r.status != 0 || ct == ~0ull) {
        r.best_ns = r.status != 0 ? r.status : r.heur_ns;
        r.cand_best_ns = -1;
        r.best_sample = 0;
        r.from_heuristic = r.status != 0 ? 0 : 1;
        if (r.status == 0)
            for (int i = 0; i < n; ++i) r.best[i] = horders[(int64_t)g * 16 + i];
        out[g] = r;
        return;
    }
    const int64_t cT = (int64_t)ct;
    r.cand_best_ns = cT;
    r.best_sample = cs;
    if (r.heur_ns >= 0 && r.heur_ns <= cT) {
        r.best_ns = r.heur_ns;
        r.from_heuristic = 1;
        for (int i = 0; i < n; ++i) r.best[i] = horders[(int64_t)g * 16 + i];
    } else {
        r.best_ns = cT;
        r.from_heuristic = 0;
        const uint64_t perm = sample_ordering(n, gkeys ? gkeys[g] : (uint32_t)g, cs, seed);
        for (int i = 0; i < n; ++i) r.best[i] = (uint8_t)((perm >> (4 * i)) & 15u);
    }
    out[g] = r;
}

}  // namespace tgo

// ------------------------------------------------------------------- host

// Leading dimension of the transposed activation arrays ([feature][row]):
// max_rows plus 2,176 elements (4 KiB + 256 B per feature row), so that the
// rows a wave touches in one access, whose stride would otherwise be a power
// of two (e.g. 128 KiB at 65,536 rows), spread over the L2 and HBM channels
// instead of landing on one.  The pad also covers the rows of the last
// 128-row block past max_rows (max_rows is a multiple of 64), which the
// forward kernel writes unconditionally.
constexpr int64_t TR_LD_PAD = 2176;
static_assert(TR_LD_PAD >= tgo::TR_ROWS - 64, "the last block's rows lie inside the transposed arrays");

struct tgo_surrogate {
    int device = 0;
    int64_t max_rows = 0;
    int64_t search_rows = 0;  // rows scored per launch of the search (a multiple of the top-k run)
    int64_t ldt = 0;  // max_rows + TR_LD_PAD
    int64_t step = 0;
    void *mem = nullptr;
    // parameters: float32 masters, gradient, Adam moments; bf16 working copies
    // W [out][in] (W1 padded to 64 inputs) and, for back-propagation, W^T
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *W1 = nullptr, *W2 = nullptr, *W2t = nullptr, *W3 = nullptr, *W3t = nullptr;
    uint16_t *Wf = nullptr;  // W1, W2, W3 in the fused inference kernel's fragment order
    // training batch, transposed [feature][row] with row pitch max_rows
    uint16_t *Xt = nullptr, *H1t = nullptr, *H2t = nullptr, *G1t = nullptr, *G2t = nullptr, *G3t = nullptr;
    // kept by tgo_surrogate_grad for inspection: h3 [row][256] and scores
    uint16_t *H3 = nullptr;
    float *score = nullptr;
    int64_t kept_rows = 0;
    // per-block vectors and per-chunk partial sums of a training step
    float *vec = nullptr, *wpart = nullptr, *vpart = nullptr;
    float *F = nullptr;
    int max_groups = 0;
    int32_t *status = nullptr;
    uint8_t *horders = nullptr;
    int64_t *hns = nullptr;
    tgo::BestPair *best = nullptr;
    unsigned long long *keys = nullptr;
    unsigned long long *cand[2] = {nullptr, nullptr};
    size_t cand_bytes = 0;
    size_t bytes = 0;  // the main allocation
};

namespace tgo {

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// K chunks of the weight-gradient launch: at most WG_KS_MAX, each a whole
// number of row blocks.
static void wgrad_chunks(int rows, int *ks, int *kc) {
    int k = (rows + WG_KC - 1) / WG_KC;
    k = k < 1 ? 1 : (k > WG_KS_MAX ? WG_KS_MAX : k);
    int c = ((rows + k - 1) / k + TR_ROWS - 1) / TR_ROWS * TR_ROWS;
    *kc = c;
    *ks = (rows + c - 1) / c;
}

// Forward + backward and the weight-gradient partials of one batch; returns
// the number of K chunks.
static int train_pass(tgo_surrogate *s, const tgo_task *d_tasks, const int32_t *d_offs, const uint8_t *d_orders,
                      const int32_t *d_gid, const int64_t *d_T, int rows, bool keep, int *ks_out, hipStream_t st) {
    const int blocks = (rows + TR_ROWS - 1) / TR_ROWS;
    hipLaunchKernelGGL(train_fwd_bwd_kernel, dim3(blocks), dim3(TR_THREADS), 0, st, d_tasks, d_offs, d_orders, d_gid,
                       d_T, rows, 1.0f / (float)rows, s->W1, s->W2, s->W3, s->W2t, s->W3t, s->p, s->ldt, s->Xt,
                       s->H1t, s->H2t, s->G3t, s->G2t, s->G1t, s->vec, keep ? s->H3 : (uint16_t *)nullptr,
                       keep ? s->score : (float *)nullptr);
    int ks = 0, kc = 0;
    wgrad_chunks(rows, &ks, &kc);
    hipLaunchKernelGGL(train_wgrad_kernel, dim3((WG_TILES + WG_VEC_BLOCKS) * 8 * ((ks + 7) / 8)), dim3(256), 0, st,
                       s->Xt, s->H1t,
                       s->H2t, s->G1t, s->G2t, s->G3t, s->ldt, rows, kc, s->vec, s->wpart, s->vpart);
    TGO_HIP(hipGetLastError());
    *ks_out = ks;
    return TGO_OK;
}

static AdamArgs adam_args(int64_t step, float lr) {
    AdamArgs a;
    a.lr = lr;
    a.beta1 = 0.9f;
    a.beta2 = 0.999f;
    a.eps = 1e-8f;
    a.c1 = (float)(1.0 - std::pow(0.9, (double)step));
    a.c2 = (float)(1.0 - std::pow(0.999, (double)step));
    a.omb1 = (float)(1.0 - 0.9);
    a.omb2 = (float)(1.0 - 0.999);
    return a;
}

static void launch_update(tgo_surrogate *s, int mode, int ks, const float *gin, const AdamArgs &a, float *loss,
                          hipStream_t st) {
    hipLaunchKernelGGL(train_update_kernel, dim3((SG_NPARAM + 255) / 256), dim3(256), 0, st, mode, s->wpart,
                       s->vpart, ks, gin, s->p, s->g, s->m, s->v, a, loss, s->W1, s->W2, s->W2t, s->W3, s->W3t);
}

}  // namespace tgo

using namespace tgo;

extern "C" {

int tgo_surrogate_create(int64_t max_rows, int max_groups, tgo_surrogate **out) {
    if (!out) return fail(TGO_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_rows < 64 || max_rows > (int64_t)1 << 24 || (max_rows % 64) != 0)
        return fail(TGO_EINVAL, "max_rows must be a multiple of 64 in 64..2^24");
    if (max_groups < 1 || max_groups > (1 << 22)) return fail(TGO_EINVAL, "max_groups out of range");
    tgo_surrogate *s = new (std::nothrow) tgo_surrogate();
    if (!s) return fail(TGO_ENOMEM, "surrogate");
    s->max_rows = max_rows;
    // the search's only per-row buffer is its key array, so it scores in
    // launches of at least 2^20 rows: a launch of 1,024 blocks of 64 rows
    // (4 per CU, 3 resident) ends with a round on a third of the CUs
    s->search_rows = std::max<int64_t>(max_rows, (int64_t)1 << 20) / TK_RUN * TK_RUN;
    s->ldt = max_rows + TR_LD_PAD;
    s->max_groups = max_groups;
    (void)hipGetDevice(&s->device);
    const size_t R = (size_t)max_rows, LT = (size_t)s->ldt;
    const size_t blocks = (R + TR_ROWS - 1) / TR_ROWS;
    std::vector<std::pair<void **, size_t>> parts = {
        {(void **)&s->p, 4 * SG_NPARAM}, {(void **)&s->g, 4 * SG_NPARAM}, {(void **)&s->m, 4 * SG_NPARAM},
        {(void **)&s->v, 4 * SG_NPARAM},
        {(void **)&s->W1, 2 * SG_H * SG_K0}, {(void **)&s->W2, 2 * SG_H * SG_H}, {(void **)&s->W2t, 2 * SG_H * SG_H},
        {(void **)&s->W3, 2 * SG_H * SG_H}, {(void **)&s->W3t, 2 * SG_H * SG_H}, {(void **)&s->Wf, 2 * (size_t)FM_WF},
        {(void **)&s->Xt, 2 * LT * SG_K0}, {(void **)&s->H1t, 2 * LT * SG_H}, {(void **)&s->H2t, 2 * LT * SG_H},
        {(void **)&s->G1t, 2 * LT * SG_H}, {(void **)&s->G2t, 2 * LT * SG_H}, {(void **)&s->G3t, 2 * LT * SG_H},
        {(void **)&s->H3, 2 * R * SG_H}, {(void **)&s->score, 4 * R},
        {(void **)&s->vec, 4 * blocks * TR_VSTRIDE},
        {(void **)&s->wpart, 4 * (size_t)WG_KS_MAX * SG_NPARAM},
        {(void **)&s->vpart, 4 * (size_t)WG_KS_MAX},
        {(void **)&s->F, 4 * (size_t)max_groups * SG_POS * 3},
        {(void **)&s->status, 4 * (size_t)max_groups}, {(void **)&s->horders, 16 * (size_t)max_groups},
        {(void **)&s->hns, 8 * (size_t)max_groups}, {(void **)&s->best, sizeof(BestPair) * (size_t)max_groups},
        {(void **)&s->keys, 8 * (size_t)s->search_rows},
    };
    size_t total = 0;
    for (auto &pt : parts) total += align256(pt.second);
    s->bytes = total;
    hipError_t e = hipMalloc(&s->mem, total);
    if (e != hipSuccess) {
        delete s;
        return fail(TGO_ENOMEM, std::string("surrogate memory: ") + hipGetErrorString(e));
    }
    size_t off = 0;
    for (auto &pt : parts) {
        *pt.first = (char *)s->mem + off;
        off += align256(pt.second);
    }
    *out = s;
    return TGO_OK;
}

void tgo_surrogate_destroy(tgo_surrogate *s) {
    if (!s) return;
    (void)hipDeviceSynchronize();
    (void)hipFree(s->mem);
    if (s->cand[0]) (void)hipFree(s->cand[0]);
    if (s->cand[1]) (void)hipFree(s->cand[1]);
    delete s;
}

static int refresh(tgo_surrogate *s, hipStream_t st) {
    hipLaunchKernelGGL(refresh_bf16_kernel, dim3((SG_H * SG_H + 255) / 256), dim3(256), 0, st, s->p, s->W1,
                       s->W2, s->W2t, s->W3, s->W3t);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

int tgo_surrogate_init(tgo_surrogate *s, uint64_t seed, tgo_stream stream) {
    if (!s) return fail(TGO_EINVAL, "surrogate is NULL");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(init_params_kernel, dim3((SG_NPARAM + 255) / 256), dim3(256), 0, st, s->p, seed);
    TGO_HIP(hipMemsetAsync(s->m, 0, 4 * SG_NPARAM, st));
    TGO_HIP(hipMemsetAsync(s->v, 0, 4 * SG_NPARAM, st));
    s->step = 0;
    return refresh(s, st);
}

int tgo_surrogate_set_params(tgo_surrogate *s, const float *h_params, tgo_stream stream) {
    if (!s || !h_params) return fail(TGO_EINVAL, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    TGO_HIP(hipMemcpyAsync(s->p, h_params, 4 * SG_NPARAM, hipMemcpyHostToDevice, st));
    TGO_HIP(hipMemsetAsync(s->m, 0, 4 * SG_NPARAM, st));
    TGO_HIP(hipMemsetAsync(s->v, 0, 4 * SG_NPARAM, st));
    TGO_HIP(hipStreamSynchronize(st));
    s->step = 0;
    return refresh(s, st);
}

int tgo_surrogate_get_params(tgo_surrogate *s, float *h_params, tgo_stream stream) {
    if (!s || !h_params) return fail(TGO_EINVAL, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    TGO_HIP(hipMemcpyAsync(h_params, s->p, 4 * SG_NPARAM, hipMemcpyDeviceToHost, st));
    TGO_HIP(hipStreamSynchronize(st));
    return TGO_OK;
}

// File: 8-byte magic, uint32 parameter count, uint32 zero, float32 masters
// (little-endian, the layout of tgo_surrogate_get_params).
static const char SG_MAGIC[8] = {'T', 'G', 'O', 'S', 'U', 'R', 'R', '1'};

int tgo_surrogate_save(tgo_surrogate *s, const char *path) {
    if (!s || !path) return fail(TGO_EINVAL, "bad argument");
    std::vector<float> h(SG_NPARAM);
    int rc = tgo_surrogate_get_params(s, h.data(), nullptr);
    if (rc) return rc;
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(TGO_EINVAL, std::string("cannot open ") + path);
    const uint32_t hdr[2] = {(uint32_t)SG_NPARAM, 0u};
    const bool ok = std::fwrite(SG_MAGIC, 1, 8, f) == 8 && std::fwrite(hdr, 4, 2, f) == 2 &&
                    std::fwrite(h.data(), 4, SG_NPARAM, f) == (size_t)SG_NPARAM;
    const bool closed = std::fclose(f) == 0;
    if (!ok || !closed) return fail(TGO_EINVAL, std::string("write failed: ") + path);
    return TGO_OK;
}

int tgo_surrogate_load(tgo_surrogate *s, const char *path) {
    if (!s || !path) return fail(TGO_EINVAL, "bad argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(TGO_EINVAL, std::string("cannot open ") + path);
    char magic[8];
    uint32_t hdr[2];
    std::vector<float> h(SG_NPARAM);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, SG_MAGIC, 8) == 0 &&
              std::fread(hdr, 4, 2, f) == 2 && hdr[0] == (uint32_t)SG_NPARAM &&
              std::fread(h.data(), 4, SG_NPARAM, f) == (size_t)SG_NPARAM;
    char extra;
    ok = ok && std::fread(&extra, 1, 1, f) == 0;  // nothing after the parameters
    std::fclose(f);
    if (!ok) return fail(TGO_EINVAL, std::string("not a parameter file of this network: ") + path);
    for (float v : h)
        if (!std::isfinite(v)) return fail(TGO_EINVAL, "parameter file holds a non-finite value");
    return tgo_surrogate_set_params(s, h.data(), nullptr);
}

static int check_groups(const tgo_task *d_tasks, const int32_t *d_offs, int G, int max_groups) {
    if (!d_tasks || !d_offs) return fail(TGO_EINVAL, "NULL buffer");
    if (G < 1 || G > max_groups) return fail(TGO_EINVAL, "n_groups out of range");
    return TGO_OK;
}

int tgo_surrogate_pairs(const tgo_model *model, const tgo_task *d_tasks, const int32_t *d_offs, int G,
                        int64_t per_group, uint64_t seed, int32_t *d_status, uint8_t *d_orders,
                        int32_t *d_gid, int64_t *d_T, tgo_stream stream) {
    Rates r;
    int rc = make_rates(model, &r);
    if (rc) return rc;
    rc = check_groups(d_tasks, d_offs, G, 1 << 22);
    if (rc) return rc;
    if (per_group < 64 || per_group % 64) return fail(TGO_EINVAL, "per_group must be a positive multiple of 64");
    if (!d_status || !d_orders || !d_gid || !d_T) return fail(TGO_EINVAL, "NULL buffer");
    hipStream_t st = (hipStream_t)stream;
    int32_t *mode = nullptr;
    rc = workspace(4 * (size_t)G, (void **)&mode, st);
    if (rc) return rc;
    hipLaunchKernelGGL(group_status_kernel, dim3((G + 255) / 256), dim3(256), 0, st, d_tasks, d_offs, G, r, mode,
                       d_status);
    const int64_t tiles = per_group / 64 * G;
    const int blocks = (int)std::min<int64_t>((tiles + 3) / 4, 8192);
    hipLaunchKernelGGL(pairs_kernel<uint32_t>, dim3(blocks), dim3(SG_THREADS), lane_queue_bytes<uint32_t>(), st,
                       d_tasks, d_offs, G, r, per_group, seed, mode, d_orders, d_gid, d_T);
    // groups on the 64-bit time path (the blocks skip every other group)
    hipLaunchKernelGGL(pairs_kernel<uint64_t>, dim3(2 * blocks), dim3(lane_threads<uint64_t>()), lane_queue_bytes<uint64_t>(), st,
                       d_tasks, d_offs, G, r, per_group, seed, mode, d_orders, d_gid, d_T);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

int tgo_surrogate_score(tgo_surrogate *s, const tgo_task *d_tasks, const int32_t *d_offs, int G,
                        const uint8_t *d_orders, const int32_t *d_gid, int64_t rows, float *d_scores,
                        tgo_stream stream) {
    if (!s) return fail(TGO_EINVAL, "surrogate is NULL");
    int rc = check_groups(d_tasks, d_offs, G, s->max_groups);
    if (rc) return rc;
    if (rows < 1 || rows > s->max_rows || !d_orders || !d_gid || !d_scores)
        return fail(TGO_EINVAL, "rows out of range or NULL buffer");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(group_features_kernel, dim3((G * SG_POS + 255) / 256), dim3(256), 0, st, d_tasks, d_offs,
                       G, s->F);
    hipLaunchKernelGGL(pack_frag_kernel, dim3((FM_WF + 255) / 256), dim3(256), 0, st, s->W1, s->W2, s->W3, s->Wf);
    hipLaunchKernelGGL(mlp_fused_kernel, dim3((unsigned)((rows + FM_ROWS - 1) / FM_ROWS)), dim3(FM_THREADS), 0, st, s->F,
                       d_offs, (const uint32_t *)nullptr, d_orders, d_gid, (int64_t)0, rows, (int64_t)1, (int64_t)1,
                       (uint64_t)0, s->Wf, s->Wf + FM_WF1, s->Wf + FM_WF1 + SG_H * SG_H, s->p, d_scores,
                       (unsigned long long *)nullptr);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

int tgo_surrogate_grad(tgo_surrogate *s, const tgo_task *d_tasks, const int32_t *d_offs, int G,
                       const uint8_t *d_orders, const int32_t *d_gid, const int64_t *d_T, int rows,
                       float *d_grad, float *d_loss, tgo_stream stream) {
    if (!s) return fail(TGO_EINVAL, "surrogate is NULL");
    int rc = check_groups(d_tasks, d_offs, G, s->max_groups);
    if (rc) return rc;
    if (rows < 64 || rows > s->max_rows || rows % 64 || !d_orders || !d_gid || !d_T || !d_loss)
        return fail(TGO_EINVAL, "rows must be a multiple of 64 up to max_rows; no NULL buffers");
    hipStream_t st = (hipStream_t)stream;
    int ks = 0;
    rc = train_pass(s, d_tasks, d_offs, d_orders, d_gid, d_T, rows, true, &ks, st);
    if (rc) return rc;
    s->kept_rows = rows;
    launch_update(s, 0, ks, nullptr, adam_args(1, 0.f), d_loss, st);
    TGO_HIP(hipGetLastError());
    if (d_grad) TGO_HIP(hipMemcpyAsync(d_grad, s->g, 4 * SG_NPARAM, hipMemcpyDeviceToDevice, st));
    return TGO_OK;
}

int tgo_surrogate_train_step(tgo_surrogate *s, const tgo_task *d_tasks, const int32_t *d_offs, int G,
                             const uint8_t *d_orders, const int32_t *d_gid, const int64_t *d_T, int rows,
                             float lr, float *d_loss, tgo_stream stream) {
    if (!s) return fail(TGO_EINVAL, "surrogate is NULL");
    int rc = check_groups(d_tasks, d_offs, G, s->max_groups);
    if (rc) return rc;
    if (rows < 64 || rows > s->max_rows || rows % 64 || !d_orders || !d_gid || !d_T || !d_loss)
        return fail(TGO_EINVAL, "rows must be a multiple of 64 up to max_rows; no NULL buffers");
    if (!(lr > 0.f)) return fail(TGO_EINVAL, "lr must be > 0");
    hipStream_t st = (hipStream_t)stream;
    int ks = 0;
    rc = train_pass(s, d_tasks, d_offs, d_orders, d_gid, d_T, rows, false, &ks, st);
    if (rc) return rc;
    s->step += 1;
    launch_update(s, 1, ks, nullptr, adam_args(s->step, lr), d_loss, st);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

int tgo_surrogate_adam_step(tgo_surrogate *s, const float *d_grad, float lr, tgo_stream stream) {
    if (!s || !d_grad) return fail(TGO_EINVAL, "NULL argument");
    if (!(lr > 0.f)) return fail(TGO_EINVAL, "lr must be > 0");
    s->step += 1;
    launch_update(s, 2, 0, d_grad, adam_args(s->step, lr), nullptr, (hipStream_t)stream);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

int tgo_surrogate_get_moments(tgo_surrogate *s, float *h_m, float *h_v, int64_t *h_step, tgo_stream stream) {
    if (!s) return fail(TGO_EINVAL, "surrogate is NULL");
    hipStream_t st = (hipStream_t)stream;
    if (h_m) TGO_HIP(hipMemcpyAsync(h_m, s->m, 4 * SG_NPARAM, hipMemcpyDeviceToHost, st));
    if (h_v) TGO_HIP(hipMemcpyAsync(h_v, s->v, 4 * SG_NPARAM, hipMemcpyDeviceToHost, st));
    TGO_HIP(hipStreamSynchronize(st));
    if (h_step) *h_step = s->step;
    return TGO_OK;
}

int tgo_surrogate_get_batch(tgo_surrogate *s, int what, int64_t rows, void *h_out, tgo_stream stream) {
    if (!s || !h_out) return fail(TGO_EINVAL, "NULL argument");
    if (what < 0 || what > 7) return fail(TGO_EINVAL, "what must be in 0..7");
    if (rows < 1 || rows > s->kept_rows) return fail(TGO_EINVAL, "rows must be in 1..rows of the last tgo_surrogate_grad");
    hipStream_t st = (hipStream_t)stream;
    if (what == 3 || what == 4) {
        const size_t b = what == 3 ? 2 * (size_t)rows * SG_H : 4 * (size_t)rows;
        TGO_HIP(hipMemcpyAsync(h_out, what == 3 ? (void *)s->H3 : (void *)s->score, b, hipMemcpyDeviceToHost, st));
        TGO_HIP(hipStreamSynchronize(st));
        return TGO_OK;
    }
    const uint16_t *src = what == 0 ? s->Xt : what == 1 ? s->H1t : what == 2 ? s->H2t
                        : what == 5 ? s->G3t : what == 6 ? s->G2t : s->G1t;
    const int width = what == 0 ? SG_K0 : SG_H, keep = what == 0 ? SG_FEAT : SG_H;
    std::vector<uint16_t> t((size_t)width * rows);
    TGO_HIP(hipMemcpy2DAsync(t.data(), 2 * (size_t)rows, src, 2 * (size_t)s->ldt, 2 * (size_t)rows, width,
                             hipMemcpyDeviceToHost, st));
    TGO_HIP(hipStreamSynchronize(st));
    uint16_t *o = (uint16_t *)h_out;
    for (int64_t r = 0; r < rows; ++r)
        for (int c = 0; c < keep; ++c) o[r * keep + c] = t[(size_t)c * rows + r];
    return TGO_OK;
}

}  // extern "C"

size_t tgo::surrogate_device_bytes(const tgo_surrogate *s) { return s ? s->bytes + 2 * s->cand_bytes : 0; }

extern "C" {

// Candidate-key buffers, grown on demand.  The object is either fully sized
// (both buffers, cand_bytes) or empty (no buffers, cand_bytes = 0): a failed
// growth leaves it empty, so the next call tries to allocate again instead of
// using a buffer that is not there.
static int grow_cand(tgo_surrogate *s, size_t bytes) {
    if (s->cand_bytes >= bytes && s->cand[0] && s->cand[1]) return TGO_OK;
    s->cand_bytes = 0;
    if (s->cand[0] || s->cand[1]) TGO_HIP(hipDeviceSynchronize());
    for (int i = 0; i < 2; ++i) {
        if (s->cand[i]) (void)hipFree(s->cand[i]);
        s->cand[i] = nullptr;
    }
    for (int i = 0; i < 2; ++i) {
        hipError_t e = hipMalloc((void **)&s->cand[i], bytes);
        if (e != hipSuccess) {
            for (int j = 0; j < 2; ++j) {
                if (s->cand[j]) (void)hipFree(s->cand[j]);
                s->cand[j] = nullptr;
            }
            return fail(TGO_ENOMEM, std::string("candidate keys: ") + hipGetErrorString(e));
        }
    }
    s->cand_bytes = bytes;
    return TGO_OK;
}

}  // extern "C"

// Size the candidate buffers for searches of up to G groups of `samples`
// draws each, so that such searches allocate nothing more.
int tgo::surrogate_reserve(tgo_surrogate *s, int G, int64_t samples) {
    const int64_t runs = (samples + TK_RUN - 1) / TK_RUN;
    return grow_cand(s, sizeof(unsigned long long) * (size_t)G * (size_t)runs * TK_KEEP);
}

extern "C" {

// The candidate stage of the search: sample, score and keep the TK_KEEP
// smallest keys of every group.  On return cand[*cur] holds per group a
// sorted list of *len keys (group stride *len) whose first TK_KEEP are the
// group's smallest keys.
static int search_candidates(tgo_surrogate *s, const Rates &r, const tgo_task *d_tasks, const int32_t *d_offs,
                             const uint32_t *d_keys, int G, int64_t samples, uint64_t seed, hipStream_t st,
                             int *cur_out, int64_t *len_out) {
    const int64_t chunk = s->search_rows;  // a multiple of TK_RUN
    const int64_t spad = (samples + TK_RUN - 1) / TK_RUN * TK_RUN;
    const int64_t runs = spad / TK_RUN;
    int rc = grow_cand(s, sizeof(unsigned long long) * (size_t)G * (size_t)runs * TK_KEEP);
    if (rc) return rc;
    hipLaunchKernelGGL(group_status_kernel, dim3((G + 255) / 256), dim3(256), 0, st, d_tasks, d_offs, G, r,
                       s->status, (int32_t *)nullptr);
    hipLaunchKernelGGL(group_features_kernel, dim3((G * SG_POS + 255) / 256), dim3(256), 0, st, d_tasks, d_offs,
                       G, s->F);
    hipLaunchKernelGGL(pack_frag_kernel, dim3((FM_WF + 255) / 256), dim3(256), 0, st, s->W1, s->W2, s->W3, s->Wf);
    const int64_t total = (int64_t)G * spad;
    for (int64_t row0 = 0; row0 < total; row0 += chunk) {
        const int64_t rows = std::min(chunk, total - row0);
        // rows is a multiple of TK_RUN, hence of FM_ROWS
        hipLaunchKernelGGL(mlp_fused_kernel, dim3((unsigned)(rows / FM_ROWS)), dim3(FM_THREADS), 0, st, s->F, d_offs, d_keys,
                           (const uint8_t *)nullptr, (const int32_t *)nullptr, row0, rows, spad, samples, seed, s->Wf,
                           s->Wf + FM_WF1, s->Wf + FM_WF1 + SG_H * SG_H, s->p, (float *)nullptr, s->keys);
        const int nrun = (int)(rows / TK_RUN);
        hipLaunchKernelGGL(topk_pass_kernel, dim3(nrun, 1), dim3(TK_THREADS), 0, st, s->keys, (int64_t)0, rows, nrun,
                           s->cand[0] + (row0 / TK_RUN) * TK_KEEP, (int64_t)0);
    }
    int64_t len = runs * TK_KEEP;
    int cur = 0;
    while (len > TK_KEEP) {
        const int nrun = (int)((len + TK_RUN - 1) / TK_RUN);
        hipLaunchKernelGGL(topk_pass_kernel, dim3(nrun, G), dim3(TK_THREADS), 0, st, s->cand[cur], len, len, nrun,
                           s->cand[cur ^ 1], (int64_t)nrun * TK_KEEP);
        len = (int64_t)nrun * TK_KEEP;
        cur ^= 1;
    }
    TGO_HIP(hipGetLastError());
    *cur_out = cur;
    *len_out = len;
    return TGO_OK;
}

static int check_search_args(tgo_surrogate *s, const tgo_model *model, Rates *r, const tgo_task *d_tasks,
                             const int32_t *d_offs, int G, int64_t samples, int topk) {
    if (!s) return fail(TGO_EINVAL, "surrogate is NULL");
    int rc = make_rates(model, r);
    if (rc) return rc;
    rc = check_groups(d_tasks, d_offs, G, s->max_groups);
    if (rc) return rc;
    if (G > 65535) return fail(TGO_EINVAL, "search handles at most 65535 groups per call");
    if (samples < 1 || samples > ((int64_t)1 << 32)) return fail(TGO_EINVAL, "samples out of range");
    if (topk < 1 || topk > TK_KEEP) return fail(TGO_EINVAL, "topk must be in 1..64");
    return TGO_OK;
}

// out[g][i] = in[g * stride + i] for i < k
__global__ void copy_candidates_kernel(const unsigned long long *__restrict__ in, int64_t stride, int G, int k,
                                       unsigned long long *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= G * k) return;
    const int g = i / k, j = i % k;
    out[i] = in[(int64_t)g * stride + j];
}

int tgo_surrogate_search(tgo_surrogate *s, const tgo_model *model, const tgo_task *d_tasks,
                         const int32_t *d_offs, const uint32_t *d_keys, int G, int64_t samples, int topk,
                         uint64_t seed, tgo_search_result *d_out, tgo_stream stream) {
    Rates r;
    int rc = check_search_args(s, model, &r, d_tasks, d_offs, G, samples, topk);
    if (rc) return rc;
    if (!d_out) return fail(TGO_EINVAL, "NULL buffer");
    hipStream_t st = (hipStream_t)stream;
    int cur = 0;
    int64_t len = 0;
    rc = search_candidates(s, r, d_tasks, d_offs, d_keys, G, samples, seed, st, &cur, &len);
    if (rc) return rc;
    rc = launch_heuristic(r, d_tasks, d_offs, G, s->horders, 16, s->hns, 1, st);
    if (rc) return rc;
    hipLaunchKernelGGL(rescore_kernel<uint32_t>, dim3((G + 3) / 4), dim3(SG_THREADS), lane_queue_bytes<uint32_t>(), st,
                       d_tasks, d_offs, G, r, topk, seed, s->status, d_keys, s->cand[cur], (int)len, s->best);
    hipLaunchKernelGGL(rescore_kernel<uint64_t>, dim3((G + 1) / 2), dim3(lane_threads<uint64_t>()), lane_queue_bytes<uint64_t>(), st,
                       d_tasks, d_offs, G, r, topk, seed, s->status, d_keys, s->cand[cur], (int)len, s->best);
    hipLaunchKernelGGL(search_finish_kernel, dim3((G + 255) / 256), dim3(256), 0, st, d_offs, G, seed, d_keys,
                       s->status, s->best, (const unsigned long long *)nullptr, (const BestPair *)nullptr, 0,
                       s->horders, s->hns, d_out);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

int tgo_surrogate_candidates(tgo_surrogate *s, const tgo_model *model, const tgo_task *d_tasks,
                             const int32_t *d_offs, const uint32_t *d_keys, int G, int64_t samples, int topk,
                             uint64_t seed, uint64_t *d_cand, tgo_stream stream) {
    Rates r;
    int rc = check_search_args(s, model, &r, d_tasks, d_offs, G, samples, topk);
    if (rc) return rc;
    if (!d_cand) return fail(TGO_EINVAL, "NULL buffer");
    hipStream_t st = (hipStream_t)stream;
    int cur = 0;
    int64_t len = 0;
    rc = search_candidates(s, r, d_tasks, d_offs, d_keys, G, samples, seed, st, &cur, &len);
    if (rc) return rc;
    hipLaunchKernelGGL(copy_candidates_kernel, dim3((G * topk + 255) / 256), dim3(256), 0, st, s->cand[cur], len,
                       G, topk, (unsigned long long *)d_cand);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

int tgo_random_search(const tgo_model *model, const tgo_task *d_tasks, const int32_t *d_offs, int G,
                      int64_t samples, uint64_t seed, tgo_search_result *d_out, tgo_stream stream) {
    Rates r;
    int rc = make_rates(model, &r);
    if (rc) return rc;
    rc = check_groups(d_tasks, d_offs, G, 1 << 22);
    if (rc) return rc;
    if (samples < 0 || samples > ((int64_t)1 << 32) || !d_out) return fail(TGO_EINVAL, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    const int64_t per = (samples + 63) / 64 * 64;
    char *ws = nullptr;
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t need = al(4 * (size_t)G) + al(8 * (size_t)G) + al(8 * (size_t)G) + al(16 * (size_t)G) +
                        sizeof(BestPair) * RS_WIDE_CHUNKS * (size_t)G;
    rc = workspace(need, (void **)&ws, st);
    if (rc) return rc;
    int32_t *mode = (int32_t *)ws;
    int64_t *hns = (int64_t *)(ws + al(4 * (size_t)G));
    unsigned long long *best = (unsigned long long *)((char *)hns + al(8 * (size_t)G));
    uint8_t *horders = (uint8_t *)((char *)best + al(8 * (size_t)G));
    BestPair *wpart = (BestPair *)(horders + al(16 * (size_t)G));
    hipLaunchKernelGGL(group_status_kernel, dim3((G + 255) / 256), dim3(256), 0, st, d_tasks, d_offs, G, r, mode,
                       (int32_t *)nullptr);
    rc = launch_heuristic(r, d_tasks, d_offs, G, horders, 16, hns, 1, st);
    if (rc) return rc;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((G + 255) / 256), dim3(256), 0, st, best, (int64_t)G, ~0ull);
    int wchunks = 0;
    if (per > 0) {
        // chunks of up to 64 tiles, while keeping at least ~64k wave tasks
        const int64_t tpg = per / 64;
        const int64_t tiles = tpg * G;
        const int64_t chunk_tiles = std::max<int64_t>(1, std::min<int64_t>(64, tiles >> 16));
        const int64_t chunks = (tpg + chunk_tiles - 1) / chunk_tiles * G;
        const int blocks = (int)std::min<int64_t>((chunks + 3) / 4, 16384);
        hipLaunchKernelGGL(random_search_kernel<uint32_t>, dim3(blocks), dim3(SG_THREADS),
                           lane_queue_bytes<uint32_t>(), st, d_tasks, d_offs, G, r, per, seed, chunk_tiles, mode,
                           best, wpart);
        // groups on the 64-bit time path: at most RS_WIDE_CHUNKS chunks each
        const int64_t wct = std::max<int64_t>(chunk_tiles, (tpg + RS_WIDE_CHUNKS - 1) / RS_WIDE_CHUNKS);
        wchunks = (int)((tpg + wct - 1) / wct);
        const int wblocks = (int)std::min<int64_t>(((int64_t)wchunks * G + 1) / 2, 16384);
        hipLaunchKernelGGL(random_search_kernel<uint64_t>, dim3(wblocks), dim3(lane_threads<uint64_t>()),
                           lane_queue_bytes<uint64_t>(), st, d_tasks, d_offs, G, r, per, seed, wct, mode, best,
                           wpart);
    }
    hipLaunchKernelGGL(search_finish_kernel, dim3((G + 255) / 256), dim3(256), 0, st, d_offs, G, seed,
                       (const uint32_t *)nullptr, mode, (const BestPair *)nullptr, best, wpart, wchunks, horders,
                       hns, d_out);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

int tgo_surrogate_param_count(void) { return SG_NPARAM; }

}  // extern "C"
