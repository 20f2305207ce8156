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
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>

#include <cmath>
#include <cstdlib>
#include <string>
#include <vector>

#include "surrogate_dev.h"
#include "tables_dev.h"
#include "tgo_internal.h"

namespace tgo {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int SG_THREADS = 256;

// ------------------------------------------------------------- exact lanes
// Exact evaluation of (group, ordering) items, one wave per group tile: the
// wave loads the group's task table into its own LDS area and each lane
// evaluates one ordering with the 32-bit window code.

struct WaveTables {
    Quad<uint32_t> H[4][MAXN];
    DRec<uint32_t> D[4][MAXN];
};

__device__ __forceinline__ uint32_t eval_perm(uint64_t perm, int n, const View<uint32_t, 1, SG_THREADS> &v,
                                              const Rates &r) {
    Lane<uint32_t> st = lane_init<uint32_t>();
    for (int j = 0; j < n; ++j) window(st, j, (uint32_t)((perm >> (4 * j)) & 15u), v, r);
    return tail(st, r);
}

__device__ __forceinline__ void load_group(WaveTables &wt, int w, int lane, const tgo_task *t, int n,
                                           const Rates &r) {
    if (lane < n) table_entry<uint32_t>(t[lane], r, &wt.H[w][lane], &wt.D[w][lane]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// status per group: 0, or a TGO_E* code (size out of range, or outside the
// 32-bit time path which the search kernels use)
__global__ void group_status_kernel(const tgo_task *__restrict__ tasks, const int32_t *__restrict__ offs,
                                    int G, Rates r, int32_t *status) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const int n = offs[g + 1] - offs[g];
    int st = 0;
    if (n < 1 || n > SG_POS) st = TGO_EINVAL;
    else st = classify_group(tasks + offs[g], n, r) == 0 ? 0 : TGO_ERANGE;
    status[g] = st;
}

// Training pairs: per group `per` sampled orderings (per is a multiple of 64)
// and their exact T.
__global__ __launch_bounds__(SG_THREADS) void pairs_kernel(const tgo_task *__restrict__ tasks,
                                                           const int32_t *__restrict__ offs, int G,
                                                           Rates r, int64_t per, uint64_t seed,
                                                           const int32_t *__restrict__ status,
                                                           uint8_t *orders, int32_t *gid, int64_t *T) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ WaveTables wt;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    View<uint32_t, 1, SG_THREADS> v;
    v.H = wt.H[w];
    v.D = wt.D[w];
    v.Q = reinterpret_cast<Slot<uint32_t> *>(smem) + threadIdx.x;
    const int64_t tiles_per_group = per / 64;
    const int64_t total = tiles_per_group * G;
    const int64_t wstride = (int64_t)gridDim.x * (SG_THREADS / 64);
    for (int64_t tile = (int64_t)blockIdx.x * (SG_THREADS / 64) + w; tile < total; tile += wstride) {
        const int g = (int)(tile / tiles_per_group);
        const int64_t s = (tile % tiles_per_group) * 64 + lane;
        const int64_t row = (int64_t)g * per + s;
        const int n = offs[g + 1] - offs[g];
        uint8_t *o = orders + row * SG_POS;
        gid[row] = g;
        if (status[g] != 0) {
            T[row] = status[g];
            for (int p = 0; p < SG_POS; ++p) o[p] = 0xff;
            continue;
        }
        load_group(wt, w, lane, tasks + offs[g], n, r);
        const uint64_t perm = sample_ordering(n, (uint32_t)g, (uint64_t)s, seed);
        T[row] = (int64_t)eval_perm(perm, n, v, r);
        for (int p = 0; p < SG_POS; ++p) o[p] = p < n ? (uint8_t)((perm >> (4 * p)) & 15u) : 0xff;
        __builtin_amdgcn_wave_barrier();
    }
}

// Plain exact search: `per` sampled orderings per group (a multiple of 64),
// keep the smallest (T << 32 | sample).
// Each wave takes chunks of `chunk` consecutive 64-sample tiles of one group,
// so the group's table is loaded and the wave's minimum published once per
// chunk; wave-uniform values are kept in scalar registers.

__global__ __launch_bounds__(SG_THREADS) void random_search_kernel(const tgo_task *__restrict__ tasks,
                                                                   const int32_t *__restrict__ offs,
                                                                   int G, Rates r, int64_t per,
                                                                   uint64_t seed, int64_t chunk_tiles,
                                                                   const int32_t *__restrict__ status,
                                                                   unsigned long long *best) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ WaveTables wt;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    View<uint32_t, 1, SG_THREADS> v;
    v.H = wt.H[w];
    v.D = wt.D[w];
    v.Q = reinterpret_cast<Slot<uint32_t> *>(smem) + threadIdx.x;
    const int64_t tiles_per_group = per / 64;
    const int64_t chunks_per_group = (tiles_per_group + chunk_tiles - 1) / chunk_tiles;
    const int64_t total = chunks_per_group * G;
    const int64_t wstride = (int64_t)gridDim.x * (SG_THREADS / 64);
    for (int64_t chunk = (int64_t)blockIdx.x * (SG_THREADS / 64) + w; chunk < total; chunk += wstride) {
        const int g = (int)(chunk / chunks_per_group);
        if (status[g] != 0) continue;
        const int n = offs[g + 1] - offs[g];
        load_group(wt, w, lane, tasks + offs[g], n, r);
        const int64_t t0 = (chunk % chunks_per_group) * chunk_tiles;
        const int64_t t1 = t0 + chunk_tiles < tiles_per_group ? t0 + chunk_tiles : tiles_per_group;
        unsigned long long key = ~0ull;
        for (int64_t tile = t0; tile < t1; ++tile) {
            const int64_t s = tile * 64 + lane;
            const uint64_t perm = sample_ordering(n, (uint32_t)g, (uint64_t)s, seed);
            const unsigned long long k = ((unsigned long long)eval_perm(perm, n, v, r) << 32) | (uint64_t)s;
            key = k < key ? k : key;
        }
        for (int m = 32; m >= 1; m >>= 1) {
            const unsigned long long o = __shfl_xor(key, m);
            key = o < key ? o : key;
        }
        if (lane == 0) atomicMin(&best[g], key);
        __builtin_amdgcn_wave_barrier();
    }
}

// Exact re-score of the k best-scored candidates of every group (k <= 64,
// one wave per group): keys hold the sample index in the low 32 bits.
__global__ __launch_bounds__(SG_THREADS) void rescore_kernel(const tgo_task *__restrict__ tasks,
                                                             const int32_t *__restrict__ offs, int G,
                                                             Rates r, int k, uint64_t seed,
                                                             const int32_t *__restrict__ status,
                                                             const uint32_t *__restrict__ gkeys,
                                                             const unsigned long long *__restrict__ keys,
                                                             int key_stride,
                                                             unsigned long long *best) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ WaveTables wt;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    View<uint32_t, 1, SG_THREADS> v;
    v.H = wt.H[w];
    v.D = wt.D[w];
    v.Q = reinterpret_cast<Slot<uint32_t> *>(smem) + threadIdx.x;
    for (int g = blockIdx.x * (SG_THREADS / 64) + w; g < G; g += gridDim.x * (SG_THREADS / 64)) {
        if (status[g] != 0) continue;
        const int n = offs[g + 1] - offs[g];
        load_group(wt, w, lane, tasks + offs[g], n, r);
        unsigned long long key = ~0ull;
        const unsigned long long kk = lane < k ? keys[(int64_t)g * key_stride + lane] : ~0ull;
        if (kk != ~0ull) {
            const uint64_t s = kk & 0xffffffffull;
            const uint64_t perm = sample_ordering(n, gkeys ? gkeys[g] : (uint32_t)g, s, seed);
            key = ((unsigned long long)eval_perm(perm, n, v, r) << 32) | s;
        }
        for (int m = 32; m >= 1; m >>= 1) {
            const unsigned long long o = __shfl_xor(key, m);
            key = o < key ? o : key;
        }
        if (lane == 0) best[g] = key;
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

// First-layer input of one row as 32 words of packed bf16 pairs (48
// features + 16 zeros): the ordering is orders[i] (orders != null, group
// gid[i]) or sample (row mod spad) of group (row div spad) for row = row0 + i
// (samples >= S are padding: *ok = false, all-zero input).
__device__ __forceinline__ void row_input(const float *__restrict__ F, const int32_t *__restrict__ offs,
                                          const uint32_t *__restrict__ gkeys, const uint8_t *__restrict__ orders,
                                          const int32_t *__restrict__ gid, int64_t i, int64_t row0, int64_t spad,
                                          int64_t S, uint64_t seed, uint32_t (&w)[SG_K0 / 2], bool *okp) {
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
#pragma unroll
    for (int c = 0; c < SG_K0 / 2; ++c) w[c] = 0;
    const float *Fg = F + (int64_t)g * SG_POS * 3;
#pragma unroll
    for (int p = 0; p < SG_POS; ++p) {
        if (ok && p < n) {
            const int t = (int)((perm >> (4 * p)) & 15u);
            const uint32_t f0 = f2bf(Fg[t * 3]), f1 = f2bf(Fg[t * 3 + 1]), f2 = f2bf(Fg[t * 3 + 2]);
            // features 3p, 3p+1, 3p+2 -> halves of words (3p)/2 ...
            const int c0 = 3 * p;
            if ((c0 & 1) == 0) {
                w[c0 / 2] = f0 | (f1 << 16);
                w[c0 / 2 + 1] |= f2;
            } else {
                w[c0 / 2] |= f0 << 16;
                w[c0 / 2 + 1] = f1 | (f2 << 16);
            }
        }
    }
    *okp = ok;
}

// Rows of the first-layer input (bf16 [rows][64]), see row_input; padding
// rows are flagged in `valid`.
__global__ void features_kernel(const float *__restrict__ F, const int32_t *__restrict__ offs,
                                const uint32_t *__restrict__ gkeys,
                                const uint8_t *__restrict__ orders, const int32_t *__restrict__ gid,
                                int64_t row0, int64_t rows, int64_t spad, int64_t S, uint64_t seed,
                                uint16_t *X, uint16_t *Xt, int64_t xt_rows, uint8_t *valid) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    uint32_t w[SG_K0 / 2];
    bool ok;
    row_input(F, offs, gkeys, orders, gid, i, row0, spad, S, seed, w, &ok);
    uint4 *dst = reinterpret_cast<uint4 *>(X + i * SG_K0);
#pragma unroll
    for (int c = 0; c < SG_K0 / 8; ++c) {
        uint4 q;
        q.x = w[4 * c];
        q.y = w[4 * c + 1];
        q.z = w[4 * c + 2];
        q.w = w[4 * c + 3];
        dst[c] = q;
    }
    if (Xt) {
#pragma unroll
        for (int c = 0; c < SG_K0 / 2; ++c) {
            Xt[(int64_t)(2 * c) * xt_rows + i] = (uint16_t)w[c];
            Xt[(int64_t)(2 * c + 1) * xt_rows + i] = (uint16_t)(w[c] >> 16);
        }
    }
    if (valid) valid[i] = ok ? 1 : 0;
}

// ------------------------------------------------------------------- GEMM
// C[M][N] = sum_k A[M][K] * B[N][K] (both K-contiguous, bf16), float32
// accumulation on MFMA.  Block 256 threads, tile 64 x 64, K step 32; wave w
// computes rows 16w..16w+15 against the 64 columns (four 16 x 16 tiles).
// M, N multiples of 64, K a multiple of 32.
//
// Epilogue: v = acc (+ bias[n]); relu; multiply by (mask[m][n] > 0); then
// store as bf16 [M][N] (Y), bf16 [N][M] (Yt) and/or float [M][N] (Cf).
enum : int { EPI_BIAS = 1, EPI_RELU = 2, EPI_MASK = 4 };

struct GemmOut {
    uint16_t *Y;
    uint16_t *Yt;
    float *Cf;
    const float *bias;
    const uint16_t *mask;
};

constexpr int GT = 64, GK = 32, GPAD = 8;

// With SPLITK the K range is cut into gridDim.z pieces and each block adds its
// partial product into out.Cf (float atomics; Cf must start at zero).
template <int EPI, bool SPLITK = false>
__global__ __launch_bounds__(256) void gemm_nt_kernel(const uint16_t *__restrict__ A,
                                                      const uint16_t *__restrict__ B, int M, int N, int K,
                                                      GemmOut out) {
    __shared__ __align__(16) uint16_t As[GT][GK + GPAD];
    __shared__ __align__(16) uint16_t Bs[GT][GK + GPAD];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    f32x4 acc[4];
    for (int c = 0; c < 4; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int lr = tid >> 2, lk = (tid & 3) * 8;
    int kbeg = 0, kend = K;
    if constexpr (SPLITK) {
        const int per = K / gridDim.z;  // a multiple of GK (checked by the launcher)
        kbeg = blockIdx.z * per;
        kend = kbeg + per;
    }
    for (int k0 = kbeg; k0 < kend; k0 += GK) {
        const uint4 a = *reinterpret_cast<const uint4 *>(A + (int64_t)(m0 + lr) * K + k0 + lk);
        const uint4 b = *reinterpret_cast<const uint4 *>(B + (int64_t)(n0 + lr) * K + k0 + lk);
        __syncthreads();
        *reinterpret_cast<uint4 *>(&As[lr][lk]) = a;
        *reinterpret_cast<uint4 *>(&Bs[lr][lk]) = b;
        __syncthreads();
        const bf16x8 fa = *reinterpret_cast<const bf16x8 *>(&As[w * 16 + (l & 15)][(l >> 4) * 8]);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const bf16x8 fb = *reinterpret_cast<const bf16x8 *>(&Bs[c * 16 + (l & 15)][(l >> 4) * 8]);
            acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb, acc[c], 0, 0, 0);
        }
    }
    // lane l holds C[16w + 4(l/16) + i][16c + l%16], i = 0..3
    if constexpr (SPLITK) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int col = n0 + c * 16 + (l & 15);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                atomicAdd(&out.Cf[(int64_t)(m0 + w * 16 + (l >> 4) * 4 + i) * N + col], acc[c][i]);
        }
        return;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int col = n0 + c * 16 + (l & 15);
        const float bb = (EPI & EPI_BIAS) ? out.bias[col] : 0.f;
        uint16_t yv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = m0 + w * 16 + (l >> 4) * 4 + i;
            float vv = acc[c][i] + bb;
            if (EPI & EPI_RELU) vv = vv > 0.f ? vv : 0.f;
            if (EPI & EPI_MASK) vv = bf2f(out.mask[(int64_t)row * N + col]) > 0.f ? vv : 0.f;
            if (out.Cf) out.Cf[(int64_t)row * N + col] = vv;
            yv[i] = f2bf(vv);
            if (out.Y) out.Y[(int64_t)row * N + col] = yv[i];
        }
        if (out.Yt) {
            const int row0 = m0 + w * 16 + (l >> 4) * 4;
            uint2 q;
            q.x = yv[0] | ((uint32_t)yv[1] << 16);
            q.y = yv[2] | ((uint32_t)yv[3] << 16);
            *reinterpret_cast<uint2 *>(out.Yt + (int64_t)col * M + row0) = q;
        }
    }
}

// Large-M variant for the forward passes: block tile 128 x 128, wave w owns
// the 64 x 64 quadrant (w/2, w%2) as 4 x 4 MFMA tiles, so every K step issues
// 16 MFMAs per wave between two barriers; the next K slice is fetched into
// registers while the current one is multiplied.  M, N multiples of 128.
constexpr int BT2 = 128;

__device__ __forceinline__ void epilogue_store(const GemmOut &out, int EPI, int M, int N, int row0, int col,
                                               const f32x4 &acc) {
    const float bb = (EPI & EPI_BIAS) ? out.bias[col] : 0.f;
    uint16_t yv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row = row0 + i;
        float vv = acc[i] + bb;
        if (EPI & EPI_RELU) vv = vv > 0.f ? vv : 0.f;
        if (EPI & EPI_MASK) vv = bf2f(out.mask[(int64_t)row * N + col]) > 0.f ? vv : 0.f;
        if (out.Cf) out.Cf[(int64_t)row * N + col] = vv;
        yv[i] = f2bf(vv);
        if (out.Y) out.Y[(int64_t)row * N + col] = yv[i];
    }
    if (out.Yt) {
        uint2 q;
        q.x = yv[0] | ((uint32_t)yv[1] << 16);
        q.y = yv[2] | ((uint32_t)yv[3] << 16);
        *reinterpret_cast<uint2 *>(out.Yt + (int64_t)col * M + row0) = q;
    }
}

template <int EPI>
__global__ __launch_bounds__(256) void gemm_nt_big_kernel(const uint16_t *__restrict__ A,
                                                          const uint16_t *__restrict__ B, int M, int N, int K,
                                                          GemmOut out) {
    __shared__ __align__(16) uint16_t As[BT2][GK + GPAD];
    __shared__ __align__(16) uint16_t Bs[BT2][GK + GPAD];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int m0 = blockIdx.y * BT2, n0 = blockIdx.x * BT2;
    const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    // each thread moves rows (tid / 4) and (tid / 4 + 64), 8 bf16 at column (tid % 4) * 8
    const int lr = tid >> 2, lk = (tid & 3) * 8;
    const uint16_t *a0 = A + (int64_t)(m0 + lr) * K + lk, *a1 = a0 + (int64_t)64 * K;
    const uint16_t *b0 = B + (int64_t)(n0 + lr) * K + lk, *b1 = b0 + (int64_t)64 * K;
    uint4 ra0 = *reinterpret_cast<const uint4 *>(a0), ra1 = *reinterpret_cast<const uint4 *>(a1);
    uint4 rb0 = *reinterpret_cast<const uint4 *>(b0), rb1 = *reinterpret_cast<const uint4 *>(b1);
    for (int k0 = 0; k0 < K; k0 += GK) {
        __syncthreads();
        *reinterpret_cast<uint4 *>(&As[lr][lk]) = ra0;
        *reinterpret_cast<uint4 *>(&As[lr + 64][lk]) = ra1;
        *reinterpret_cast<uint4 *>(&Bs[lr][lk]) = rb0;
        *reinterpret_cast<uint4 *>(&Bs[lr + 64][lk]) = rb1;
        __syncthreads();
        if (k0 + GK < K) {
            ra0 = *reinterpret_cast<const uint4 *>(a0 + k0 + GK);
            ra1 = *reinterpret_cast<const uint4 *>(a1 + k0 + GK);
            rb0 = *reinterpret_cast<const uint4 *>(b0 + k0 + GK);
            rb1 = *reinterpret_cast<const uint4 *>(b1 + k0 + GK);
        }
        bf16x8 fa[4], fb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            fa[t] = *reinterpret_cast<const bf16x8 *>(&As[wr + t * 16 + (l & 15)][(l >> 4) * 8]);
            fb[t] = *reinterpret_cast<const bf16x8 *>(&Bs[wc + t * 16 + (l & 15)][(l >> 4) * 8]);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            epilogue_store(out, EPI, M, N, m0 + wr + a * 16 + (l >> 4) * 4, n0 + wc + b * 16 + (l & 15),
                           acc[a][b]);
}

// float C[M][N] += A B^T with the K range split over blocks (weight gradients:
// M, N <= 256 and K = batch rows)
static void gemm_splitk(const uint16_t *A, const uint16_t *B, int M, int N, int K, float *C, hipStream_t st) {
    int ks = 1;
    while (ks < 64 && (M / GT) * (N / GT) * ks < 512 && K % (2 * ks * GK) == 0) ks *= 2;
    GemmOut o{};
    o.Cf = C;
    hipLaunchKernelGGL((gemm_nt_kernel<0, true>), dim3(N / GT, M / GT, ks), dim3(256), 0, st, A, B, M, N, K, o);
}

template <int EPI>
static void gemm(const uint16_t *A, const uint16_t *B, int M, int N, int K, const GemmOut &o,
                 hipStream_t st) {
    if (M % BT2 == 0 && N % BT2 == 0 && M >= 4096)
        hipLaunchKernelGGL(gemm_nt_big_kernel<EPI>, dim3(N / BT2, M / BT2), dim3(256), 0, st, A, B, M, N, K, o);
    else
        hipLaunchKernelGGL(gemm_nt_kernel<EPI>, dim3(N / GT, M / GT), dim3(256), 0, st, A, B, M, N, K, o);
}

// ----------------------------------------------------------- head, loss

// score[i] = h3[i] . w4 + b4 (one wave per row); invalid rows get +inf
__global__ void head_kernel(const uint16_t *__restrict__ H3, const float *__restrict__ w4,
                            const float *__restrict__ b4, int64_t rows, const uint8_t *__restrict__ valid,
                            float *score) {
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int l = threadIdx.x & 63;
    if (row >= rows) return;
    const uint2 q = *reinterpret_cast<const uint2 *>(H3 + row * SG_H + l * 4);
    float s = bf2f((uint16_t)q.x) * w4[l * 4] + bf2f((uint16_t)(q.x >> 16)) * w4[l * 4 + 1] +
              bf2f((uint16_t)q.y) * w4[l * 4 + 2] + bf2f((uint16_t)(q.y >> 16)) * w4[l * 4 + 3];
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
    if (l == 0) score[row] = (valid && !valid[row]) ? INFINITY : s + b4[0];
}

// float -> uint32 with the same order (top-k keys compare as integers)
__device__ __forceinline__ uint32_t orderable(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// --------------------------------------------------------- fused inference
// One block scores 64 rows end to end: it builds their first-layer inputs in
// LDS, runs the three hidden layers on MFMA with the activations kept in LDS
// (rounded to bf16, as the layer-by-layer path stores them) and applies the
// head, so only the 64 scores (or top-k keys) leave the block.  Each of the
// 8 waves computes 32 output columns of each layer for all 64 rows as 4 x 2
// MFMA tiles; weights (bf16 [out][in]) come from global memory, where every
// block reads the same 282 KB.
constexpr int FM_ROWS = 64;
constexpr int FM_LD = SG_H + 8;        // LDS row pitch in bf16
constexpr int FM_WAVES = 8;            // wave w owns output columns FM_CT * 16 * w ..
constexpr int FM_CT = SG_H / 16 / FM_WAVES;  // column tiles per wave
constexpr int FM_THREADS = 64 * FM_WAVES;

template <int K>
__device__ __forceinline__ void fm_layer(const uint16_t (*Hs)[FM_LD], const uint16_t *__restrict__ W, int w, int l,
                                         f32x4 (&acc)[4][FM_CT]) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < FM_CT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t *wrow = W + (int64_t)(16 * FM_CT * w + (l & 15)) * K + (l >> 4) * 8;
    bf16x8 fb[FM_CT], nb[FM_CT];
#pragma unroll
    for (int t = 0; t < FM_CT; ++t) fb[t] = *reinterpret_cast<const bf16x8 *>(wrow + (int64_t)16 * t * K);
#pragma unroll 1
    for (int k0 = 0; k0 < K; k0 += GK) {
        if (k0 + GK < K) {
#pragma unroll
            for (int t = 0; t < FM_CT; ++t)
                nb[t] = *reinterpret_cast<const bf16x8 *>(wrow + (int64_t)16 * t * K + k0 + GK);
        }
        bf16x8 fa[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            fa[t] = *reinterpret_cast<const bf16x8 *>(&Hs[16 * t + (l & 15)][k0 + (l >> 4) * 8]);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < FM_CT; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < FM_CT; ++t) fb[t] = nb[t];
    }
}

// relu(acc + bias) as bf16 into Hs (lane l holds rows 16a + 4(l/16) + i of
// column 16 (FM_CT w + b) + l%16)
__device__ __forceinline__ void fm_store(uint16_t (*Hs)[FM_LD], const float *__restrict__ bias, int w, int l,
                                         const f32x4 (&acc)[4][FM_CT]) {
#pragma unroll
    for (int b = 0; b < FM_CT; ++b) {
        const int col = 16 * (FM_CT * w + b) + (l & 15);
        const float bb = bias[col];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float v = acc[a][b][i] + bb;
                Hs[16 * a + 4 * (l >> 4) + i][col] = f2bf(v > 0.f ? v : 0.f);
            }
    }
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
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int64_t base = (int64_t)blockIdx.x * FM_ROWS;
    if (tid < FM_ROWS) {
        const int64_t i = base + tid;
        uint32_t x[SG_K0 / 2];
        bool ok = false;
        if (i < rows) {
            row_input(F, offs, gkeys, orders, gid, i, row0, spad, S, seed, x, &ok);
        } else {
#pragma unroll
            for (int c = 0; c < SG_K0 / 2; ++c) x[c] = 0;
        }
        okrow[tid] = ok ? 1 : 0;
        uint4 *dst = reinterpret_cast<uint4 *>(&Hs[tid][0]);
#pragma unroll
        for (int c = 0; c < SG_K0 / 8; ++c) dst[c] = uint4{x[4 * c], x[4 * c + 1], x[4 * c + 2], x[4 * c + 3]};
    }
    __syncthreads();
    f32x4 acc[4][FM_CT];
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
    // wave's columns, reduced across the 16 lanes that share rows
    float sum[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) sum[a][i] = 0.f;
#pragma unroll
    for (int b = 0; b < FM_CT; ++b) {
        const int col = 16 * (FM_CT * w + b) + (l & 15);
        const float bb = p[SG_OFF_B3 + col], w4 = p[SG_OFF_W4 + col];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float v = acc[a][b][i] + bb;
                sum[a][i] += bf2f(f2bf(v > 0.f ? v : 0.f)) * w4;
            }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float v = sum[a][i];
            for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m);
            if ((l & 15) == 0) part[w][16 * a + 4 * (l >> 4) + i] = v;
        }
    __syncthreads();
    if (tid < FM_ROWS) {
        const int64_t i = base + tid;
        if (i < rows) {
            float sc = p[SG_OFF_B4];
#pragma unroll
            for (int v = 0; v < FM_WAVES; ++v) sc += part[v][tid];
            if (keys) {
                const int64_t smp = (row0 + i) % spad;
                keys[i] = okrow[tid] ? (((unsigned long long)orderable(sc) << 32) | (uint64_t)smp) : ~0ull;
            } else {
                score[i] = okrow[tid] ? sc : INFINITY;
            }
        }
    }
}

// targets y = T / LB - 1 (LB: largest machine lower bound of the group)
__global__ void target_kernel(const tgo_task *__restrict__ tasks, const int32_t *__restrict__ offs,
                              const int32_t *__restrict__ gid, const int64_t *__restrict__ T, int rows,
                              float *y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    const int g = gid[i];
    const tgo_task *t = tasks + offs[g];
    const int n = offs[g + 1] - offs[g];
    int64_t sh = 0, sk = 0, sd = 0, mh = INT64_MAX, md = INT64_MAX, mkd = INT64_MAX, mhk = INT64_MAX;
    for (int x = 0; x < n; ++x) {
        const int64_t h = t[x].htd_ns, k = t[x].kern_ns, d = t[x].dth_ns;
        sh += h; sk += k; sd += d;
        mh = h < mh ? h : mh;
        md = d < md ? d : md;
        mkd = k + d < mkd ? k + d : mkd;
        mhk = h + k < mhk ? h + k : mhk;
    }
    int64_t lb = sh + mkd;
    lb = mh + sk + md > lb ? mh + sk + md : lb;
    lb = mhk + sd > lb ? mhk + sd : lb;
    lb = lb < 1 ? 1 : lb;
    y[i] = (float)((double)T[i] / (double)lb - 1.0);
}

// dscore = 2 (score - y) / rows;  loss = mean (score - y)^2 (atomic sum)
__global__ void loss_kernel(const float *__restrict__ score, const float *__restrict__ y, int rows,
                            float *dscore, float *loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float e = 0.f;
    if (i < rows) {
        const float d = score[i] - y[i];
        dscore[i] = 2.f * d / (float)rows;
        e = d * d / (float)rows;
    }
    for (int m = 32; m >= 1; m >>= 1) e += __shfl_xor(e, m);
    if ((threadIdx.x & 63) == 0) atomicAdd(loss, e);
}

// dh3 = dscore w4 * (h3 > 0), bf16 [rows][256] and [256][rows] (one wave per row)
__global__ void head_bwd_kernel(const uint16_t *__restrict__ H3, const float *__restrict__ w4,
                                const float *__restrict__ dscore, int rows, uint16_t *dH, uint16_t *dHt) {
    const int row = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const int l = threadIdx.x & 63;
    if (row >= rows) return;
    const float ds = dscore[row];
    for (int j = 0; j < 4; ++j) {
        const int c = l * 4 + j;
        const float h = bf2f(H3[(int64_t)row * SG_H + c]);
        const uint16_t g = f2bf(h > 0.f ? ds * w4[c] : 0.f);
        dH[(int64_t)row * SG_H + c] = g;
        dHt[(int64_t)c * rows + row] = g;
    }
}

// grad w4[c] = sum_i dscore_i h3[i][c] from the transposed activations (block
// c < 256), grad b4 = sum_i dscore_i (block 256)
__global__ void head_wgrad_kernel(const uint16_t *__restrict__ H3t, const float *__restrict__ dscore, int rows,
                                  float *gw4, float *gb4) {
    const int c = blockIdx.x;
    float acc = 0.f;
    for (int i = threadIdx.x; i < rows; i += blockDim.x)
        acc += dscore[i] * (c < SG_H ? bf2f(H3t[(int64_t)c * rows + i]) : 1.f);
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m);
    __shared__ float red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float t = red[0] + red[1] + red[2] + red[3];
        if (c < SG_H) gw4[c] = t;
        else gb4[0] = t;
    }
}

// bias gradient: gb[c] = sum_i Gt[c][i] (rows of the transposed gradient)
__global__ void colsum_kernel(const uint16_t *__restrict__ Gt, int rows, float *gb) {
    const int c = blockIdx.x;
    float s = 0.f;
    for (int i = threadIdx.x; i < rows; i += blockDim.x) s += bf2f(Gt[(int64_t)c * rows + i]);
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
    __shared__ float red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) gb[c] = red[0] + red[1] + red[2] + red[3];
}

// first-layer weight gradient arrives as [256][64] (padded input); keep the 48 real columns
__global__ void pack_w1_grad_kernel(const float *__restrict__ g64, float *g48) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= SG_H * SG_FEAT) return;
    const int o = i / SG_FEAT, c = i % SG_FEAT;
    g48[i] = g64[o * SG_K0 + c];
}

// Adam on the float32 masters, then refresh the bf16 working copies
// (W [out][in] and Wt [in][out]; the first layer padded to 64 inputs).
struct AdamArgs {
    float lr, beta1, beta2, eps, c1, c2;  // c1 = 1 - beta1^t, c2 = 1 - beta2^t
};

__global__ void adam_kernel(float *p, const float *__restrict__ g, float *m, float *v, int count,
                            AdamArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = a.beta1 * m[i] + (1.f - a.beta1) * gi;
    const float vi = a.beta2 * v[i] + (1.f - a.beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
}

__global__ void refresh_bf16_kernel(const float *__restrict__ p, uint16_t *W1, uint16_t *W1t, uint16_t *W2,
                                    uint16_t *W2t, uint16_t *W3, uint16_t *W3t) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < SG_H * SG_K0) {
        const int o = i / SG_K0, c = i % SG_K0;
        const uint16_t b = c < SG_FEAT ? f2bf(p[SG_OFF_W1 + o * SG_FEAT + c]) : (uint16_t)0;
        W1[o * SG_K0 + c] = b;
        W1t[c * SG_H + o] = b;
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
// the 64 smallest of every run of 1024 keys (bitonic sort in LDS).


constexpr int TK_RUN = 1024;
constexpr int TK_THREADS = 256;
constexpr int TK_KEEP = 64;

// in: [G][len] keys (group stride in_stride); out: [G][ceil(len/TK_RUN)*64]
__global__ __launch_bounds__(TK_THREADS) void topk_pass_kernel(const unsigned long long *__restrict__ in,
                                                         int64_t in_stride, int64_t len, int runs,
                                                         unsigned long long *out, int64_t out_stride) {
    __shared__ unsigned long long s[TK_RUN];
    const int g = blockIdx.y, run = blockIdx.x;
    const int64_t base = (int64_t)run * TK_RUN;
    for (int i = threadIdx.x; i < TK_RUN; i += blockDim.x)
        s[i] = base + i < len ? in[(int64_t)g * in_stride + base + i] : ~0ull;
    __syncthreads();
    for (int k = 2; k <= TK_RUN; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < TK_RUN; i += blockDim.x) {
                const int p = i ^ j;
                if (p > i) {
                    const bool up = (i & k) == 0;
                    const unsigned long long a = s[i], b = s[p];
                    if ((a > b) == up) { s[i] = b; s[p] = a; }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < TK_KEEP; i += blockDim.x)
        out[(int64_t)g * out_stride + (int64_t)run * TK_KEEP + i] = s[i];
}

__global__ void fill_u64_kernel(unsigned long long *p, int64_t n, unsigned long long v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// results: best of candidates (exact) and the heuristic
__global__ void search_finish_kernel(const int32_t *__restrict__ offs, int G, uint64_t seed,
                                     const uint32_t *__restrict__ gkeys,
                                     const int32_t *__restrict__ status,
                                     const unsigned long long *__restrict__ best,
                                     const uint8_t *__restrict__ horders, const int64_t *__restrict__ hns,
                                     tgo_search_result *out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    tgo_search_result r;
    const int n = offs[g + 1] - offs[g];
    r.n = n;
    r.status = status[g];
    r.pad = 0;
    for (int i = 0; i < 16; ++i) r.best[i] = 0xff;
    r.heur_ns = hns[g];
    if (r.status != 0 || best[g] == ~0ull) {
        r.best_ns = r.status != 0 ? r.status : r.heur_ns;
        r.cand_best_ns = -1;
        r.best_sample = 0;
        r.from_heuristic = r.status != 0 ? 0 : 1;
        if (r.status == 0)
            for (int i = 0; i < n; ++i) r.best[i] = horders[(int64_t)g * 16 + i];
        out[g] = r;
        return;
    }
    const int64_t cT = (int64_t)(best[g] >> 32);
    const uint64_t cs = best[g] & 0xffffffffull;
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

struct tgo_surrogate {
    int device = 0;
    int64_t max_rows = 0;
    int64_t step = 0;
    void *mem = nullptr;
    // parameters
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr, *gw1 = nullptr;
    uint16_t *W1 = nullptr, *W1t = nullptr, *W2 = nullptr, *W2t = nullptr, *W3 = nullptr, *W3t = nullptr;
    // activations (rows x width)
    uint16_t *X = nullptr, *Xt = nullptr, *H1 = nullptr, *H1t = nullptr, *H2 = nullptr, *H2t = nullptr;
    uint16_t *H3 = nullptr, *H3t = nullptr, *D3 = nullptr, *D3t = nullptr, *D2 = nullptr, *D2t = nullptr;
    uint16_t *D1 = nullptr, *D1t = nullptr;
    float *score = nullptr, *y = nullptr, *dscore = nullptr, *F = nullptr;
    uint8_t *valid = nullptr;
    int max_groups = 0;
    int32_t *status = nullptr;
    uint8_t *horders = nullptr;
    int64_t *hns = nullptr;
    unsigned long long *best = nullptr, *keys = nullptr;
    unsigned long long *cand[2] = {nullptr, nullptr};
    size_t cand_bytes = 0;
};

namespace tgo {

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

static int sur_forward(tgo_surrogate *s, int64_t rows, bool keep_t, hipStream_t st) {
    // rows is a multiple of 64; X holds the first-layer input
    GemmOut o{};
    o.bias = s->p + SG_OFF_B1;
    o.Y = s->H1;
    o.Yt = keep_t ? s->H1t : nullptr;
    gemm<EPI_BIAS | EPI_RELU>(s->X, s->W1, (int)rows, SG_H, SG_K0, o, st);
    o.bias = s->p + SG_OFF_B2;
    o.Y = s->H2;
    o.Yt = keep_t ? s->H2t : nullptr;
    gemm<EPI_BIAS | EPI_RELU>(s->H1, s->W2, (int)rows, SG_H, SG_H, o, st);
    o.bias = s->p + SG_OFF_B3;
    o.Y = s->H3;
    o.Yt = keep_t ? s->H3t : nullptr;
    gemm<EPI_BIAS | EPI_RELU>(s->H2, s->W3, (int)rows, SG_H, SG_H, o, st);
    return TGO_OK;
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
    s->max_groups = max_groups;
    (void)hipGetDevice(&s->device);
    const size_t R = (size_t)max_rows;
    std::vector<std::pair<void **, size_t>> parts = {
        {(void **)&s->p, 4 * SG_NPARAM}, {(void **)&s->g, 4 * SG_NPARAM}, {(void **)&s->m, 4 * SG_NPARAM},
        {(void **)&s->v, 4 * SG_NPARAM}, {(void **)&s->gw1, 4 * SG_H * SG_K0},
        {(void **)&s->W1, 2 * SG_H * SG_K0}, {(void **)&s->W1t, 2 * SG_H * SG_K0},
        {(void **)&s->W2, 2 * SG_H * SG_H}, {(void **)&s->W2t, 2 * SG_H * SG_H},
        {(void **)&s->W3, 2 * SG_H * SG_H}, {(void **)&s->W3t, 2 * SG_H * SG_H},
        {(void **)&s->X, 2 * R * SG_K0}, {(void **)&s->Xt, 2 * R * SG_K0},
        {(void **)&s->H1, 2 * R * SG_H}, {(void **)&s->H1t, 2 * R * SG_H},
        {(void **)&s->H2, 2 * R * SG_H}, {(void **)&s->H2t, 2 * R * SG_H},
        {(void **)&s->H3, 2 * R * SG_H}, {(void **)&s->H3t, 2 * R * SG_H},
        {(void **)&s->D3, 2 * R * SG_H}, {(void **)&s->D3t, 2 * R * SG_H},
        {(void **)&s->D2, 2 * R * SG_H}, {(void **)&s->D2t, 2 * R * SG_H},
        {(void **)&s->D1, 2 * R * SG_H}, {(void **)&s->D1t, 2 * R * SG_H},
        {(void **)&s->score, 4 * R}, {(void **)&s->y, 4 * R}, {(void **)&s->dscore, 4 * R},
        {(void **)&s->valid, R}, {(void **)&s->F, 4 * (size_t)max_groups * SG_POS * 3},
        {(void **)&s->status, 4 * (size_t)max_groups}, {(void **)&s->horders, 16 * (size_t)max_groups},
        {(void **)&s->hns, 8 * (size_t)max_groups}, {(void **)&s->best, 8 * (size_t)max_groups},
        {(void **)&s->keys, 8 * R},
    };
    size_t total = 0;
    for (auto &pt : parts) total += align256(pt.second);
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
    hipDeviceSynchronize();
    hipFree(s->mem);
    if (s->cand[0]) hipFree(s->cand[0]);
    if (s->cand[1]) hipFree(s->cand[1]);
    delete s;
}

static int refresh(tgo_surrogate *s, hipStream_t st) {
    hipLaunchKernelGGL(refresh_bf16_kernel, dim3((SG_H * SG_H + 255) / 256), dim3(256), 0, st, s->p, s->W1,
                       s->W1t, s->W2, s->W2t, s->W3, s->W3t);
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
    hipLaunchKernelGGL(group_status_kernel, dim3((G + 255) / 256), dim3(256), 0, st, d_tasks, d_offs, G, r,
                       d_status);
    const size_t shm = sizeof(Slot<uint32_t>) * SG_THREADS * SG_POS;
    const int64_t tiles = per_group / 64 * G;
    const int blocks = (int)std::min<int64_t>((tiles + 3) / 4, 8192);
    hipLaunchKernelGGL(pairs_kernel, dim3(blocks), dim3(SG_THREADS), shm, st, d_tasks, d_offs, G, r, per_group,
                       seed, d_status, d_orders, d_gid, d_T);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

// features of given orderings into X (rows padded to a multiple of 64 with zero rows)
static int given_features(tgo_surrogate *s, const tgo_task *d_tasks, const int32_t *d_offs, int G,
                          const uint8_t *d_orders, const int32_t *d_gid, int64_t rows, bool with_t,
                          hipStream_t st) {
    hipLaunchKernelGGL(group_features_kernel, dim3((G * SG_POS + 255) / 256), dim3(256), 0, st, d_tasks, d_offs,
                       G, s->F);
    const int64_t pad = (rows + 63) / 64 * 64;
    if (pad > rows) TGO_HIP(hipMemsetAsync(s->X + rows * SG_K0, 0, 2 * (pad - rows) * SG_K0, st));
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, s->F, d_offs,
                       (const uint32_t *)nullptr, d_orders, d_gid, (int64_t)0, rows, (int64_t)1, (int64_t)1,
                       (uint64_t)0, s->X,
                       with_t ? s->Xt : (uint16_t *)nullptr, rows, (uint8_t *)nullptr);
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
    hipLaunchKernelGGL(mlp_fused_kernel, dim3((unsigned)((rows + FM_ROWS - 1) / FM_ROWS)), dim3(FM_THREADS), 0, st, s->F,
                       d_offs, (const uint32_t *)nullptr, d_orders, d_gid, (int64_t)0, rows, (int64_t)1, (int64_t)1,
                       (uint64_t)0, s->W1, s->W2, s->W3, s->p, d_scores, (unsigned long long *)nullptr);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

// forward + backward on a batch of pairs; gradient (float [NPARAM]) into s->g, loss into d_loss
static int sur_grad(tgo_surrogate *s, const tgo_task *d_tasks, const int32_t *d_offs, int G,
                    const uint8_t *d_orders, const int32_t *d_gid, const int64_t *d_T, int rows,
                    float *d_loss, hipStream_t st) {
    int rc = given_features(s, d_tasks, d_offs, G, d_orders, d_gid, rows, true, st);
    if (rc) return rc;
    rc = sur_forward(s, rows, true, st);
    if (rc) return rc;
    hipLaunchKernelGGL(head_kernel, dim3((unsigned)((rows * 64 + 255) / 256)), dim3(256), 0, st, s->H3,
                       s->p + SG_OFF_W4, s->p + SG_OFF_B4, (int64_t)rows, (const uint8_t *)nullptr, s->score);
    hipLaunchKernelGGL(target_kernel, dim3((rows + 255) / 256), dim3(256), 0, st, d_tasks, d_offs, d_gid, d_T,
                       rows, s->y);
    TGO_HIP(hipMemsetAsync(d_loss, 0, 4, st));
    TGO_HIP(hipMemsetAsync(s->g, 0, 4 * SG_NPARAM, st));
    hipLaunchKernelGGL(loss_kernel, dim3((rows + 255) / 256), dim3(256), 0, st, s->score, s->y, rows, s->dscore,
                       d_loss);
    hipLaunchKernelGGL(head_bwd_kernel, dim3((unsigned)((rows * 64 + 255) / 256)), dim3(256), 0, st, s->H3,
                       s->p + SG_OFF_W4, s->dscore, rows, s->D3, s->D3t);
    hipLaunchKernelGGL(head_wgrad_kernel, dim3(SG_H + 1), dim3(256), 0, st, s->H3t, s->dscore, rows,
                       s->g + SG_OFF_W4, s->g + SG_OFF_B4);
    // layer 3: grad W3 = D3^T H2 ; grad b3 = colsum ; D2 = (D3 W3) * (H2 > 0)
    gemm_splitk(s->D3t, s->H2t, SG_H, SG_H, rows, s->g + SG_OFF_W3, st);
    hipLaunchKernelGGL(colsum_kernel, dim3(SG_H), dim3(256), 0, st, s->D3t, rows, s->g + SG_OFF_B3);
    GemmOut o{};
    o.Y = s->D2;
    o.Yt = s->D2t;
    o.mask = s->H2;
    gemm<EPI_MASK>(s->D3, s->W3t, rows, SG_H, SG_H, o, st);
    // layer 2
    gemm_splitk(s->D2t, s->H1t, SG_H, SG_H, rows, s->g + SG_OFF_W2, st);
    hipLaunchKernelGGL(colsum_kernel, dim3(SG_H), dim3(256), 0, st, s->D2t, rows, s->g + SG_OFF_B2);
    o = GemmOut{};
    o.Y = s->D1;
    o.Yt = s->D1t;
    o.mask = s->H1;
    gemm<EPI_MASK>(s->D2, s->W2t, rows, SG_H, SG_H, o, st);
    // layer 1: grad W1 = D1^T X
    TGO_HIP(hipMemsetAsync(s->gw1, 0, 4 * SG_H * SG_K0, st));
    gemm_splitk(s->D1t, s->Xt, SG_H, SG_K0, rows, s->gw1, st);
    hipLaunchKernelGGL(colsum_kernel, dim3(SG_H), dim3(256), 0, st, s->D1t, rows, s->g + SG_OFF_B1);
    hipLaunchKernelGGL(pack_w1_grad_kernel, dim3((SG_H * SG_FEAT + 255) / 256), dim3(256), 0, st, s->gw1,
                       s->g + SG_OFF_W1);
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
    rc = sur_grad(s, d_tasks, d_offs, G, d_orders, d_gid, d_T, rows, d_loss, st);
    if (rc) return rc;
    if (d_grad) TGO_HIP(hipMemcpyAsync(d_grad, s->g, 4 * SG_NPARAM, hipMemcpyDeviceToDevice, st));
    return TGO_OK;
}

int tgo_surrogate_train_step(tgo_surrogate *s, const tgo_task *d_tasks, const int32_t *d_offs, int G,
                             const uint8_t *d_orders, const int32_t *d_gid, const int64_t *d_T, int rows,
                             float lr, float *d_loss, tgo_stream stream) {
    int rc = tgo_surrogate_grad(s, d_tasks, d_offs, G, d_orders, d_gid, d_T, rows, nullptr, d_loss, stream);
    if (rc) return rc;
    if (!(lr > 0.f)) return fail(TGO_EINVAL, "lr must be > 0");
    hipStream_t st = (hipStream_t)stream;
    s->step += 1;
    AdamArgs a;
    a.lr = lr;
    a.beta1 = 0.9f;
    a.beta2 = 0.999f;
    a.eps = 1e-8f;
    a.c1 = (float)(1.0 - std::pow(0.9, (double)s->step));
    a.c2 = (float)(1.0 - std::pow(0.999, (double)s->step));
    hipLaunchKernelGGL(adam_kernel, dim3((SG_NPARAM + 255) / 256), dim3(256), 0, st, s->p, s->g, s->m, s->v,
                       SG_NPARAM, a);
    TGO_HIP(hipGetLastError());
    return refresh(s, st);
}

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

// The candidate stage of the search: sample, score and keep the TK_KEEP
// smallest keys of every group.  On return cand[*cur] holds per group a
// sorted list of *len keys (group stride *len) whose first TK_KEEP are the
// group's smallest keys.
static int search_candidates(tgo_surrogate *s, const Rates &r, const tgo_task *d_tasks, const int32_t *d_offs,
                             const uint32_t *d_keys, int G, int64_t samples, uint64_t seed, hipStream_t st,
                             int *cur_out, int64_t *len_out) {
    const int64_t chunk = s->max_rows / TK_RUN * TK_RUN;
    if (chunk < TK_RUN) return fail(TGO_EINVAL, "search needs max_rows >= 1024");
    const int64_t spad = (samples + TK_RUN - 1) / TK_RUN * TK_RUN;
    const int64_t runs = spad / TK_RUN;
    int rc = grow_cand(s, sizeof(unsigned long long) * (size_t)G * (size_t)runs * TK_KEEP);
    if (rc) return rc;
    hipLaunchKernelGGL(group_status_kernel, dim3((G + 255) / 256), dim3(256), 0, st, d_tasks, d_offs, G, r,
                       s->status);
    hipLaunchKernelGGL(group_features_kernel, dim3((G * SG_POS + 255) / 256), dim3(256), 0, st, d_tasks, d_offs,
                       G, s->F);
    const int64_t total = (int64_t)G * spad;
    for (int64_t row0 = 0; row0 < total; row0 += chunk) {
        const int64_t rows = std::min(chunk, total - row0);
        // rows is a multiple of TK_RUN, hence of FM_ROWS
        hipLaunchKernelGGL(mlp_fused_kernel, dim3((unsigned)(rows / FM_ROWS)), dim3(FM_THREADS), 0, st, s->F, d_offs, d_keys,
                           (const uint8_t *)nullptr, (const int32_t *)nullptr, row0, rows, spad, samples, seed, s->W1,
                           s->W2, s->W3, s->p, (float *)nullptr, s->keys);
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
    hipLaunchKernelGGL(fill_u64_kernel, dim3((G + 255) / 256), dim3(256), 0, st, s->best, (int64_t)G, ~0ull);
    const size_t shm = sizeof(Slot<uint32_t>) * SG_THREADS * SG_POS;
    hipLaunchKernelGGL(rescore_kernel, dim3((G + 3) / 4), dim3(SG_THREADS), shm, st, d_tasks, d_offs, G, r, topk,
                       seed, s->status, d_keys, s->cand[cur], (int)len, s->best);
    hipLaunchKernelGGL(search_finish_kernel, dim3((G + 255) / 256), dim3(256), 0, st, d_offs, G, seed, d_keys,
                       s->status, s->best, s->horders, s->hns, d_out);
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
    const size_t need = (size_t)G * (4 + 16 + 8 + 8) + 1024;
    rc = workspace(need, (void **)&ws, st);
    if (rc) return rc;
    int32_t *status = (int32_t *)ws;
    int64_t *hns = (int64_t *)(ws + ((4 * (size_t)G + 255) & ~size_t(255)));
    unsigned long long *best = (unsigned long long *)((char *)hns + ((8 * (size_t)G + 255) & ~size_t(255)));
    uint8_t *horders = (uint8_t *)((char *)best + ((8 * (size_t)G + 255) & ~size_t(255)));
    hipLaunchKernelGGL(group_status_kernel, dim3((G + 255) / 256), dim3(256), 0, st, d_tasks, d_offs, G, r, status);
    rc = launch_heuristic(r, d_tasks, d_offs, G, horders, 16, hns, 1, st);
    if (rc) return rc;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((G + 255) / 256), dim3(256), 0, st, best, (int64_t)G, ~0ull);
    if (per > 0) {
        const size_t shm = sizeof(Slot<uint32_t>) * SG_THREADS * SG_POS;
        // chunks of up to 64 tiles, while keeping at least ~64k wave tasks
        const int64_t tiles = per / 64 * G;
        const int64_t chunk_tiles = std::max<int64_t>(1, std::min<int64_t>(64, tiles >> 16));
        const int64_t chunks = (per / 64 + chunk_tiles - 1) / chunk_tiles * G;
        const int blocks = (int)std::min<int64_t>((chunks + 3) / 4, 16384);
        hipLaunchKernelGGL(random_search_kernel, dim3(blocks), dim3(SG_THREADS), shm, st, d_tasks, d_offs, G, r,
                           per, seed, chunk_tiles, status, best);
    }
    hipLaunchKernelGGL(search_finish_kernel, dim3((G + 255) / 256), dim3(256), 0, st, d_offs, G, seed,
                       (const uint32_t *)nullptr, status, best, horders, hns, d_out);
    TGO_HIP(hipGetLastError());
    return TGO_OK;
}

int tgo_surrogate_param_count(void) { return SG_NPARAM; }

}  // extern "C"
