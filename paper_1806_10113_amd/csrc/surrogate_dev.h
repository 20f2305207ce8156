// Device helpers of the learned proposal: counter-based sampling of
// orderings, per-position features, bfloat16 conversion.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tgo.h"
#include "model_dev.h"

namespace tgo {

constexpr int SG_POS = 16;       // positions per ordering (shorter groups padded at the tail)
constexpr int SG_FEAT = 48;      // 3 features per position
constexpr int SG_K0 = 64;        // first-layer input width (features zero-padded)
constexpr int SG_H = 256;        // hidden width
// parameter layout (fp32 masters and gradients): W1[256][48] b1[256]
// W2[256][256] b2[256] W3[256][256] b3[256] W4[256] b4[1]
constexpr int SG_OFF_W1 = 0;
constexpr int SG_OFF_B1 = SG_OFF_W1 + SG_H * SG_FEAT;
constexpr int SG_OFF_W2 = SG_OFF_B1 + SG_H;
constexpr int SG_OFF_B2 = SG_OFF_W2 + SG_H * SG_H;
constexpr int SG_OFF_W3 = SG_OFF_B2 + SG_H;
constexpr int SG_OFF_B3 = SG_OFF_W3 + SG_H * SG_H;
constexpr int SG_OFF_W4 = SG_OFF_B3 + SG_H;
constexpr int SG_OFF_B4 = SG_OFF_W4 + SG_H;
constexpr int SG_NPARAM = SG_OFF_B4 + 1;  // 144,385

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        U4 o;
        o.x = hi1 ^ c.y ^ k0;
        o.y = lo1;
        o.z = hi0 ^ c.w ^ k1;
        o.w = lo0;
        c = o;
    }
    return c;
}

// Ordering s of group g: Fisher-Yates from the last position down; position
// i takes j = hi32(x (i + 1)), x keeps lo32(x (i + 1)) and is reloaded from
// the next Philox word every four draws.  Returns the ordering as nibbles.
__device__ __forceinline__ uint64_t sample_ordering(int n, uint32_t g, uint64_t s, uint64_t seed) {
    U4 c;
    c.x = (uint32_t)s;
    c.y = (uint32_t)(s >> 32);
    c.z = g;
    c.w = 0;
    const U4 u = philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    uint64_t perm = 0;
    for (int i = n - 1; i >= 0; --i) perm = (perm << 4) | (uint64_t)i;
    uint32_t x = u.x;
    int k = 0;
    for (int i = n - 1; i >= 1; --i, ++k) {
        if (k == 4) x = u.y;
        if (k == 8) x = u.z;
        if (k == 12) x = u.w;
        const uint64_t p = (uint64_t)x * (uint64_t)(i + 1);
        const uint32_t j = (uint32_t)(p >> 32);
        x = (uint32_t)p;
        const uint64_t vi = (perm >> (4 * i)) & 15u, vj = (perm >> (4 * j)) & 15u;
        perm &= ~((15ull << (4 * i)) | (15ull << (4 * j)));
        perm |= (vi << (4 * j)) | (vj << (4 * i));
    }
    return perm;
}

// float -> bf16, round to nearest even (one v_cvt_pk_bf16_f32 on gfx950)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// log1p(x / 1 us) / log1p(20 ms / 1 us), in float32 as log2(1 + x) times
// ln 2 / ln 20001 with the hardware base-2 logarithm (a few float32 ulp of
// the exact value for durations of 100 ns and more; the network sees it
// rounded to bf16)
__device__ __forceinline__ float feature_value(int64_t x_ns) {
    constexpr float SCALE = (float)(0.69314718055994531 / 9.90353755128617);  // ln 2 / ln 20001
    return __log2f(1.0f + (float)x_ns * 1e-3f) * SCALE;
}

}  // namespace tgo
