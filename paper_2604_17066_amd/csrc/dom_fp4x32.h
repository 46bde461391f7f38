// Shared device code of the FP4 dominance contraction on 32 x 32 x 64
// matrix-core tiles: the dominance classification kernel (k_dom_mfma.hip),
// the persistent LABEL cascade (k_cascade_persist.hip) and the cascade's
// matrix-core round 0 (k_casc_head.hip) use it.
// Blocks are kMfBlock threads (kMfWaves wavefronts) unless a pass is given
// another block size.
#pragma once

#include "rsr_internal.h"

namespace rsr {
namespace mf {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kMfBlock = 512;
constexpr int kMfWaves = kMfBlock / 64;

__device__ __forceinline__ int expand8_fp4(uint32_t v) {
    // Bits b0..b7 of v (v < 256) -> nibbles 2*b0 .. 2*b7 (FP4 E2M1 1.0 = 0x2).
    v = (v | (v << 12)) & 0x000F000Fu;
    v = (v | (v << 6)) & 0x03030303u;
    v = (v | (v << 3)) & 0x11111111u;
    return static_cast<int>(v << 1);
}

// acc + 8 * (number of negative values among the four of a).  The values are
// first packed in pairs to int16 with saturation, which keeps their signs (for
// the FP4 form the raw fp32 bits are used: a negative float is a negative
// int32).  v_perm_b32 selector bytes 8..11 then replicate bits 15 / 31 of both
// sources into four bytes, and one accumulating popcount adds them: four VALU
// ops per v4i.  (Packing the FP4 form's floats with v_cvt_pkrtz_f16_f32
// instead is not safe: the compiler treats the second operand of that pack as
// unused in this pattern and drops it.)
__device__ __forceinline__ uint32_t add_negatives8(v4i a, uint32_t acc) {
    const uint32_t lo = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pk_i16(a.x, a.y));
    const uint32_t hi = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pk_i16(a.z, a.w));
    return static_cast<uint32_t>(__builtin_popcount(__builtin_amdgcn_perm(lo, hi, 0x0B0A0908u))) + acc;
}

// Signed minimum of the four values (for FP4 the raw fp32 bits: a negative
// float is a negative int32, which is all the test needs).
__device__ __forceinline__ int min4(v4i a) { return min(min(a.x, a.y), min(a.z, a.w)); }

// ---- FP4 form on 32 x 32 tiles ------------------------------------------------
//
// v_mfma_scale_f32_32x32x64_f8f6f4 contracts 64 k per instruction (twice the
// rows and samples of the 16 x 16 x 128 form, half its k), so a row of W
// packed words takes ceil(32 W / 64) steps: the bits rounded up to 64, as in
// the int8 form, instead of to 128 (295 bits: 320 k instead of 384).  Lane l
// supplies row / column l % 32 and nibbles j = 0..31 of k = 64 s + 32 (l / 32)
// + j, i.e. the whole packed word 2 s + l / 32.  The result lane l holds
// column l % 32 and, in register v, row 8 (v / 4) + 4 (l / 32) + v % 4.
//
// Both sides contract +1 nibbles with a constant start of -1/2, so no
// per-row start is staged: the lower pass contracts NOT t(r) with t(x)
// (|t(x) & ~t(r)| - 1/2, negative iff x <= r), the upper pass t(r) with the
// complement of t(x) within the valid bits (|t(r) & ~t(x)| - 1/2, negative
// iff x >= r).  The complement is formed in registers by XOR with the FP4
// expansion of the valid-bit mask, since a sample has no pad bits set.

typedef float v16f __attribute__((ext_vector_type(16)));

__device__ __forceinline__ v16f mfma32_step(v4i a, v4i b, v16f acc) {
    const v8i a8 = {a.x, a.y, a.z, a.w, 0, 0, 0, 0};
    const v8i b8 = {b.x, b.y, b.z, b.w, 0, 0, 0, 0};
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a8, b8, acc, 4, 4, 0, 127, 0, 127);
}

typedef int v16i __attribute__((ext_vector_type(16)));

template <bool COUNT>
__device__ __forceinline__ int fold32(v16f r, int acc) {
    const v16i ri = __builtin_bit_cast(v16i, r);
    const v4i q0 = __builtin_shufflevector(ri, ri, 0, 1, 2, 3);
    const v4i q1 = __builtin_shufflevector(ri, ri, 4, 5, 6, 7);
    const v4i q2 = __builtin_shufflevector(ri, ri, 8, 9, 10, 11);
    const v4i q3 = __builtin_shufflevector(ri, ri, 12, 13, 14, 15);
    if (COUNT) {
        uint32_t u = static_cast<uint32_t>(acc);
        u = add_negatives8(q0, u);
        u = add_negatives8(q1, u);
        u = add_negatives8(q2, u);
        u = add_negatives8(q3, u);
        return static_cast<int>(u);
    }
    return min(acc, min(min(min4(q0), min4(q1)), min(min4(q2), min4(q3))));
}

// Reference tiles (32 rows) per staged group; the double-buffered stage takes
// 2 * TPS * KS KB of LDS.
template <int KS>
constexpr int tiles_per_stage32() {
    return KS <= 3 ? 10 : KS <= 5 ? 7 : (KS <= 10 ? 3 : 2);
}

// Sample tiles (32 samples) per wave: B fragments take 4 MT KS VGPRs and the
// two accumulator sets of the pipelined fold 32 MT (LABEL mode also keeps the
// vote state, so it allows one tile less from KS = 5 on).
template <int KS, bool COUNT>
constexpr int sample_tiles32() {
    return KS <= 4 ? 4 : KS == 5 ? (COUNT ? 4 : 3) : KS <= 8 ? 3 : KS <= 13 ? 2 : 1;
}

// A smaller count also built where the grid's last round of blocks matters
// (see prefer_alt).
template <int KS>
constexpr int sample_tiles32_alt() {
    return KS == 5 ? 2 : 0;
}

// fold32 over a tile whose rows from `rows` on are padding: their values
// (which start at -1/2 like every row) are replaced by +1/2 first.  Row of
// value v in lane half h: 8 (v / 4) + 4 h + v % 4.
template <bool COUNT>
__device__ __forceinline__ int fold32_last(v16f r, int acc, int rows, int half) {
#pragma unroll
    for (int v = 0; v < 16; ++v)
        if (8 * (v / 4) + 4 * half + v % 4 >= rows) r[v] = 0.5f;
    return fold32<COUNT>(r, acc);
}

// One pass over the 32-row tiles of one side (R rows).  acc_out[t] = 8 *
// matches (COUNT) or the running signed minimum (LABEL) for this lane's
// column of sample tile t, over this lane's 16 rows of each tile.
template <int KS, int MT, bool COUNT, int TPS = tiles_per_stage32<KS>(), int BLOCK = kMfBlock>
__device__ __forceinline__ void mfma32_pass(const v4i (&bf)[MT][KS], const v4i* __restrict__ frag,
                                            int64_t R, v4i* __restrict__ lds, int (&acc_out)[MT],
                                            const bool (&pre_done)[MT], const bool (&valid)[MT],
                                            int* vote) {
    constexpr int kTileV4 = KS * 64;  // operand v4i per reference tile
    constexpr int kStageV4 = TPS * kTileV4;
    constexpr int kPerThread = (kStageV4 + BLOCK - 1) / BLOCK;
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5;
    if (R <= 0) return;
    const int tiles = static_cast<int>((R + 31) / 32);
    const int last_rows = static_cast<int>(R - 32 * static_cast<int64_t>(tiles - 1));
    const int groups = (tiles + TPS - 1) / TPS;

    // Each thread stages the same slots of every group (slot q = element idx
    // of the group's contiguous fragments).
    v4i stage[kPerThread];
    int slot_tile[kPerThread];
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
        const int idx = q * BLOCK + threadIdx.x;
        slot_tile[q] = idx < kStageV4 ? idx / kTileV4 : 1 << 30;
    }
    auto fetch = [&](int G) {
        const v4i* src = frag + static_cast<int64_t>(G) * kStageV4 + threadIdx.x;
#pragma unroll
        for (int q = 0; q < kPerThread; ++q) {
            v4i v = {0, 0, 0, 0};
            if (G * TPS + slot_tile[q] < tiles) v = src[q * BLOCK];
            stage[q] = v;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < kPerThread; ++q) {
            const int idx = q * BLOCK + threadIdx.x;
            if (idx < kStageV4) lds[buf * kStageV4 + idx] = stage[q];
        }
    };

    const v16f start = v16f{} - 0.5f;
    v16f prev[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) prev[t] = start;
    fetch(0);
    store(0);
    __syncthreads();
    for (int G = 0; G < groups; ++G) {
        const int cur = G & 1;
        if (G + 1 < groups) fetch(G + 1);
        const int in_group = tiles - G * TPS < TPS ? tiles - G * TPS : TPS;
        for (int tt = 0; tt < in_group; ++tt) {
            __builtin_amdgcn_sched_barrier(0);
            const v4i* tile = lds + cur * kStageV4 + tt * kTileV4;
            v4i a[KS];
#pragma unroll
            for (int s = 0; s < KS; ++s) a[s] = tile[s * 64 + lane];
            v16f acc[MT];
            constexpr bool kPrio = KS * MT < 30;
            if constexpr (kPrio) __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int t = 0; t < MT; ++t)
                    acc[t] = mfma32_step(a[s], bf[t][s], s == 0 ? start : acc[t]);
            if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
            // The previous tile (a full one: only the last tile can be partial,
            // and it is folded after the loop).  Before the first tile prev
            // holds -1/2 starts that no row produced: skip it.
            if (G + tt > 0) {
#pragma unroll
                for (int t = 0; t < MT; ++t) acc_out[t] = fold32<COUNT>(prev[t], acc_out[t]);
            }
#pragma unroll
            for (int t = 0; t < MT; ++t) prev[t] = acc[t];
#pragma unroll
            for (int t = 0; t < MT; ++t) asm volatile("" ::"v"(acc_out[t]));
        }
        if (G + 1 < groups) store(cur ^ 1);
        bool leave = false;
        if (!COUNT) {
            bool done = true;
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                int m = min(acc_out[t], __shfl_xor(acc_out[t], 32));
                done = done && (!valid[t] || pre_done[t] || m < 0);
            }
            const int wave_done = __all(done) ? 1 : 0;
            if (lane == 0) vote[threadIdx.x >> 6] = wave_done;
            __syncthreads();
            int all = 1;
#pragma unroll
            for (int w = 0; w < BLOCK / 64; ++w) all &= vote[w];
            // A pass left early never reaches the last tile: the tile in prev
            // is full (the last tile can only be in prev after the loop).
            leave = all != 0 && G + 1 < groups;
        }
        __syncthreads();
        if (leave) {
#pragma unroll
            for (int t = 0; t < MT; ++t) acc_out[t] = fold32<COUNT>(prev[t], acc_out[t]);
            return;
        }
    }
#pragma unroll
    for (int t = 0; t < MT; ++t) acc_out[t] = fold32_last<COUNT>(prev[t], acc_out[t], last_rows, half);
}

// Valid-bit mask of packed word w of an n-component sample (plane-major
// thermometer words of PW words each, pad bits 0); 0 past the W words.
__device__ __forceinline__ uint32_t valid_word(int w, int n, int PW, int W) {
    if (w >= W) return 0u;
    const int left = n - 32 * (w % PW);
    return left >= 32 ? 0xFFFFFFFFu : ((1u << left) - 1u);
}

__device__ __forceinline__ v4i expand_word_fp4(uint32_t bits) {
    v4i f;
    f.x = expand8_fp4(bits & 0xFFu);
    f.y = expand8_fp4((bits >> 8) & 0xFFu);
    f.z = expand8_fp4((bits >> 16) & 0xFFu);
    f.w = expand8_fp4(bits >> 24);
    return f;
}

// Sample operand of the wave's MT sample tiles (32 samples each): lane l holds
// sample wbase + 32 t + l % 32, and for k-step s its packed word 2 s + l / 32
// as 32 FP4 nibbles.
template <int KS, int MT>
__device__ __forceinline__ void load_samples32(const uint32_t* __restrict__ xs, int64_t stride,
                                               int64_t count, int W, int64_t wbase, int lane,
                                               v4i (&bf)[MT][KS], bool (&valid)[MT]) {
    const int col = lane & 31, half = lane >> 5;
    // Reads from clamped positions, all issued before any is used (reads
    // behind a condition make the wait counts cover every path).  Each
    // sample word is read once: the non-temporal hint keeps the stream from
    // evicting the reference fragments, which every block of an XCD re-reads
    // from its L2 (HBM fetch per graph2 launch 107 -> 63 MiB).
    uint32_t raw[MT][KS];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        const int64_t h = wbase + 32 * t + col;
        const int64_t hc = h < count ? h : count - 1;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int w = 2 * s + half;
            raw[t][s] = __builtin_nontemporal_load(xs + static_cast<int64_t>(w < W ? w : W - 1) * stride + hc);
        }
    }
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        valid[t] = wbase + 32 * t + col < count;
#pragma unroll
        for (int s = 0; s < KS; ++s)
            bf[t][s] = expand_word_fp4((valid[t] && 2 * s + half < W) ? raw[t][s] : 0u);
    }
}

}  // namespace mf
}  // namespace rsr
