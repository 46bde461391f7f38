// Dominance classification, matrix-core form: the violation matrix of the
// paper (section 3.3.2, eq. violation_matrix) as an int8 contraction on the
// gfx950 MFMA units, with int32 accumulation.
//
// Operands are the thermometer bits of rsr.h as bytes, k = packed bit index,
// encoded so that a row matches exactly when its accumulator is negative.  For
// a lower row r the A bytes are NOT t(r) in {0, 1} and the accumulator starts
// at -1: the result is |t(x) & ~t(r)| - 1, negative iff x <= r.  For an upper
// row the A bytes are -t(r) in {0, -1} and the start is |t(r)| - 1: the result
// is |t(r)| - |t(r) & t(x)| - 1 = |t(r) & ~t(x)| - 1, negative iff x >= r.
// Pad rows (R rounded up to 16) and pad tiles are all zero and never match.
//
// Two operand formats share the kernel.  int8: one v_mfma_i32_16x16x64_i8
// per 64 k, exact int32 accumulation.  FP4: 0 and +-1 are exact in FP4 E2M1
// (nibbles 0x0, 0x2, 0xA), so v_mfma_scale_f32_16x16x128_f8f6f4 with unit
// block scales contracts 128 k per instruction at twice the int8 rate, and the
// fp32 accumulator holds the same integers exactly (|sum| <= 4096 < 2^24).
// The FP4 starts are offset by 1/2 (-1/2 lower, |t(r)| - 1/2 upper, +1/2 pad)
// so that no accumulator is ever a signed zero; a match is still exactly a
// negative value, i.e. sign bit set, and the fold works on the raw bits.
//
// One v_mfma_i32_16x16x64_i8 multiplies a 16 x 64 tile of reference rows (A)
// by a 64 x 16 tile of samples (B).  Lane l supplies row / column l % 16 and
// the 16 bytes of k-chunk l / 16 of each operand; the result lane l holds rows
// 4 (l / 16) .. +3 of column l % 16.  A wave keeps the B fragments of MT
// sample tiles (16 MT samples) in VGPRs for the whole kernel (expanded once
// from the packed bits); the eight waves of a block share reference tiles,
// which are staged through LDS with double buffering, several tiles per
// barrier.  Reference rows are stored on the device in fragment order
// ([tile][k-step][lane][16 bytes]), so a tile is one contiguous block and every
// LDS read is one 16-byte access.
//
// The accumulators of a tile are folded into the per-sample result while the
// matrix products of the next tile run, so the VALU work hides under the
// MFMA pipe.  COUNT mode counts negative accumulators (a byte-sign permute and
// a popcount per pair, so 8 per match); LABEL mode keeps the signed minimum
// (negative = some row matched) and the block leaves a pass early when every
// sample is decided (vote once per staged group; lower-flagged samples are
// decided for the upper pass).
#include "compact.h"
#include "dom_fp4x32.h"

namespace rsr {
namespace {

using namespace mf;

// One k-step of the contraction: 64 k (int8) or 128 k (FP4) into acc.
template <bool FP4>
__device__ __forceinline__ v4i mfma_step(v4i a, v4i b, v4i acc) {
    if constexpr (FP4) {
        const v8i a8 = {a.x, a.y, a.z, a.w, 0, 0, 0, 0};
        const v8i b8 = {b.x, b.y, b.z, b.w, 0, 0, 0, 0};
        // Formats 4/4 = FP4 E2M1 for A and B; block scales 127 = 2^0 (E8M0).
        const v4f r = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
            a8, b8, __builtin_bit_cast(v4f, acc), 4, 4, 0, 127, 0, 127);
        return __builtin_bit_cast(v4i, r);
    } else {
        return __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc, 0, 0, 0);
    }
}

constexpr int kBlock = 512;
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ int expand4(uint32_t v) {
    // Bits b0..b3 of v (v < 16) -> bytes b0, b1, b2, b3.
    return static_cast<int>((v * 0x00204081u) & 0x01010101u);
}

template <int MT, bool COUNT, bool FP4>
__device__ __forceinline__ void fold(const v4i (&r)[MT], int (&acc_out)[MT]) {
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        if (COUNT)
            acc_out[t] = static_cast<int>(add_negatives8(r[t], static_cast<uint32_t>(acc_out[t])));
        else
            acc_out[t] = min(acc_out[t], min4(r[t]));
    }
}

// Reference tiles staged per barrier.  One block fills a CU (two waves per
// SIMD), so the barrier at the end of a group idles the whole CU; large groups
// make that rare and give the global loads of the next group a whole group of
// matrix work to land.  The double-buffered stage takes 2 * TPS * (KS KB +
// 64 B) of LDS, at most 83 KB (75 KB at KS = 3, where twelve tiles measure
// faster than eight).
template <int KS>
constexpr int tiles_per_stage() {
    return KS == 3 ? 12 : KS <= 5 ? 8 : (KS <= 10 ? 4 : 2);
}

// Reference tiles per stage of the cascade's FP4 kernels: eight at KS = 3
// (their short row ranges gain nothing from twelve), else as above.
template <int KS>
constexpr int casc_tiles_per_stage() {
    return KS == 3 ? 8 : tiles_per_stage<KS>();
}

// Sample tiles per wave: B fragments take MT * KS * 4 VGPRs, and with the two
// accumulator sets of the pipelined fold everything must fit 256 VGPRs (two
// waves per SIMD) without spilling.  This is the largest count that fits at
// each width (the FP4 instruction's 8-register operand slots raise the count
// a little); more tiles per wave means fewer LDS reads per matrix product.
template <int KS, bool FP4>
constexpr int sample_tiles() {
    if (FP4 && KS == 3) return 8;
    if (FP4 && KS >= 9) return 3;
    return KS <= 2 ? 8 : KS == 3 ? 7 : KS == 4 ? 6 : KS == 5 ? 5 : KS <= 10 ? 30 / KS
                                                                   : KS <= 13 ? 3 : 2;
}

// A smaller count also built for the widths of the 295-edge workloads (int8
// KS = 5, FP4 KS = 3), or 0.  One block fills a CU, so the grid runs in
// ceil(blocks / CUs) rounds and the last one may be mostly idle: at 10^6
// samples int8 with five tiles takes 7 rounds against 8 of four tiles, one of
// them 10 % full, and FP4 with eight tiles 4 rounds against 8.
template <int KS, bool FP4>
constexpr int sample_tiles_alt() {
    return (FP4 && KS == 3) || (!FP4 && KS == 5) ? 4 : 0;
}

// Tile count of the split-round kernel (FP4), which also holds the lowered
// flags and the compacted-sample indexing: the largest count that does not
// spill at each width, except KS = 10, where two tiles with a small spill
// measure faster than one.
template <int KS>
constexpr int casc_sample_tiles() {
    return KS <= 2 ? 8 : KS == 3 ? 4 : KS == 4 ? 6 : KS == 5 ? 3 : KS == 6 ? 4 : KS <= 8 ? 3 : 2;
}

// Whether the smaller count `alt` finishes N samples sooner than `mt`: a wave
// of MT tiles takes time about proportional to MT, so the cost of a count is
// MT times the rounds of blocks it needs over `cus` CUs; ties go to the larger
// count, whose staged reference tiles serve more samples.
inline bool prefer_alt(int64_t N, int cus, int mt, int alt) {
    if (alt <= 0 || cus <= 0) return false;
    auto cost = [&](int m) {
        const int64_t per_block = static_cast<int64_t>(kWaves) * 16 * m;
        const int64_t blocks = (N + per_block - 1) / per_block;
        return ((blocks + cus - 1) / cus) * m;
    };
    return cost(alt) < cost(mt);
}

// One pass over the tiles of one side.  acc_out[t] = 8 * matches (COUNT) or
// the running signed minimum (LABEL) for this lane's column of sample tile t.
// An LDS tile holds the KS*64 operand fragments followed by the 16
// accumulator starts, so the loop has no global load on its critical path;
// tiles past the end are staged as zeros (never a match), so every group
// runs all of its tiles without a branch.
template <int KS, int MT, bool COUNT, bool FP4, bool PRIO = (KS * MT < 30),
          int TPS = tiles_per_stage<KS>()>
__device__ __forceinline__ void mfma_pass(const v4i (&bf)[MT][KS], const v4i* __restrict__ frag,
                                          const v4i* __restrict__ cinit, int tiles,
                                          v4i* __restrict__ lds, int (&acc_out)[MT],
                                          const bool (&pre_done)[MT], const bool (&valid)[MT],
                                          int* vote) {
    constexpr int kFragV4 = KS * 64;      // operand v4i per reference tile
    constexpr int kTileV4 = kFragV4 + 4;  // plus 16 accumulator starts
    constexpr int kStageV4 = TPS * kTileV4;
    constexpr int kPerThread = (kStageV4 + kBlock - 1) / kBlock;
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 4;
    if (tiles <= 0) return;
    const int groups = (tiles + TPS - 1) / TPS;

    // Each thread stages the same slots of every group: slot q is element
    // `within` of tile t of the group, read from frag or cinit.  Its source
    // pointer and per-group stride are fixed here; a group only adds a
    // multiple of the stride.
    v4i stage[kPerThread];
    const v4i* src[kPerThread];
    int src_step[kPerThread], slot_tile[kPerThread];
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
        const int idx = q * kBlock + threadIdx.x;
        const int t = idx / kTileV4, within = idx % kTileV4;
        slot_tile[q] = idx < kStageV4 ? t : 1 << 30;  // out of the stage: never loaded
        const bool is_frag = within < kFragV4;
        src[q] = is_frag ? frag + static_cast<int64_t>(t) * kFragV4 + within
                         : cinit + static_cast<int64_t>(t) * 4 + (within - kFragV4);
        src_step[q] = is_frag ? TPS * kFragV4 : TPS * 4;
    }
    auto fetch = [&](int G) {
#pragma unroll
        for (int q = 0; q < kPerThread; ++q) {
            v4i v = {0, 0, 0, 0};
            if (G * TPS + slot_tile[q] < tiles) v = src[q][static_cast<int64_t>(G) * src_step[q]];
            stage[q] = v;
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < kPerThread; ++q) {
            const int idx = q * kBlock + threadIdx.x;
            if (idx < kStageV4) lds[buf * kStageV4 + idx] = stage[q];
        }
    };

    v4i prev[MT];  // accumulators of the previous tile, folded one tile late
#pragma unroll
    for (int t = 0; t < MT; ++t) prev[t] = v4i{0, 0, 0, 0};
    fetch(0);
    store(0);
    __syncthreads();
    for (int G = 0; G < groups; ++G) {
        const int cur = G & 1;
        if (G + 1 < groups) fetch(G + 1);
#pragma unroll
        for (int tt = 0; tt < TPS; ++tt) {
            // Nothing crosses a tile start, so the fold of the previous tile
            // (whose products are long finished) is scheduled among this
            // tile's products instead of right behind its own.
            __builtin_amdgcn_sched_barrier(0);
            const v4i* tile = lds + cur * kStageV4 + tt * kTileV4;
            const v4i c0 = tile[kFragV4 + grp];
            v4i a[KS];
#pragma unroll
            for (int s = 0; s < KS; ++s) a[s] = tile[s * 64 + lane];
            v4i acc[MT];
            // The two waves of a SIMD alternate between products and folds:
            // a wave issuing products goes first, so the matrix core is fed
            // while the other wave folds.  The priority changes keep the
            // products together, which needs more registers; PRIO is off
            // where that would spill (from KS * MT = 30 on, and in the
            // cascade kernels beyond KS = 3).
            constexpr bool kPrio = PRIO;
            if constexpr (kPrio) __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int t = 0; t < MT; ++t)
                    acc[t] = mfma_step<FP4>(a[s], bf[t][s], s == 0 ? c0 : acc[t]);
            if constexpr (kPrio) __builtin_amdgcn_s_setprio(0);
            fold<MT, COUNT, FP4>(prev, acc_out);
#pragma unroll
            for (int t = 0; t < MT; ++t) prev[t] = acc[t];
            // The empty asm pins the fold to this tile: otherwise it sinks to
            // the end of the group and waits there for the last products.
#pragma unroll
            for (int t = 0; t < MT; ++t) asm volatile("" ::"v"(acc_out[t]));
        }
        if (G + 1 < groups) store(cur ^ 1);
        bool leave = false;
        if (!COUNT) {
            bool done = true;
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                int m = acc_out[t];
                m = min(m, __shfl_xor(m, 16));
                m = min(m, __shfl_xor(m, 32));
                done = done && (!valid[t] || pre_done[t] || m < 0);
            }
            const int wave_done = __all(done) ? 1 : 0;
            if (lane == 0) vote[threadIdx.x >> 6] = wave_done;
            __syncthreads();
            int all = 1;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) all &= vote[w];
            leave = all != 0;
        }
        __syncthreads();
        if (leave) break;
    }
    fold<MT, COUNT, FP4>(prev, acc_out);
}

// Sample operand of the wave's MT sample tiles (samples wbase .. +16 MT of
// the word-major array xs with row stride `stride`; those at or past `count`,
// or whose `done` word is set, are not valid).
//   int8: bytes 16*grp .. +15 of k-step s are packed bits 64 s + 16 grp .. +15,
//         i.e. half (grp & 1) of word 2 s + (grp >> 1).
//   FP4:  nibbles 32*grp .. +31 of k-step s are bits 128 s + 32 grp .. +31,
//         i.e. the whole word 4 s + grp.
// The reference fragments use the same positions, so A and B agree on the k
// of every operand element.  NT: the samples are read once per launch (the
// whole-set classification), so a non-temporal hint keeps them from evicting
// the reference fragments from L2; the cascade's split rounds read theirs
// once per chunk and keep them cached.
template <int KS, int MT, bool FP4, bool NT = false>
__device__ __forceinline__ void load_samples(const uint32_t* __restrict__ xs, int64_t stride,
                                             int64_t count, int W, int64_t wbase, int col, int grp,
                                             const uint32_t* __restrict__ done, v4i (&bf)[MT][KS],
                                             bool (&valid)[MT]) {
    // Every read is issued before any is used, from clamped positions (a
    // position past the end reads the last sample and is masked below): reads
    // behind a condition, or a word read that waits for the match word, would
    // each cost a memory round trip of their own.
    uint32_t raw[MT][KS], skip[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        const int64_t h = wbase + 16 * t + col;
        const int64_t hc = h < count ? h : count - 1;
        skip[t] = done ? done[hc] : 0u;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int w = FP4 ? 4 * s + grp : 2 * s + (grp >> 1);
            const uint32_t* at = xs + static_cast<int64_t>(w < W ? w : W - 1) * stride + hc;
            raw[t][s] = NT ? __builtin_nontemporal_load(at) : *at;
        }
    }
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        const int64_t h = wbase + 16 * t + col;
        valid[t] = h < count && skip[t] == 0u;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            v4i f;
            if constexpr (FP4) {
                const int w = 4 * s + grp;
                const uint32_t bits = (valid[t] && w < W) ? raw[t][s] : 0u;
                f.x = expand8_fp4(bits & 0xFFu);
                f.y = expand8_fp4((bits >> 8) & 0xFFu);
                f.z = expand8_fp4((bits >> 16) & 0xFFu);
                f.w = expand8_fp4(bits >> 24);
            } else {
                const int w = 2 * s + (grp >> 1);
                uint32_t bits = (valid[t] && w < W) ? raw[t][s] : 0u;
                bits = (bits >> (16 * (grp & 1))) & 0xFFFFu;
                f.x = expand4(bits & 0xFu);
                f.y = expand4((bits >> 4) & 0xFu);
                f.z = expand4((bits >> 8) & 0xFu);
                f.w = expand4(bits >> 12);
            }
            bf[t][s] = f;
        }
    }
}

template <int KS, int MT, bool COUNT, bool FP4>
__global__ __launch_bounds__(kBlock) void k_dom_mfma(
    const uint32_t* __restrict__ xs, int64_t N, int W, const v4i* __restrict__ low_frag,
    const v4i* __restrict__ low_c, int TL, const v4i* __restrict__ up_frag,
    const v4i* __restrict__ up_c, int TU, uint8_t* __restrict__ flags,
    uint32_t* __restrict__ match) {
    __shared__ v4i lds[2 * tiles_per_stage<KS>() * (KS * 64 + 4)];
    __shared__ int vote[kWaves];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int64_t wbase = (static_cast<int64_t>(blockIdx.x) * kWaves + wave) * (16 * MT);

    v4i bf[MT][KS];
    bool valid[MT];
    load_samples<KS, MT, FP4, true>(xs, N, N, W, wbase, col, grp, nullptr, bf, valid);

    int accL[MT], accU[MT];  // 0 = no match yet in both modes
    bool none[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        accL[t] = 0;
        accU[t] = 0;
        none[t] = false;
    }
    mfma_pass<KS, MT, COUNT, FP4>(bf, low_frag, low_c, TL, lds, accL, none, valid, vote);

    // Per-sample lower result across the four lane groups (COUNT: matches;
    // LABEL: negative iff some lower row matched).
    bool lowered[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        int m = accL[t];
        if (COUNT) {
            uint32_t u = static_cast<uint32_t>(m);
            u += static_cast<uint32_t>(__shfl_xor(static_cast<int>(u), 16));
            u += static_cast<uint32_t>(__shfl_xor(static_cast<int>(u), 32));
            m = static_cast<int>(u >> 3);
        } else {
            m = min(m, __shfl_xor(m, 16));
            m = min(m, __shfl_xor(m, 32));
        }
        accL[t] = m;
        lowered[t] = COUNT ? false : (m < 0);
    }
    bool skip_upper = false;
    if (!COUNT) {
        bool done = true;
#pragma unroll
        for (int t = 0; t < MT; ++t) done = done && (!valid[t] || lowered[t]);
        const int wave_done = __all(done) ? 1 : 0;
        if (lane == 0) vote[wave] = wave_done;
        __syncthreads();
        int all = 1;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) all &= vote[w];
        skip_upper = all != 0;
        __syncthreads();
    }
    if (!skip_upper) mfma_pass<KS, MT, COUNT, FP4>(bf, up_frag, up_c, TU, lds, accU, lowered, valid, vote);

#pragma unroll
    for (int t = 0; t < MT; ++t) {
        int m = accU[t];
        if (COUNT) {
            uint32_t u = static_cast<uint32_t>(m);
            u += static_cast<uint32_t>(__shfl_xor(static_cast<int>(u), 16));
            u += static_cast<uint32_t>(__shfl_xor(static_cast<int>(u), 32));
            m = static_cast<int>(u >> 3);
        } else {
            m = min(m, __shfl_xor(m, 16));
            m = min(m, __shfl_xor(m, 32));
        }
        accU[t] = m;
    }
    if (grp == 0) {
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            if (!valid[t]) continue;
            const int64_t h = wbase + 16 * t + col;
            uint8_t f;
            if (COUNT) {
                f = static_cast<uint8_t>((accL[t] ? 1 : 0) | (accU[t] ? 2 : 0));
                if (match) {
                    match[2 * h] = static_cast<uint32_t>(accL[t]);
                    match[2 * h + 1] = static_cast<uint32_t>(accU[t]);
                }
            } else {
                f = static_cast<uint8_t>(lowered[t] ? 1 : (accU[t] < 0 ? 2 : 0));
            }
            flags[h] = f;
        }
    }
}

template <int KS, int MT, bool COUNT>
__global__ __launch_bounds__(kBlock) void k_dom_fp4x32(
    const uint32_t* __restrict__ xs, int64_t N, int n, int PW, int W,
    const v4i* __restrict__ low_frag, int64_t R_L, const v4i* __restrict__ up_frag, int64_t R_U,
    uint8_t* __restrict__ flags, uint32_t* __restrict__ match) {
    __shared__ v4i lds[2 * tiles_per_stage32<KS>() * KS * 64];
    __shared__ int vote[kWaves];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t wbase = (static_cast<int64_t>(blockIdx.x) * kWaves + wave) * (32 * MT);

    v4i bf[MT][KS];
    bool valid[MT];
    load_samples32<KS, MT>(xs, N, N, W, wbase, lane, bf, valid);

    int accL[MT], accU[MT];
    bool none[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        accL[t] = 0;
        accU[t] = 0;
        none[t] = false;
    }
    mfma32_pass<KS, MT, COUNT>(bf, low_frag, R_L, lds, accL, none, valid, vote);
    bool lowered[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        int m = accL[t];
        if (COUNT) {
            const uint32_t u = static_cast<uint32_t>(m) +
                               static_cast<uint32_t>(__shfl_xor(static_cast<int>(m), 32));
            m = static_cast<int>(u >> 3);
        } else {
            m = min(m, __shfl_xor(m, 32));
        }
        accL[t] = m;
        lowered[t] = COUNT ? false : (m < 0);
    }
    bool skip_upper = false;
    if (!COUNT) {
        bool done = true;
#pragma unroll
        for (int t = 0; t < MT; ++t) done = done && (!valid[t] || lowered[t]);
        const int wave_done = __all(done) ? 1 : 0;
        if (lane == 0) vote[wave] = wave_done;
        __syncthreads();
        int all = 1;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) all &= vote[w];
        skip_upper = all != 0;
        __syncthreads();
    }
    if (!skip_upper) {
        // Upper pass on the complement of the samples within the valid bits.
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const v4i m = expand_word_fp4(valid_word(2 * s + (lane >> 5), n, PW, W));
#pragma unroll
            for (int t = 0; t < MT; ++t) bf[t][s] ^= m;
        }
        mfma32_pass<KS, MT, COUNT>(bf, up_frag, R_U, lds, accU, lowered, valid, vote);
    }
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        int m = accU[t];
        if (COUNT) {
            const uint32_t u = static_cast<uint32_t>(m) +
                               static_cast<uint32_t>(__shfl_xor(static_cast<int>(m), 32));
            m = static_cast<int>(u >> 3);
        } else {
            m = min(m, __shfl_xor(m, 32));
        }
        accU[t] = m;
    }
    if (lane < 32) {
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            if (!valid[t]) continue;
            const int64_t h = wbase + 32 * t + lane;
            uint8_t f;
            if (COUNT) {
                f = static_cast<uint8_t>((accL[t] ? 1 : 0) | (accU[t] ? 2 : 0));
                if (match) {
                    match[2 * h] = static_cast<uint32_t>(accL[t]);
                    match[2 * h + 1] = static_cast<uint32_t>(accU[t]);
                }
            } else {
                f = static_cast<uint8_t>(lowered[t] ? 1 : (accU[t] < 0 ? 2 : 0));
            }
            flags[h] = f;
        }
    }
}

// One chunk of a split LABEL round of the cascade (k_cascade.hip) in the FP4
// form: the compacted undecided samples (word-major, row stride cstride, their
// number on the device) against the reference tiles of chunk blockIdx.y of
// the round's tile ranges, both sides; a match is ORed into the sample's
// match word (bit0 lower, bit1 upper).  The tile ranges may reach a few rows
// outside the round's rows: on a consistent reference set any match decides
// the label, so testing a row early or twice changes nothing.
template <int KS, int MT>
__global__ __launch_bounds__(kBlock) void k_casc_mfma(
    const uint32_t* __restrict__ csrc, int64_t cstride,
    const unsigned long long* __restrict__ src_count, int W, const v4i* __restrict__ low_frag,
    const v4i* __restrict__ low_c, int lt0, int lt1, const v4i* __restrict__ up_frag,
    const v4i* __restrict__ up_c, int ut0, int ut1, uint32_t* __restrict__ match) {
    __shared__ v4i lds[2 * casc_tiles_per_stage<KS>() * (KS * 64 + 4)];
    __shared__ int vote[kWaves];
    const int64_t total = static_cast<int64_t>(*src_count);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int chunks = gridDim.y, c = blockIdx.y;
    const int nL = lt1 - lt0, nU = ut1 - ut0;
    const int cl0 = lt0 + static_cast<int>((static_cast<int64_t>(nL) * c) / chunks);
    const int cl1 = lt0 + static_cast<int>((static_cast<int64_t>(nL) * (c + 1)) / chunks);
    const int cu0 = ut0 + static_cast<int>((static_cast<int64_t>(nU) * c) / chunks);
    const int cu1 = ut0 + static_cast<int>((static_cast<int64_t>(nU) * (c + 1)) / chunks);
    constexpr int kFragV4 = KS * 64;
    constexpr int64_t kPerBlock = static_cast<int64_t>(kWaves) * 16 * MT;
    // Block-uniform loop (the passes synchronise the block).
    for (int64_t b0 = static_cast<int64_t>(blockIdx.x) * kPerBlock; b0 < total;
         b0 += static_cast<int64_t>(gridDim.x) * kPerBlock) {
        const int64_t wbase = b0 + static_cast<int64_t>(wave) * 16 * MT;
        v4i bf[MT][KS];
        bool valid[MT];
        load_samples<KS, MT, true>(csrc, cstride, total, W, wbase, col, grp, match, bf, valid);
        int accL[MT], accU[MT];
        bool none[MT], lowered[MT];
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            accL[t] = accU[t] = 0;
            none[t] = false;
        }
        mfma_pass<KS, MT, false, true, (KS <= 3), casc_tiles_per_stage<KS>()>(
            bf, low_frag + static_cast<int64_t>(cl0) * kFragV4,
            low_c + static_cast<int64_t>(cl0) * 4, cl1 - cl0, lds, accL,
            none, valid, vote);
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            int m = accL[t];
            m = min(m, __shfl_xor(m, 16));
            m = min(m, __shfl_xor(m, 32));
            lowered[t] = m < 0;
        }
        mfma_pass<KS, MT, false, true, (KS <= 3), casc_tiles_per_stage<KS>()>(
            bf, up_frag + static_cast<int64_t>(cu0) * kFragV4,
            up_c + static_cast<int64_t>(cu0) * 4, cu1 - cu0, lds, accU,
            lowered, valid, vote);
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            int m = accU[t];
            m = min(m, __shfl_xor(m, 16));
            m = min(m, __shfl_xor(m, 32));
            const uint32_t bits = (lowered[t] ? 1u : 0u) | (m < 0 ? 2u : 0u);
            if (grp == 0 && valid[t] && bits)
                atomicOr(&match[wbase + 16 * t + col], bits);
        }
    }
}

// A whole round of the LABEL cascade (k_cascade.hip) in the FP4 form when its
// rows are not split over chunks: the round's samples (the sample array
// itself in round 0, src_idx null; the compacted undecided samples later)
// against the tile ranges of both sides, then, in the same block, the flags
// of the decided samples (of all samples in the last round) and the
// compaction of the others into dst, with their words, indices and cleared
// match words.  Tile ranges may reach rows outside the round's rows: on a
// consistent reference set any match decides the label.
template <int KS, int MT>
__global__ __launch_bounds__(kBlock) void k_casc_mfma_round(
    SegSrc seg, const uint32_t* __restrict__ csrc, int64_t cstride,
    const int32_t* __restrict__ src_idx, const unsigned long long* __restrict__ src_count,
    int64_t host_count, int W, const v4i* __restrict__ low_frag, const v4i* __restrict__ low_c,
    int lt0, int lt1, const v4i* __restrict__ up_frag, const v4i* __restrict__ up_c, int ut0,
    int ut1, uint32_t* __restrict__ dst, int32_t* __restrict__ dst_idx,
    uint32_t* __restrict__ dst_match, int64_t dst_stride,
    unsigned long long* __restrict__ dst_count, int last) {
    constexpr int kFragV4 = KS * 64;
    constexpr int kPerBlock = kWaves * 16 * MT;
    __shared__ v4i lds[2 * casc_tiles_per_stage<KS>() * (KS * 64 + 4)];
    __shared__ int vote[kWaves];
    __shared__ uint8_t s_bits[kPerBlock];
    __shared__ int s_counts[kWaves];
    __shared__ unsigned long long s_base;
    const int64_t total = src_count ? static_cast<int64_t>(*src_count) : host_count;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    // Block-uniform loop (the passes and the compaction synchronise the block).
    for (int64_t b0 = static_cast<int64_t>(blockIdx.x) * kPerBlock; b0 < total;
         b0 += static_cast<int64_t>(gridDim.x) * kPerBlock) {
        const int64_t wbase = b0 + static_cast<int64_t>(wave) * 16 * MT;
        v4i bf[MT][KS];
        bool valid[MT];
        load_samples<KS, MT, true>(csrc, cstride, total, W, wbase, col, grp, nullptr, bf, valid);
        int accL[MT], accU[MT];
        bool none[MT], lowered[MT];
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            accL[t] = accU[t] = 0;
            none[t] = false;
        }
        mfma_pass<KS, MT, false, true, (KS <= 3), casc_tiles_per_stage<KS>()>(
            bf, low_frag + static_cast<int64_t>(lt0) * kFragV4,
            low_c + static_cast<int64_t>(lt0) * 4, lt1 - lt0, lds, accL,
            none, valid, vote);
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            int m = accL[t];
            m = min(m, __shfl_xor(m, 16));
            m = min(m, __shfl_xor(m, 32));
            lowered[t] = m < 0;
        }
        mfma_pass<KS, MT, false, true, (KS <= 3), casc_tiles_per_stage<KS>()>(
            bf, up_frag + static_cast<int64_t>(ut0) * kFragV4,
            up_c + static_cast<int64_t>(ut0) * 4, ut1 - ut0, lds, accU,
            lowered, valid, vote);
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            int m = accU[t];
            m = min(m, __shfl_xor(m, 16));
            m = min(m, __shfl_xor(m, 32));
            if (grp == 0)
                s_bits[wave * 16 * MT + 16 * t + col] =
                    static_cast<uint8_t>((lowered[t] ? 1u : 0u) | (m < 0 ? 2u : 0u));
        }
        __syncthreads();
        // One sample per thread (kPerBlock / kBlock passes, the same for all).
        for (int j0 = 0; j0 < kPerBlock; j0 += kBlock) {
            const int j = j0 + static_cast<int>(threadIdx.x);
            const int64_t d = b0 + j;
            const bool in = j < kPerBlock && d < total;
            const uint32_t bits = in ? s_bits[j] : 0u;
            const int64_t g = in ? (src_idx ? static_cast<int64_t>(src_idx[d]) : d) : 0;
            if (in && (bits || last)) {
                int job;
                int64_t h;
                seg_locate(seg, g, job, h);
                seg_flags(seg, job)[h] =
                    static_cast<uint8_t>((bits & 1u) ? 1 : ((bits & 2u) ? 2 : 0));
            }
            if (last) continue;
            const bool carry[1] = {in && bits == 0u};
            int64_t slot[1];
            block_reserve<kWaves, 1>(carry, dst_count, s_counts, &s_base, slot);
            if (carry[0]) {
                dst_idx[slot[0]] = static_cast<int32_t>(g);
                dst_match[slot[0]] = 0u;
                for (int w = 0; w < W; ++w) dst[w * dst_stride + slot[0]] = csrc[w * cstride + d];
            }
        }
        __syncthreads();
    }
}

// Blocks of `kernel` (kBlock threads) the device holds at once.  The
// cascade's round kernels read their sample count on the device and loop
// over it, so a grid beyond this only adds blocks that find no samples: the
// host's bound (all N samples) would launch thousands of them for a round
// that keeps a few thousand samples, in as many waves of one block per CU.
// Cached per kernel and device (0: not yet known).
int resident_blocks(const void* kernel, int (&cache)[RSR_MAX_DEVICES]) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= RSR_MAX_DEVICES) return 1 << 30;
    if (cache[dev] == 0) {
        int cus = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess ||
            per_cu <= 0)
            return 1 << 30;
        cache[dev] = per_cu * cus;
    }
    return cache[dev];
}

template <int KS>
hipError_t launch_round_ks(hipStream_t st, const rsr_refs* refs, const SegSrc& seg,
                           const uint32_t* csrc, int64_t cstride, const int32_t* src_idx,
                           const unsigned long long* src_count, int64_t host_count,
                           int64_t max_count, int l0, int l1, int u0, int u1, int grid_cap,
                           uint32_t* dst, int32_t* dst_idx, uint32_t* dst_match,
                           int64_t dst_stride, unsigned long long* dst_count, int last) {
    constexpr int MT = casc_sample_tiles<KS>();
    const int64_t per_block = static_cast<int64_t>(kWaves) * 16 * MT;
    static int cache[RSR_MAX_DEVICES] = {};
    const int resident = resident_blocks(reinterpret_cast<const void*>(k_casc_mfma_round<KS, MT>), cache);
    int64_t bx = (max_count + per_block - 1) / per_block;
    if (bx > grid_cap) bx = grid_cap;
    if (src_count && bx > resident) bx = resident;
    if (bx < 1) bx = 1;
    hipLaunchKernelGGL((k_casc_mfma_round<KS, MT>), dim3(static_cast<unsigned>(bx)), dim3(kBlock),
                       0, st, seg, csrc, cstride, src_idx, src_count, host_count, refs->W,
                       reinterpret_cast<const v4i*>(refs->d_lower_frag4),
                       reinterpret_cast<const v4i*>(refs->d_lower_cinit4), l0 / 16, (l1 + 15) / 16,
                       reinterpret_cast<const v4i*>(refs->d_upper_frag4),
                       reinterpret_cast<const v4i*>(refs->d_upper_cinit4), u0 / 16, (u1 + 15) / 16,
                       dst, dst_idx, dst_match, dst_stride, dst_count, last);
    return hipGetLastError();
}

template <int KS>
hipError_t launch_casc_ks(hipStream_t st, const rsr_refs* refs, const uint32_t* csrc,
                          int64_t cstride, const unsigned long long* src_count, int64_t max_count,
                          int l0, int l1, int u0, int u1, int chunks, int grid_cap,
                          uint32_t* match) {
    constexpr int MT = casc_sample_tiles<KS>();
    const int64_t per_block = static_cast<int64_t>(kWaves) * 16 * MT;
    static int cache[RSR_MAX_DEVICES] = {};
    const int resident = resident_blocks(reinterpret_cast<const void*>(k_casc_mfma<KS, MT>), cache);
    int64_t bx = (max_count + per_block - 1) / per_block;
    const int64_t cap = grid_cap / chunks > 0 ? grid_cap / chunks : 1;
    if (bx > cap) bx = cap;
    if (bx > resident / chunks) bx = resident / chunks;
    if (bx < 1) bx = 1;
    hipLaunchKernelGGL((k_casc_mfma<KS, MT>), dim3(static_cast<unsigned>(bx), chunks),
                       dim3(kBlock), 0, st, csrc, cstride, src_count, refs->W,
                       reinterpret_cast<const v4i*>(refs->d_lower_frag4),
                       reinterpret_cast<const v4i*>(refs->d_lower_cinit4), l0 / 16, (l1 + 15) / 16,
                       reinterpret_cast<const v4i*>(refs->d_upper_frag4),
                       reinterpret_cast<const v4i*>(refs->d_upper_cinit4), u0 / 16, (u1 + 15) / 16,
                       match);
    return hipGetLastError();
}

template <int KS, int MT, bool COUNT>
hipError_t launch_fp4x32_mt(hipStream_t st, const rsr_refs* refs, const uint32_t* xs, int64_t N,
                            uint8_t* flags, uint32_t* match) {
    const int64_t per_block = static_cast<int64_t>(kWaves) * 32 * MT;
    const dim3 grid(static_cast<unsigned>((N + per_block - 1) / per_block));
    hipLaunchKernelGGL((k_dom_fp4x32<KS, MT, COUNT>), grid, dim3(kBlock), 0, st, xs, N, refs->n,
                       plane_words(refs->n), refs->W,
                       reinterpret_cast<const v4i*>(refs->d_lower_frag32), refs->R_L,
                       reinterpret_cast<const v4i*>(refs->d_upper_frag32), refs->R_U, flags,
                       match);
    return hipGetLastError();
}

// Cost of a sample-tile count: blocks of kWaves * 32 * mt samples, one per CU
// at a time, each taking time about proportional to mt.
inline bool prefer_alt32(int64_t N, int cus, int mt, int alt) {
    if (alt <= 0 || cus <= 0) return false;
    auto cost = [&](int m) {
        const int64_t per_block = static_cast<int64_t>(kWaves) * 32 * m;
        const int64_t blocks = (N + per_block - 1) / per_block;
        return ((blocks + cus - 1) / cus) * m;
    };
    return cost(alt) < cost(mt);
}

template <int KS, bool COUNT>
hipError_t launch_fp4x32_mode(hipStream_t st, const rsr_refs* refs, const uint32_t* xs, int64_t N,
                              int cus, uint8_t* flags, uint32_t* match) {
    constexpr int MT = sample_tiles32<KS, COUNT>();
    constexpr int ALT = sample_tiles32_alt<KS>();
    if constexpr (ALT > 0) {
        if (prefer_alt32(N, cus, MT, ALT))
            return launch_fp4x32_mt<KS, ALT, COUNT>(st, refs, xs, N, flags, match);
    }
    return launch_fp4x32_mt<KS, MT, COUNT>(st, refs, xs, N, flags, match);
}

template <int KS>
hipError_t launch_fp4x32_ks(hipStream_t st, const rsr_refs* refs, const uint32_t* xs, int64_t N,
                            int mode, int cus, uint8_t* flags, uint32_t* match) {
    return mode == RSR_COUNT ? launch_fp4x32_mode<KS, true>(st, refs, xs, N, cus, flags, match)
                             : launch_fp4x32_mode<KS, false>(st, refs, xs, N, cus, flags, match);
}

template <int KS, int MT, bool FP4>
hipError_t launch_mt(hipStream_t st, const rsr_refs* refs, const uint32_t* xs, int64_t N,
                     int mode, uint8_t* flags, uint32_t* match) {
    const int64_t per_block = static_cast<int64_t>(kWaves) * 16 * MT;
    const dim3 grid(static_cast<unsigned>((N + per_block - 1) / per_block));
    const v4i* lf = reinterpret_cast<const v4i*>(FP4 ? refs->d_lower_frag4 : refs->d_lower_frag);
    const v4i* lc = FP4 ? reinterpret_cast<const v4i*>(refs->d_lower_cinit4)
                        : reinterpret_cast<const v4i*>(refs->d_lower_cinit);
    const v4i* uf = reinterpret_cast<const v4i*>(FP4 ? refs->d_upper_frag4 : refs->d_upper_frag);
    const v4i* uc = FP4 ? reinterpret_cast<const v4i*>(refs->d_upper_cinit4)
                        : reinterpret_cast<const v4i*>(refs->d_upper_cinit);
    if (mode == RSR_COUNT)
        hipLaunchKernelGGL((k_dom_mfma<KS, MT, true, FP4>), grid, dim3(kBlock), 0, st, xs, N,
                           refs->W, lf, lc, refs->TL, uf, uc, refs->TU, flags, match);
    else
        hipLaunchKernelGGL((k_dom_mfma<KS, MT, false, FP4>), grid, dim3(kBlock), 0, st, xs, N,
                           refs->W, lf, lc, refs->TL, uf, uc, refs->TU, flags, match);
    return hipGetLastError();
}

template <int KS, bool FP4>
hipError_t launch_ks(hipStream_t st, const rsr_refs* refs, const uint32_t* xs, int64_t N,
                     int mode, int cus, uint8_t* flags, uint32_t* match) {
    constexpr int MT = sample_tiles<KS, FP4>();
    constexpr int ALT = sample_tiles_alt<KS, FP4>();
    if constexpr (ALT > 0) {
        if (prefer_alt(N, cus, MT, ALT))
            return launch_mt<KS, ALT, FP4>(st, refs, xs, N, mode, flags, match);
    }
    return launch_mt<KS, MT, FP4>(st, refs, xs, N, mode, flags, match);
}

}  // namespace

hipError_t launch_dom_mfma(hipStream_t st, const rsr_refs* refs, const uint32_t* xs, int64_t N,
                           int mode, bool fp4, int cus, uint8_t* flags, uint32_t* match) {
    if (fp4) {
        // FP4 on 32 x 32 tiles: k-steps of 64, the same count as the int8 form.
        switch (refs->KS) {
#define RSR_KS_CASE(k) \
    case k: return launch_fp4x32_ks<k>(st, refs, xs, N, mode, cus, flags, match);
            RSR_KS_CASE(1) RSR_KS_CASE(2) RSR_KS_CASE(3) RSR_KS_CASE(4) RSR_KS_CASE(5)
            RSR_KS_CASE(6) RSR_KS_CASE(7) RSR_KS_CASE(8) RSR_KS_CASE(9) RSR_KS_CASE(10)
            RSR_KS_CASE(11) RSR_KS_CASE(12) RSR_KS_CASE(13) RSR_KS_CASE(14) RSR_KS_CASE(15)
            RSR_KS_CASE(16) RSR_KS_CASE(17) RSR_KS_CASE(18) RSR_KS_CASE(19) RSR_KS_CASE(20)
#undef RSR_KS_CASE
            default: return hipErrorInvalidValue;
        }
    }
    switch (refs->KS) {
#define RSR_KS_CASE(k) \
    case k: return launch_ks<k, false>(st, refs, xs, N, mode, cus, flags, match);
        RSR_KS_CASE(1) RSR_KS_CASE(2) RSR_KS_CASE(3) RSR_KS_CASE(4) RSR_KS_CASE(5)
        RSR_KS_CASE(6) RSR_KS_CASE(7) RSR_KS_CASE(8) RSR_KS_CASE(9) RSR_KS_CASE(10)
        RSR_KS_CASE(11) RSR_KS_CASE(12) RSR_KS_CASE(13) RSR_KS_CASE(14) RSR_KS_CASE(15)
        RSR_KS_CASE(16) RSR_KS_CASE(17) RSR_KS_CASE(18) RSR_KS_CASE(19) RSR_KS_CASE(20)
#undef RSR_KS_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_casc_mfma_round(hipStream_t st, const rsr_refs* refs, const SegSrc& seg,
                                  const uint32_t* csrc, int64_t cstride, const int32_t* src_idx,
                                  const unsigned long long* src_count, int64_t host_count,
                                  int64_t max_count, int l0, int l1, int u0, int u1, int grid_cap,
                                  uint32_t* dst, int32_t* dst_idx, uint32_t* dst_match,
                                  int64_t dst_stride, unsigned long long* dst_count, int last) {
    switch (refs->KS4) {
#define RSR_KS_CASE(k) \
    case k: return launch_round_ks<k>(st, refs, seg, csrc, cstride, src_idx, src_count, host_count, \
                                      max_count, l0, l1, u0, u1, grid_cap, dst, dst_idx, dst_match, \
                                      dst_stride, dst_count, last);
        RSR_KS_CASE(1) RSR_KS_CASE(2) RSR_KS_CASE(3) RSR_KS_CASE(4) RSR_KS_CASE(5)
        RSR_KS_CASE(6) RSR_KS_CASE(7) RSR_KS_CASE(8) RSR_KS_CASE(9) RSR_KS_CASE(10)
#undef RSR_KS_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_casc_mfma(hipStream_t st, const rsr_refs* refs, const uint32_t* csrc,
                            int64_t cstride, const unsigned long long* src_count, int64_t max_count,
                            int l0, int l1, int u0, int u1, int chunks, int grid_cap,
                            uint32_t* match) {
    switch (refs->KS4) {
#define RSR_KS_CASE(k) \
    case k: return launch_casc_ks<k>(st, refs, csrc, cstride, src_count, max_count, l0, l1, u0, \
                                     u1, chunks, grid_cap, match);
        RSR_KS_CASE(1) RSR_KS_CASE(2) RSR_KS_CASE(3) RSR_KS_CASE(4) RSR_KS_CASE(5)
        RSR_KS_CASE(6) RSR_KS_CASE(7) RSR_KS_CASE(8) RSR_KS_CASE(9) RSR_KS_CASE(10)
#undef RSR_KS_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rsr
