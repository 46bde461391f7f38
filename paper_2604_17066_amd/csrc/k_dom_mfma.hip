// Dominance classification, matrix-core form: the violation matrix of the
// paper (section 3.3.2, eq. violation_matrix) as an int8 contraction on the
// gfx950 MFMA units, with int32 accumulation.
//
// Operands are the thermometer bits of rsr.h as 0/1 bytes, k = packed bit
// index.  For a lower row r the contraction is V = sum_k t(x)_k * NOT t(r)_k,
// zero iff x <= r.  For an upper row it is sum_k t(x)_k * t(r)_k, which equals
// |t(r)| iff x >= r; the accumulator starts at -|t(r)| so that both sides are a
// zero test.  Pad rows (R rounded up to 16) start at +1 and never match.
//
// One v_mfma_i32_16x16x64_i8 multiplies a 16 x 64 tile of reference rows (A)
// by a 64 x 16 tile of samples (B).  Lane l supplies row / column l % 16 and
// the 16 bytes of k-chunk l / 16 of each operand; the result lane l holds rows
// 4 (l / 16) .. +3 of column l % 16.  A wave keeps the B fragments of MT
// sample tiles (16 MT samples) in VGPRs for the whole kernel (expanded once
// from the packed bits); the eight waves of a block share reference tiles,
// which are staged through LDS with double buffering.  Reference rows are
// stored on the device in fragment order ([tile][k-step][lane][16 bytes]), so a
// tile is one contiguous block and every LDS read is one 16-byte access.
//
// LABEL mode keeps, per sample, the unsigned minimum of its accumulators (0 =
// some row matched), and the block leaves a pass early when every sample is
// decided (vote every 4 tiles; lower-flagged samples are decided for the upper
// pass).  COUNT mode counts the non-zero accumulators (sum of min(acc, 1)) and
// returns rows - non-zeros, the exact number of matching rows.
#include "rsr_internal.h"

namespace rsr {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kBlock = 512;
constexpr int kWaves = kBlock / 64;
constexpr int kVoteTiles = 4;

__device__ __forceinline__ int expand4(uint32_t v) {
    // Bits b0..b3 of v (v < 16) -> bytes b0, b1, b2, b3.
    return static_cast<int>((v * 0x00204081u) & 0x01010101u);
}

__device__ __forceinline__ uint32_t umin4(v4i a) {
    const uint32_t x = static_cast<uint32_t>(a.x), y = static_cast<uint32_t>(a.y);
    const uint32_t z = static_cast<uint32_t>(a.z), w = static_cast<uint32_t>(a.w);
    return min(min(x, y), min(z, w));
}

// Number of non-zero accumulators among four (min(v, 1) is 0 or 1 as unsigned).
__device__ __forceinline__ uint32_t nonzeros4(v4i a) {
    return min(static_cast<uint32_t>(a.x), 1u) + min(static_cast<uint32_t>(a.y), 1u) +
           min(static_cast<uint32_t>(a.z), 1u) + min(static_cast<uint32_t>(a.w), 1u);
}

// One pass over the tiles of one side.  acc_out[t] = running min (LABEL) or
// number of non-zero accumulators (COUNT) for this lane's column of sample
// tile t.  An LDS tile holds the KS*64 operand fragments followed by the 16
// accumulator starts, so the loop has no global load on its critical path.
template <int KS, int MT, bool COUNT>
__device__ __forceinline__ void mfma_pass(const v4i (&bf)[MT][KS], const v4i* __restrict__ frag,
                                          const v4i* __restrict__ cinit, int tiles,
                                          v4i* __restrict__ lds, uint32_t (&acc_out)[MT],
                                          const bool (&pre_done)[MT], const bool (&valid)[MT],
                                          int* vote) {
    constexpr int kFragV4 = KS * 64;      // operand v4i per reference tile
    constexpr int kTileV4 = kFragV4 + 4;  // plus 16 accumulator starts
    constexpr int kPerThread = (kTileV4 + kBlock - 1) / kBlock;
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 4;
    if (tiles <= 0) return;

    v4i stage[kPerThread];
    auto fetch = [&](int T) {
#pragma unroll
        for (int q = 0; q < kPerThread; ++q) {
            const int idx = q * kBlock + threadIdx.x;
            if (idx < kFragV4)
                stage[q] = frag[static_cast<int64_t>(T) * kFragV4 + idx];
            else if (idx < kTileV4)
                stage[q] = cinit[static_cast<int64_t>(T) * 4 + (idx - kFragV4)];
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < kPerThread; ++q) {
            const int idx = q * kBlock + threadIdx.x;
            if (idx < kTileV4) lds[buf * kTileV4 + idx] = stage[q];
        }
    };

    fetch(0);
    store(0);
    __syncthreads();
    for (int T = 0; T < tiles; ++T) {
        const int cur = T & 1;
        if (T + 1 < tiles) fetch(T + 1);
        const v4i c0 = lds[cur * kTileV4 + kFragV4 + grp];
        v4i a[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) a[s] = lds[cur * kTileV4 + s * 64 + lane];
        v4i acc[MT];
#pragma unroll
        for (int t = 0; t < MT; ++t) acc[t] = c0;
#pragma unroll
        for (int s = 0; s < KS; ++s)
#pragma unroll
            for (int t = 0; t < MT; ++t)
                acc[t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[s], bf[t][s], acc[t], 0, 0, 0);
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            if (COUNT)
                acc_out[t] += nonzeros4(acc[t]);
            else
                acc_out[t] = min(acc_out[t], umin4(acc[t]));
        }
        if (T + 1 < tiles) store(cur ^ 1);
        bool leave = false;
        if (!COUNT && (T % kVoteTiles) == kVoteTiles - 1) {
            bool done = true;
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                uint32_t m = acc_out[t];
                m = min(m, static_cast<uint32_t>(__shfl_xor(static_cast<int>(m), 16)));
                m = min(m, static_cast<uint32_t>(__shfl_xor(static_cast<int>(m), 32)));
                done = done && (!valid[t] || pre_done[t] || m == 0u);
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
}

template <int KS, int MT, bool COUNT>
__global__ __launch_bounds__(kBlock) void k_dom_mfma(
    const uint32_t* __restrict__ xs, int64_t N, int W, const v4i* __restrict__ low_frag,
    const v4i* __restrict__ low_c, int TL, const v4i* __restrict__ up_frag,
    const v4i* __restrict__ up_c, int TU, uint8_t* __restrict__ flags,
    uint32_t* __restrict__ match) {
    __shared__ v4i lds[2 * (KS * 64 + 4)];
    __shared__ int vote[kWaves];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int64_t wbase = (static_cast<int64_t>(blockIdx.x) * kWaves + wave) * (16 * MT);

    // Sample operand: bytes 16*grp .. +15 of k-step s are packed bits
    // 64 s + 16 grp .. +15, i.e. half (grp & 1) of word 2 s + (grp >> 1).
    v4i bf[MT][KS];
    bool valid[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        const int64_t h = wbase + 16 * t + col;
        valid[t] = h < N;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int w = 2 * s + (grp >> 1);
            uint32_t bits = (valid[t] && w < W) ? xs[static_cast<int64_t>(w) * N + h] : 0u;
            bits = (bits >> (16 * (grp & 1))) & 0xFFFFu;
            v4i f;
            f.x = expand4(bits & 0xFu);
            f.y = expand4((bits >> 4) & 0xFu);
            f.z = expand4((bits >> 8) & 0xFu);
            f.w = expand4(bits >> 12);
            bf[t][s] = f;
        }
    }

    uint32_t accL[MT], accU[MT];
    bool none[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        accL[t] = COUNT ? 0u : 0xFFFFFFFFu;
        accU[t] = COUNT ? 0u : 0xFFFFFFFFu;
        none[t] = false;
    }
    mfma_pass<KS, MT, COUNT>(bf, low_frag, low_c, TL, lds, accL, none, valid, vote);

    // Per-sample lower result across the four lane groups (COUNT: every one of
    // the 16 TL rows is either a zero or a non-zero accumulator).
    bool lowered[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
        uint32_t m = accL[t];
        if (COUNT) {
            m += static_cast<uint32_t>(__shfl_xor(static_cast<int>(m), 16));
            m += static_cast<uint32_t>(__shfl_xor(static_cast<int>(m), 32));
            m = 16u * static_cast<uint32_t>(TL) - m;
        } else {
            m = min(m, static_cast<uint32_t>(__shfl_xor(static_cast<int>(m), 16)));
            m = min(m, static_cast<uint32_t>(__shfl_xor(static_cast<int>(m), 32)));
        }
        accL[t] = m;
        lowered[t] = COUNT ? false : (m == 0u);
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
    if (!skip_upper) mfma_pass<KS, MT, COUNT>(bf, up_frag, up_c, TU, lds, accU, lowered, valid, vote);

#pragma unroll
    for (int t = 0; t < MT; ++t) {
        uint32_t m = accU[t];
        if (COUNT) {
            m += static_cast<uint32_t>(__shfl_xor(static_cast<int>(m), 16));
            m += static_cast<uint32_t>(__shfl_xor(static_cast<int>(m), 32));
            m = 16u * static_cast<uint32_t>(TU) - m;
        } else {
            m = min(m, static_cast<uint32_t>(__shfl_xor(static_cast<int>(m), 16)));
            m = min(m, static_cast<uint32_t>(__shfl_xor(static_cast<int>(m), 32)));
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
                    match[2 * h] = accL[t];
                    match[2 * h + 1] = accU[t];
                }
            } else {
                f = static_cast<uint8_t>(lowered[t] ? 1 : (accU[t] == 0u ? 2 : 0));
            }
            flags[h] = f;
        }
    }
}

template <int KS>
hipError_t launch_ks(hipStream_t st, const rsr_refs* refs, const uint32_t* xs, int64_t N,
                     int mode, uint8_t* flags, uint32_t* match) {
    // B fragments take MT * KS * 4 VGPRs; at most 120 keeps two waves per SIMD.
    constexpr int MT = KS >= 30 ? 1 : (30 / KS > 8 ? 8 : 30 / KS);
    const int64_t per_block = static_cast<int64_t>(kWaves) * 16 * MT;
    const dim3 grid(static_cast<unsigned>((N + per_block - 1) / per_block));
    const v4i* lf = reinterpret_cast<const v4i*>(refs->d_lower_frag);
    const v4i* lc = reinterpret_cast<const v4i*>(refs->d_lower_cinit);
    const v4i* uf = reinterpret_cast<const v4i*>(refs->d_upper_frag);
    const v4i* uc = reinterpret_cast<const v4i*>(refs->d_upper_cinit);
    if (mode == RSR_COUNT)
        hipLaunchKernelGGL((k_dom_mfma<KS, MT, true>), grid, dim3(kBlock), 0, st, xs, N, refs->W,
                           lf, lc, refs->TL, uf, uc, refs->TU, flags, match);
    else
        hipLaunchKernelGGL((k_dom_mfma<KS, MT, false>), grid, dim3(kBlock), 0, st, xs, N, refs->W,
                           lf, lc, refs->TL, uf, uc, refs->TU, flags, match);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dom_mfma(hipStream_t st, const rsr_refs* refs, const uint32_t* xs, int64_t N,
                           int mode, uint8_t* flags, uint32_t* match) {
    switch (refs->KS) {
#define RSR_KS_CASE(k) \
    case k: return launch_ks<k>(st, refs, xs, N, mode, flags, match);
        RSR_KS_CASE(1) RSR_KS_CASE(2) RSR_KS_CASE(3) RSR_KS_CASE(4) RSR_KS_CASE(5)
        RSR_KS_CASE(6) RSR_KS_CASE(7) RSR_KS_CASE(8) RSR_KS_CASE(9) RSR_KS_CASE(10)
        RSR_KS_CASE(11) RSR_KS_CASE(12) RSR_KS_CASE(13) RSR_KS_CASE(14) RSR_KS_CASE(15)
        RSR_KS_CASE(16) RSR_KS_CASE(17) RSR_KS_CASE(18) RSR_KS_CASE(19) RSR_KS_CASE(20)
#undef RSR_KS_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rsr
