// Popcount test of samples against a range of reference rows with early
// exit, shared by the LABEL cascade kernels (k_cascade.hip) and the
// persistent cascade (k_cascade_persist.hip).
#pragma once

#include "rsr_internal.h"

namespace rsr {
namespace casc {

// (a & b) | c in one v_bitop3_b32 (truth table indexed by a, b, c from the
// high bit down).  The builtin keeps the test of a row one dependent chain of
// W instructions; written as C the compiler splits it into ANDs and 3-input
// ORs, half as many instructions again.
__device__ __forceinline__ uint32_t and_or(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xEA);
}

// (~a & b) | c in one v_bitop3_b32: the upper-side test needs no complemented
// copy of the samples in registers.
__device__ __forceinline__ uint32_t andnot_or(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xAE);
}

// Rows per side staged in LDS at a time (at most 32 KB for both sides).
template <int W>
constexpr int tile_rows() {
    return 4096 / W > 64 ? 64 : (4096 / W < 8 ? 8 : 4096 / W);
}

// Block-level: tests S samples per lane against rows [l0, l1) (lower) and
// [u0, u1) (upper), interleaved.  The rows pass through LDS in tiles (one
// coalesced cooperative load per tile; the reads are wave-uniform, so every
// LDS access is a broadcast).  A wave stops testing once all its live lanes
// have matched (vote every 8 rows); the block leaves when every wave has.
// Lower rows are stored as NOT t(r), so x <= r iff the OR over the words of
// x & row is 0; upper rows as t(r), so x >= r iff the OR of ~x & row is 0.
// mnL / mnU keep the minimum of those ORs (0: some row matched).  Every
// thread of the block must call it.
template <int W, int S, int BLOCK>
__device__ __forceinline__ void test_rows(const uint32_t (&x)[S][W], const bool (&live)[S],
                                          const uint32_t* __restrict__ low_n, int l0, int l1,
                                          const uint32_t* __restrict__ up_b, int u0, int u1,
                                          uint32_t (&mnL)[S], uint32_t (&mnU)[S], uint32_t* lds) {
    constexpr int T = tile_rows<W>();
    const int nL = l1 - l0, nU = u1 - u0;
    const int n_max = nL > nU ? nL : nU;
    bool any_live = false;
#pragma unroll
    for (int s = 0; s < S; ++s) any_live = any_live || live[s];
    bool wave_done = !__any(any_live);
    const uint32_t* lo_src = low_n + static_cast<int64_t>(l0) * W;
    const uint32_t* up_src = up_b + static_cast<int64_t>(u0) * W;
    for (int t0 = 0; t0 < n_max; t0 += T) {
        __syncthreads();
        const int lo_words = (nL - t0 < T ? (nL - t0 > 0 ? nL - t0 : 0) : T) * W;
        const int up_words = (nU - t0 < T ? (nU - t0 > 0 ? nU - t0 : 0) : T) * W;
        for (int k = threadIdx.x; k < T * W; k += BLOCK) {
            lds[k] = k < lo_words ? lo_src[static_cast<int64_t>(t0) * W + k] : 0u;
            lds[T * W + k] = k < up_words ? up_src[static_cast<int64_t>(t0) * W + k] : 0u;
        }
        __syncthreads();
        if (!wave_done) {
            const int cnt = n_max - t0 < T ? n_max - t0 : T;
            for (int r0 = 0; r0 < cnt; r0 += 8) {
#pragma unroll
                for (int r = r0; r < r0 + 8; ++r) {
                    if (t0 + r < nL) {
                        const uint32_t* row = lds + r * W;
                        uint32_t rw[W];
#pragma unroll
                        for (int w = 0; w < W; ++w) rw[w] = row[w];
#pragma unroll
                        for (int s = 0; s < S; ++s) {
                            uint32_t t = 0;
#pragma unroll
                            for (int w = 0; w < W; ++w) t = and_or(x[s][w], rw[w], t);
                            mnL[s] = min(mnL[s], t);
                        }
                    }
                    if (t0 + r < nU) {
                        const uint32_t* row = lds + T * W + r * W;
                        uint32_t rw[W];
#pragma unroll
                        for (int w = 0; w < W; ++w) rw[w] = row[w];
#pragma unroll
                        for (int s = 0; s < S; ++s) {
                            uint32_t t = 0;
#pragma unroll
                            for (int w = 0; w < W; ++w) t = andnot_or(x[s][w], rw[w], t);
                            mnU[s] = min(mnU[s], t);
                        }
                    }
                }
                bool done = true;
#pragma unroll
                for (int s = 0; s < S; ++s) done = done && (!live[s] || mnL[s] == 0u || mnU[s] == 0u);
                if (__all(done)) {
                    wave_done = true;
                    break;
                }
            }
        }
        if (__syncthreads_and(wave_done ? 1 : 0)) break;
    }
}

}  // namespace casc
}  // namespace rsr
