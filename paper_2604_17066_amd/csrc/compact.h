// Block-level stream compaction shared by the cascade kernels: the carrying
// lanes of a whole block reserve consecutive output slots with one atomic on
// the grid-wide counter (its atomics are the contended part, so there is one
// per block and not one per wave or per sample).
#pragma once

#include "rsr_internal.h"

namespace rsr {

// Every thread of the block (WAVES wavefronts) must call it.  carry[s] says
// whether this lane's s-th sample is kept; slot[s] receives its output
// index.  Slots are ordered by (s, wave, lane).  s_counts holds S * WAVES
// ints of LDS.
template <int WAVES, int S>
__device__ __forceinline__ void block_reserve(const bool (&carry)[S], unsigned long long* counter,
                                              int* s_counts, unsigned long long* s_base,
                                              int64_t (&slot)[S]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t mask[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        mask[s] = __ballot(carry[s]);
        if (lane == 0) s_counts[s * WAVES + wave] = __popcll(mask[s]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int tot = 0;
        for (int k = 0; k < S * WAVES; ++k) {
            const int c = s_counts[k];
            s_counts[k] = tot;
            tot += c;
        }
        *s_base = tot ? atomicAdd(counter, static_cast<unsigned long long>(tot)) : 0ull;
    }
    __syncthreads();
    const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
    for (int s = 0; s < S; ++s)
        slot[s] = static_cast<int64_t>(*s_base) + s_counts[s * WAVES + wave] +
                  __popcll(mask[s] & below);
    __syncthreads();
}

}  // namespace rsr
