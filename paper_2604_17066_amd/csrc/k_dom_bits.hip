// Dominance classification, bit-packed form (section 3.3, Algorithm 1).
//
// A sample x lies below a lower reference state r iff t(x) AND NOT t(r) is
// all zero, and above an upper one iff t(r) AND NOT t(x) is all zero (t = the
// thermometer code of rsr.h).  This is the zero test of the paper's violation
// matrix (eq. violation_matrix) evaluated with one 32-bit AND-OR per word
// instead of a multiply-accumulate per bit.
//
// Mapping: one lane owns S samples and keeps their W words in VGPRs for the
// whole kernel.  Reference rows are identical for every lane of a wave, so
// they stream through the scalar cache into SGPRs, and the inner loop is one
// v_and_or_b32 per (sample, word) with the reference word as the scalar
// operand.  Lower rows are stored pre-complemented (NOT t(r), pad bits 0);
// for the upper pass the kernel complements its sample words once, so both
// passes run the same instruction.
//
// LABEL mode keeps, per sample, the minimum over rows of the OR-accumulated
// violation word (one v_min_u32 per test; zero = some row matched) and leaves
// a pass early once every lane of the wave is decided (wave vote every 32
// rows).  Lower-flagged samples count as decided for the upper pass
// (Algorithm 1's lower precedence).  COUNT mode scans every row and counts the
// zero violation words exactly.
#include "rsr_internal.h"

namespace rsr {
namespace {

constexpr int kBlock = 256;
constexpr int kVoteEvery = 32;

template <int W, int S, bool COUNT>
__global__ __launch_bounds__(kBlock) void k_dom_bits(
    const uint32_t* __restrict__ xs, int64_t N, int w_real, const uint32_t* __restrict__ low_n,
    int64_t RL, const uint32_t* __restrict__ up_b, int64_t RU, uint8_t* __restrict__ flags,
    uint32_t* __restrict__ match) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * (kBlock * S) + threadIdx.x;
    uint32_t x[S][W];
    bool valid[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int64_t h = base + static_cast<int64_t>(s) * kBlock;
        valid[s] = h < N;
#pragma unroll
        for (int w = 0; w < W; ++w)
            x[s][w] = (valid[s] && w < w_real) ? xs[static_cast<int64_t>(w) * N + h] : 0u;
    }

    // ---- lower pass: violation word of (x, r) = OR_w x[w] & NOT t(r)[w] ----
    uint32_t accL[S];
#pragma unroll
    for (int s = 0; s < S; ++s) accL[s] = COUNT ? 0u : 0xFFFFFFFFu;
    for (int64_t r0 = 0; r0 < RL; r0 += kVoteEvery) {
        const int64_t r1 = r0 + kVoteEvery < RL ? r0 + kVoteEvery : RL;
#pragma unroll 2
        for (int64_t r = r0; r < r1; ++r) {
            const uint32_t* row = low_n + r * W;
            uint32_t rw[W];
#pragma unroll
            for (int w = 0; w < W; ++w) rw[w] = row[w];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                uint32_t t = 0;
#pragma unroll
                for (int w = 0; w < W; ++w) t = (x[s][w] & rw[w]) | t;
                if (COUNT)
                    accL[s] += (t == 0u) ? 1u : 0u;
                else
                    accL[s] = min(accL[s], t);
            }
        }
        if (!COUNT) {
            bool done = true;
#pragma unroll
            for (int s = 0; s < S; ++s) done = done && (!valid[s] || accL[s] == 0u);
            if (__all(done)) break;
        }
    }

    // ---- upper pass: violation word = OR_w t(r)[w] & NOT x[w] ----
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
        for (int w = 0; w < W; ++w) x[s][w] = ~x[s][w];
    uint32_t accU[S];
#pragma unroll
    for (int s = 0; s < S; ++s) accU[s] = COUNT ? 0u : 0xFFFFFFFFu;
    bool skip_upper = false;
    if (!COUNT) {
        bool done = true;
#pragma unroll
        for (int s = 0; s < S; ++s) done = done && (!valid[s] || accL[s] == 0u);
        skip_upper = __all(done);
    }
    if (!skip_upper) {
        for (int64_t r0 = 0; r0 < RU; r0 += kVoteEvery) {
            const int64_t r1 = r0 + kVoteEvery < RU ? r0 + kVoteEvery : RU;
#pragma unroll 2
            for (int64_t r = r0; r < r1; ++r) {
                const uint32_t* row = up_b + r * W;
                uint32_t rw[W];
#pragma unroll
                for (int w = 0; w < W; ++w) rw[w] = row[w];
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    uint32_t t = 0;
#pragma unroll
                    for (int w = 0; w < W; ++w) t = (x[s][w] & rw[w]) | t;
                    if (COUNT)
                        accU[s] += (t == 0u) ? 1u : 0u;
                    else
                        accU[s] = min(accU[s], t);
                }
            }
            if (!COUNT) {
                bool done = true;
#pragma unroll
                for (int s = 0; s < S; ++s)
                    done = done && (!valid[s] || accL[s] == 0u || accU[s] == 0u);
                if (__all(done)) break;
            }
        }
    }

#pragma unroll
    for (int s = 0; s < S; ++s) {
        if (!valid[s]) continue;
        const int64_t h = base + static_cast<int64_t>(s) * kBlock;
        uint8_t f;
        if (COUNT) {
            f = static_cast<uint8_t>((accL[s] ? 1 : 0) | (accU[s] ? 2 : 0));
            if (match) {
                match[2 * h] = accL[s];
                match[2 * h + 1] = accU[s];
            }
        } else {
            const bool lo = accL[s] == 0u;
            f = static_cast<uint8_t>(lo ? 1 : (accU[s] == 0u ? 2 : 0));
        }
        flags[h] = f;
    }
}

template <int W, int S>
hipError_t launch_ws(hipStream_t st, const rsr_refs* refs, const uint32_t* xs, int64_t N,
                     int mode, uint8_t* flags, uint32_t* match) {
    const int64_t per_block = static_cast<int64_t>(kBlock) * S;
    const dim3 grid(static_cast<unsigned>((N + per_block - 1) / per_block));
    if (mode == RSR_COUNT)
        hipLaunchKernelGGL((k_dom_bits<W, S, true>), grid, dim3(kBlock), 0, st, xs, N, refs->W,
                           refs->d_lower_nbits, refs->R_L, refs->d_upper_bits, refs->R_U, flags,
                           match);
    else
        hipLaunchKernelGGL((k_dom_bits<W, S, false>), grid, dim3(kBlock), 0, st, xs, N,
                           refs->W, refs->d_lower_nbits, refs->R_L, refs->d_upper_bits,
                           refs->R_U, flags, match);
    return hipGetLastError();
}

// Samples per lane: as many as keep >= 4 waves per SIMD on a 256-CU part
// (4096 waves) and at most 64 sample words in registers.
template <int W>
hipError_t launch_w(hipStream_t st, const rsr_refs* refs, const uint32_t* xs, int64_t N,
                    int mode, uint8_t* flags, uint32_t* match) {
    const int64_t waves1 = (N + 63) / 64;
    if (W * 4 <= 64 && waves1 / 4 >= 4096)
        return launch_ws<W, (W * 4 <= 64 ? 4 : 1)>(st, refs, xs, N, mode, flags, match);
    if (W * 2 <= 64 && waves1 / 2 >= 4096)
        return launch_ws<W, (W * 2 <= 64 ? 2 : 1)>(st, refs, xs, N, mode, flags, match);
    return launch_ws<W, 1>(st, refs, xs, N, mode, flags, match);
}

}  // namespace

// Instantiated word counts; a reference set with W words uses the smallest
// instantiation >= W and pads its rows with zero words.
static const int kInstW[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32, 40, 48, 64, 96, 128};

int dom_row_words(int W) {
    for (int w : kInstW)
        if (w >= W) return w;
    return -1;
}

hipError_t launch_dom_bits(hipStream_t st, const rsr_refs* refs, const uint32_t* xs, int64_t N,
                           int mode, uint8_t* flags, uint32_t* match) {
    switch (refs->WR) {
#define RSR_W_CASE(w) \
    case w: return launch_w<w>(st, refs, xs, N, mode, flags, match);
        RSR_W_CASE(1) RSR_W_CASE(2) RSR_W_CASE(3) RSR_W_CASE(4) RSR_W_CASE(5) RSR_W_CASE(6)
        RSR_W_CASE(8) RSR_W_CASE(10) RSR_W_CASE(12) RSR_W_CASE(16) RSR_W_CASE(20)
        RSR_W_CASE(24) RSR_W_CASE(32) RSR_W_CASE(40) RSR_W_CASE(48) RSR_W_CASE(64)
        RSR_W_CASE(96) RSR_W_CASE(128)
#undef RSR_W_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rsr
