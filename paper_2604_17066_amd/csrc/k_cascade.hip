// LABEL-mode classification on a consistent reference set (no upper row lies
// below a lower row; section 2.2 valid reference sets always are): no sample
// can be dominated on both sides, so the first match on either side decides
// the label of Algorithm 1 and a sample can stop there.
//
// Rows are stored by increasing size, so most samples match among the first
// few rows.  The classification runs in rounds over row ranges
// [0, first), [first, first*growth), ... of both sides at once:
//
//   round 0 (k_casc_fused, all samples, read where they are): each lane tests
//     S samples against the round's rows of both sides, interleaved, and the
//     wave leaves the round as soon as all its lanes have matched (vote every 8
//     rows).  Matched samples get their flag; the others are copied (packed
//     words and global index) to a compact buffer.  With shape.mfma_head the
//     round is one 32-row tile per side in the FP4 matrix-core form instead
//     (k_casc_head.hip), which streams the samples at close to memory speed.
//   later rounds: the undecided samples are few, so the round's rows are split
//     into `chunks` contiguous ranges taken by different waves (k_casc_test,
//     grid y = chunk) to keep the GPU busy; a chunk that finds a match ORs it
//     into the sample's match word, and k_casc_resolve then writes flags and
//     compacts the still undecided samples.  A round whose rows do not warrant
//     a split runs k_casc_fused on the compact buffer instead.  With
//     shape.mfma_tail every round after round 0 runs in the FP4 matrix-core
//     form (k_dom_mfma.hip), which makes more tests per second once the
//     undecided samples have to be tested against many rows: an unsplit
//     round is one k_casc_mfma_round (test, flags and compaction), a split
//     round k_casc_mfma per chunk and then k_casc_resolve.
//   the last round flags every remaining sample as unclassified.
//
// Compaction reserves output slots with one atomic per block for all of the
// block's samples (wave ballots, an LDS prefix over the block's waves;
// compact.h): the grid-wide counter's atomics are the contended part.
#include "casc_popcount.h"
#include "compact.h"

namespace rsr {
namespace {

using namespace casc;

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
// Most chunks of a split round: 64 in the FP4 form (more slow the 1250-edge
// graph's rounds of 3e4-6e4 rows: 2.47 against 2.19 ms per classify), 128 in
// the popcount form (its rounds gain from the parallelism: three-state level
// 1 0.36 against 0.44 ms).
constexpr int kMaxChunks = 64;
constexpr int kMaxPopcountChunks = 128;
// Round 0 (every sample) in blocks of 512: half the slot reservations of
// 256-thread blocks on the one output counter (graph2: 0.150 against 0.153 ms
// per LABEL classify; the later rounds keep 256, where 512 is slower).
constexpr int kRound0Block = 512;

template <int W, int S, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_casc_fused(
    SegSrc seg, const uint32_t* __restrict__ csrc, int64_t cstride,
    const int32_t* __restrict__ src_idx, const unsigned long long* __restrict__ src_count,
    int w_real, const uint32_t* __restrict__ low_n, int l0, int l1,
    const uint32_t* __restrict__ up_b, int u0, int u1, uint32_t* __restrict__ dst,
    int32_t* __restrict__ dst_idx, uint32_t* __restrict__ dst_match, int64_t dst_stride,
    unsigned long long* __restrict__ dst_count, int last) {
    constexpr int kW = BLOCK / 64;
    __shared__ int s_counts[S * kW];
    __shared__ unsigned long long s_base;
    __shared__ uint32_t s_rows[2 * tile_rows<W>() * W];
    const int64_t total = src_idx ? static_cast<int64_t>(*src_count) : seg.total;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // Block-uniform loop (test_rows and block_reserve synchronise the block).
    for (int64_t b0 = static_cast<int64_t>(blockIdx.x) * BLOCK * S; b0 < total;
         b0 += static_cast<int64_t>(gridDim.x) * BLOCK * S) {
        const int64_t j0 = b0 + static_cast<int64_t>(wave) * 64 * S;
        uint32_t x[S][W];
        bool valid[S];
        int64_t jj[S], gg[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            jj[s] = j0 + s * 64 + lane;
            valid[s] = jj[s] < total;
            gg[s] = valid[s] ? (src_idx ? static_cast<int64_t>(src_idx[jj[s]]) : jj[s]) : 0;
            const uint32_t* base = csrc;
            int64_t stride = cstride, at = jj[s];
            if (!src_idx && valid[s]) {
                int job;
                seg_locate(seg, gg[s], job, at);
                base = seg_words(seg, job, stride);
            }
#pragma unroll
            for (int w = 0; w < W; ++w) {
                x[s][w] = (valid[s] && w < w_real) ? base[w * stride + at] : 0u;
            }
        }
        uint32_t mnL[S], mnU[S];
#pragma unroll
        for (int s = 0; s < S; ++s) mnL[s] = mnU[s] = 0xFFFFFFFFu;
        test_rows<W, S, BLOCK>(x, valid, low_n, l0, l1, up_b, u0, u1, mnL, mnU, s_rows);
        bool carry[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bool hit = mnL[s] == 0u || mnU[s] == 0u;
            if (valid[s] && (hit || last)) {
                int job;
                int64_t h;
                seg_locate(seg, gg[s], job, h);
                seg_flags(seg, job)[h] =
                    static_cast<uint8_t>(mnL[s] == 0u ? 1 : (mnU[s] == 0u ? 2 : 0));
            }
            carry[s] = valid[s] && !hit;
        }
        if (last) continue;
        int64_t d[S];
        block_reserve<kW, S>(carry, dst_count, s_counts, &s_base, d);
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (carry[s]) {
                dst_idx[d[s]] = static_cast<int32_t>(gg[s]);
                dst_match[d[s]] = 0u;
#pragma unroll
                for (int w = 0; w < W; ++w)
                    if (w < w_real) dst[w * dst_stride + d[s]] = x[s][w];
            }
        }
    }
}

// One chunk of a split round: rows of chunk blockIdx.y for the compacted
// samples; matches are ORed into match[d] (bit0 lower, bit1 upper).
template <int W>
__global__ __launch_bounds__(kBlock) void k_casc_test(
    const uint32_t* __restrict__ csrc, int64_t cstride, const unsigned long long* __restrict__ src_count,
    int w_real, const uint32_t* __restrict__ low_n, int l0, int l1,
    const uint32_t* __restrict__ up_b, int u0, int u1, uint32_t* __restrict__ match) {
    const int64_t total = static_cast<int64_t>(*src_count);
    const int chunks = gridDim.y, c = blockIdx.y;
    const int nL = l1 - l0, nU = u1 - u0;
    const int cl0 = l0 + static_cast<int>((static_cast<int64_t>(nL) * c) / chunks);
    const int cl1 = l0 + static_cast<int>((static_cast<int64_t>(nL) * (c + 1)) / chunks);
    const int cu0 = u0 + static_cast<int>((static_cast<int64_t>(nU) * c) / chunks);
    const int cu1 = u0 + static_cast<int>((static_cast<int64_t>(nU) * (c + 1)) / chunks);
    __shared__ uint32_t s_rows[2 * tile_rows<W>() * W];
    // Block-uniform loop (test_rows synchronises the block).
    for (int64_t b0 = static_cast<int64_t>(blockIdx.x) * kBlock; b0 < total;
         b0 += static_cast<int64_t>(gridDim.x) * kBlock) {
        const int64_t d = b0 + threadIdx.x;
        bool live[1];
        live[0] = d < total && match[d] == 0u;
        uint32_t x[1][W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            x[0][w] = (live[0] && w < w_real) ? csrc[w * cstride + d] : 0u;
        }
        uint32_t mnL[1] = {0xFFFFFFFFu}, mnU[1] = {0xFFFFFFFFu};
        test_rows<W, 1, kBlock>(x, live, low_n, cl0, cl1, up_b, cu0, cu1, mnL, mnU, s_rows);
        const uint32_t bits = (mnL[0] == 0u ? 1u : 0u) | (mnU[0] == 0u ? 2u : 0u);
        if (live[0] && bits) atomicOr(&match[d], bits);
    }
}

// Flags the samples a split round decided and compacts the others.
__global__ __launch_bounds__(kBlock) void k_casc_resolve(
    SegSrc seg, const uint32_t* __restrict__ csrc, int64_t cstride,
    const int32_t* __restrict__ src_idx, const unsigned long long* __restrict__ src_count,
    int w_real, const uint32_t* __restrict__ match, uint32_t* __restrict__ dst,
    int32_t* __restrict__ dst_idx, uint32_t* __restrict__ dst_match, int64_t dst_stride,
    unsigned long long* __restrict__ dst_count, int last) {
    __shared__ int s_counts[kWaves];
    __shared__ unsigned long long s_base;
    const int64_t total = static_cast<int64_t>(*src_count);
    for (int64_t b0 = static_cast<int64_t>(blockIdx.x) * kBlock; b0 < total;
         b0 += static_cast<int64_t>(gridDim.x) * kBlock) {
        const int64_t d = b0 + threadIdx.x;
        const bool valid = d < total;
        const uint32_t bits = valid ? match[d] : 0u;
        const int64_t g = valid ? static_cast<int64_t>(src_idx[d]) : 0;
        if (valid && (bits || last)) {
            int job;
            int64_t h;
            seg_locate(seg, g, job, h);
            seg_flags(seg, job)[h] = static_cast<uint8_t>((bits & 1u) ? 1 : ((bits & 2u) ? 2 : 0));
        }
        if (last) continue;
        const bool carry[1] = {valid && bits == 0u};
        int64_t slot[1];
        block_reserve<kWaves, 1>(carry, dst_count, s_counts, &s_base, slot);
        const int64_t o = slot[0];
        if (carry[0]) {
            dst_idx[o] = static_cast<int32_t>(g);
            dst_match[o] = 0u;
            for (int w = 0; w < w_real; ++w) dst[w * dst_stride + o] = csrc[w * cstride + d];
        }
    }
}

template <int W>
hipError_t cascade_w(hipStream_t st, const rsr_refs* refs, const SegSrc& seg,
                     const CascadeBuffers& cb, const CascadeShape& shape, int grid_cap) {
    constexpr int S0 = W <= 12 ? 4 : (W <= 24 ? 2 : 1);
    const int64_t N = seg.total;
    auto blocks_for = [&](int64_t per_block, int64_t cap) {
        int64_t b = (N + per_block - 1) / per_block;
        if (b > cap) b = cap;
        return b < 1 ? int64_t{1} : b;
    };
    const int n_max = static_cast<int>(refs->R_L > refs->R_U ? refs->R_L : refs->R_U);
    int64_t lo = 0, hi = shape.first;
    const uint32_t* csrc = nullptr;
    const int32_t* src_idx = nullptr;
    const uint32_t* src_match = nullptr;
    const unsigned long long* src_count = nullptr;
    for (int round = 0;; ++round) {
        const bool last = hi >= n_max || round + 1 >= CascadeBuffers::kMaxRounds;
        if (last) hi = n_max;
        const int l0 = static_cast<int>(lo < refs->R_L ? lo : refs->R_L);
        const int l1 = static_cast<int>(hi < refs->R_L ? hi : refs->R_L);
        const int u0 = static_cast<int>(lo < refs->R_U ? lo : refs->R_U);
        const int u1 = static_cast<int>(hi < refs->R_U ? hi : refs->R_U);
        const int rows = (l1 - l0) > (u1 - u0) ? (l1 - l0) : (u1 - u0);
        int chunks = round == 0 ? 1 : rows / (shape.split_rows > 0 ? shape.split_rows : 1 << 30);
        const int max_chunks = shape.max_chunks > 0 ? shape.max_chunks
                               : shape.mfma_tail && refs->KS4 > 0 ? kMaxChunks
                                                                  : kMaxPopcountChunks;
        if (chunks > max_chunks) chunks = max_chunks;
        if (chunks < 1) chunks = 1;
        uint32_t* dst = cb.words[round & 1];
        int32_t* dst_idx = cb.index[round & 1];
        uint32_t* dst_match = cb.match[round & 1];
        unsigned long long* dst_count = reinterpret_cast<unsigned long long*>(cb.counters) + round;
        hipError_t e;
        // With the matrix-core tail, an unsplit round after round 0 runs whole
        // in the FP4 form (test, flags and compaction in one kernel).  Round 0
        // runs in the FP4 32 x 32 form with shape.mfma_head (one tile per
        // side, no early exit needed), else on the vector ALU with a per-wave
        // early exit.
        const bool mfma_round = shape.mfma_tail && refs->KS4 > 0 && round > 0;
        if (round == 0 && shape.mfma_head && shape.first == 32 && casc_head_supported(refs)) {
            e = launch_casc_head(st, refs, seg, cb, last ? 1 : 0);
        } else if (chunks == 1 && mfma_round) {
            e = launch_casc_mfma_round(st, refs, seg, csrc, cb.stride, src_idx, src_count, N, N,
                                       l0, l1, u0, u1, grid_cap, dst, dst_idx, dst_match,
                                       cb.stride, dst_count, last ? 1 : 0);
        } else if (chunks == 1) {
            if (round == 0)
                hipLaunchKernelGGL((k_casc_fused<W, S0, kRound0Block>), dim3(static_cast<unsigned>(
                                       blocks_for(static_cast<int64_t>(kRound0Block) * S0, grid_cap))),
                                   dim3(kRound0Block), 0, st, seg, csrc, cb.stride, src_idx, src_count,
                                   refs->W, refs->d_lower_nbits, l0, l1, refs->d_upper_bits, u0,
                                   u1, dst, dst_idx, dst_match, cb.stride, dst_count, last ? 1 : 0);
            else
                hipLaunchKernelGGL((k_casc_fused<W, 1, kBlock>), dim3(static_cast<unsigned>(
                                       blocks_for(kBlock, grid_cap))),
                                   dim3(kBlock), 0, st, seg, csrc, cb.stride, src_idx, src_count,
                                   refs->W, refs->d_lower_nbits, l0, l1, refs->d_upper_bits, u0,
                                   u1, dst, dst_idx, dst_match, cb.stride, dst_count, last ? 1 : 0);
            e = hipGetLastError();
        } else {
            if (shape.mfma_tail && refs->KS4 > 0) {
                e = launch_casc_mfma(st, refs, csrc, cb.stride, src_count, N, l0, l1, u0, u1, chunks,
                                     grid_cap, const_cast<uint32_t*>(src_match));
            } else {
                const int64_t bx = blocks_for(kBlock, grid_cap / chunks > 0 ? grid_cap / chunks : 1);
                hipLaunchKernelGGL((k_casc_test<W>), dim3(static_cast<unsigned>(bx), chunks),
                                   dim3(kBlock), 0, st, csrc, cb.stride, src_count, refs->W,
                                   refs->d_lower_nbits, l0, l1, refs->d_upper_bits, u0, u1,
                                   const_cast<uint32_t*>(src_match));
                e = hipGetLastError();
            }
            if (e == hipSuccess) {
                hipLaunchKernelGGL(k_casc_resolve, dim3(static_cast<unsigned>(blocks_for(kBlock, grid_cap))),
                                   dim3(kBlock), 0, st, seg, csrc, cb.stride, src_idx, src_count,
                                   refs->W, src_match, dst, dst_idx, dst_match, cb.stride, dst_count,
                                   last ? 1 : 0);
                e = hipGetLastError();
            }
        }
        if (e != hipSuccess || last) return e;
        csrc = dst;
        src_idx = dst_idx;
        src_match = dst_match;
        src_count = dst_count;
        lo = hi;
        hi *= shape.growth;
    }
}

}  // namespace

hipError_t launch_dom_cascade(hipStream_t st, const rsr_refs* refs, const SegSrc& seg,
                              const CascadeBuffers& cb, const CascadeShape& shape, int grid_cap) {
    if (shape.first < 1 || shape.growth < 2) return hipErrorInvalidValue;
    switch (refs->WR) {
#define RSR_W_CASE(w) \
    case w: return cascade_w<w>(st, refs, seg, cb, shape, grid_cap);
        RSR_W_CASE(1) RSR_W_CASE(2) RSR_W_CASE(3) RSR_W_CASE(4) RSR_W_CASE(5) RSR_W_CASE(6)
        RSR_W_CASE(8) RSR_W_CASE(10) RSR_W_CASE(12) RSR_W_CASE(16) RSR_W_CASE(20)
        RSR_W_CASE(24) RSR_W_CASE(32) RSR_W_CASE(40) RSR_W_CASE(48) RSR_W_CASE(64)
        RSR_W_CASE(96) RSR_W_CASE(128)
#undef RSR_W_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rsr
