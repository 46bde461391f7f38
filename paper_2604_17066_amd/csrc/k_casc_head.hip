// Round 0 of the LABEL cascade (k_cascade.hip) in the FP4 matrix-core form on
// 32 x 32 x 64 tiles (dom_fp4x32.h): every sample against the first 32 rows
// of both sides, where most samples find their match (rows are stored by
// increasing size; Algorithm 1 on a consistent set stops at the first match
// on either side).
//
// One tile per side means no early exit is needed, so the round is a stream
// over the samples: each wave keeps both sides' A fragments in registers for
// the whole launch, takes 32 MT samples at a time, flags the decided ones and
// copies the others into its block's region of the compact buffer (the
// block's own span of slots, reserved through an LDS counter: no device-wide
// atomics, which serialise on one address).  k_casc_gather then packs the
// regions into the contiguous buffer the later rounds read.
#include "dom_fp4x32.h"

namespace rsr {
namespace {

using namespace mf;

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxRegions = CascadeBuffers::kMaxRegions;

constexpr int head_tiles(int KS) { return KS <= 5 ? 2 : 1; }

// Block b takes samples [b * span, (b + 1) * span) of seg and appends the
// undecided ones to slots [b * span, ...) of dst; their number goes to
// region_cnt[b].  rl, ru: rows of the first tile of each side (0..32).
template <int KS, int MT>
__global__ __launch_bounds__(kBlock) void k_casc_head(SegSrc seg, int n, int PW, int W,
                                                      const v4i* __restrict__ low32, int rl,
                                                      const v4i* __restrict__ up32, int ru,
                                                      int64_t span, uint32_t* __restrict__ dst,
                                                      int32_t* __restrict__ dst_idx,
                                                      uint32_t* __restrict__ dst_match,
                                                      int64_t dst_stride,
                                                      uint32_t* __restrict__ region_cnt, int last) {
    constexpr int G = 32 * MT;
    __shared__ unsigned s_out;
    // The wave index is uniform (readfirstlane: scalar loop and branches).
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col = lane & 31, half = lane >> 5;
    const uint32_t below = (1u << col) - 1u;
    const int64_t begin = static_cast<int64_t>(blockIdx.x) * span;
    const int64_t end = begin + span < seg.total ? begin + span : seg.total;
    if (threadIdx.x == 0) s_out = 0;
    __syncthreads();
    v4i aL[KS], aU[KS], vm[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
        aL[s] = rl > 0 ? low32[s * 64 + lane] : v4i{};
        aU[s] = ru > 0 ? up32[s * 64 + lane] : v4i{};
        vm[s] = expand_word_fp4(valid_word(2 * s + half, n, PW, W));
    }
    const v16f start = v16f{} - 0.5f;
    // Words of the step at b0, read unconditionally from clamped addresses
    // (a sample past the end reads the block's last sample and is zeroed).
    auto load_step = [&](int64_t b0, uint32_t (&raw)[MT][KS]) {
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            const int64_t g = b0 + 32 * t + col;
            const int64_t gc = g < end ? g : end - 1;
            int job;
            int64_t at, stride;
            seg_locate(seg, gc, job, at);
            const uint32_t* base = seg_words(seg, job, stride);
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                const int w = 2 * s + half;
                const uint32_t v = base[(w < W ? w : W - 1) * stride + at];
                raw[t][s] = (g < end && w < W) ? v : 0u;
            }
        }
    };
    const int64_t step = static_cast<int64_t>(kWaves) * G;
    // Wave-level loop: no block synchronisation until the end.
    for (int64_t b0 = begin + static_cast<int64_t>(wave) * G; b0 < end; b0 += step) {
        uint32_t cur[MT][KS];
        load_step(b0, cur);
        v4i bf[MT][KS];
        bool valid[MT];
        int64_t g[MT];
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            g[t] = b0 + 32 * t + col;
            valid[t] = g[t] < end;
#pragma unroll
            for (int s = 0; s < KS; ++s) bf[t][s] = expand_word_fp4(cur[t][s]);
        }
        bool lowered[MT], raised[MT];
        bool any_left = false;
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            lowered[t] = false;
            raised[t] = false;
        }
        if (rl > 0) {
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                v16f r = start;
#pragma unroll
                for (int s = 0; s < KS; ++s) r = mfma32_step(aL[s], bf[t][s], r);
                const int m = rl >= 32 ? fold32<false>(r, 0) : fold32_last<false>(r, 0, rl, half);
                lowered[t] = min(m, __shfl_xor(m, 32)) < 0;
            }
        }
#pragma unroll
        for (int t = 0; t < MT; ++t) any_left = any_left || (valid[t] && !lowered[t]);
        if (ru > 0 && __any(any_left)) {
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                v16f r = start;
#pragma unroll
                for (int s = 0; s < KS; ++s) r = mfma32_step(aU[s], bf[t][s] ^ vm[s], r);
                const int m = ru >= 32 ? fold32<false>(r, 0) : fold32_last<false>(r, 0, ru, half);
                raised[t] = min(m, __shfl_xor(m, 32)) < 0;
            }
        }
        // Lanes col and col + 32 hold the words 2 s and 2 s + 1 of sample col:
        // both copy theirs; the lower half writes the flag, index and match.
#pragma unroll
        for (int t = 0; t < MT; ++t) {
            const bool hit = lowered[t] || raised[t];
            if (half == 0 && valid[t] && (hit || last)) {
                int job;
                int64_t h;
                seg_locate(seg, g[t], job, h);
                seg_flags(seg, job)[h] = static_cast<uint8_t>(lowered[t] ? 1 : (raised[t] ? 2 : 0));
            }
            if (last) continue;
            const bool carry = valid[t] && !hit;
            const uint32_t mask = static_cast<uint32_t>(__ballot(carry && half == 0));
            if (mask == 0u) continue;
            unsigned base = 0;
            if (lane == 0) base = atomicAdd(&s_out, static_cast<unsigned>(__popc(mask)));
            base = __shfl(base, 0);
            if (carry) {
                const int64_t o = begin + base + __popc(mask & below);
                if (half == 0) {
                    dst_idx[o] = static_cast<int32_t>(g[t]);
                    dst_match[o] = 0u;
                }
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    const int w = 2 * s + half;
                    if (w < W) dst[w * dst_stride + o] = cur[t][s];
                }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) region_cnt[blockIdx.x] = s_out;
}

// Packs the regions written by k_casc_head (region j: region_cnt[j] samples
// from slot j * span of src) into slots [0, total) of dst, in region order,
// and stores total in *dst_count.  Block j moves region j.
__global__ __launch_bounds__(kBlock) void k_casc_gather(
    const uint32_t* __restrict__ region_cnt, int64_t span, int W,
    const uint32_t* __restrict__ src, const int32_t* __restrict__ src_idx, int64_t src_stride,
    uint32_t* __restrict__ dst, int32_t* __restrict__ dst_idx, uint32_t* __restrict__ dst_match,
    int64_t dst_stride, unsigned long long* __restrict__ dst_count) {
    __shared__ unsigned long long s_part[kWaves];
    const int j = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long before = 0;
    for (int i = threadIdx.x; i < j; i += kBlock) before += region_cnt[i];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) before += __shfl_xor(before, d);
    if (lane == 0) s_part[wave] = before;
    __syncthreads();
    unsigned long long pre = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) pre += s_part[k];
    const int64_t cnt = region_cnt[j];
    if (j + 1 == static_cast<int>(gridDim.x) && threadIdx.x == 0) *dst_count = pre + cnt;
    const int64_t from = static_cast<int64_t>(j) * span;
    for (int64_t i = threadIdx.x; i < cnt; i += kBlock) {
        const int64_t o = static_cast<int64_t>(pre) + i;
        dst_idx[o] = src_idx[from + i];
        dst_match[o] = 0u;
        for (int w = 0; w < W; ++w) dst[w * dst_stride + o] = src[w * src_stride + from + i];
    }
}

template <int KS>
hipError_t head_ks(hipStream_t st, const rsr_refs* refs, const SegSrc& seg, int grid, int64_t span,
                   const CascadeBuffers& cb, int last) {
    constexpr int MT = head_tiles(KS);
    const int rl = static_cast<int>(refs->R_L < 32 ? refs->R_L : 32);
    const int ru = static_cast<int>(refs->R_U < 32 ? refs->R_U : 32);
    hipLaunchKernelGGL((k_casc_head<KS, MT>), dim3(static_cast<unsigned>(grid)), dim3(kBlock), 0, st,
                       seg, refs->n, plane_words(refs->n), refs->W,
                       reinterpret_cast<const v4i*>(refs->d_lower_frag32), rl,
                       reinterpret_cast<const v4i*>(refs->d_upper_frag32), ru, span, cb.words[1],
                       cb.index[1], cb.match[1], cb.stride, cb.regions, last);
    return hipGetLastError();
}

}  // namespace

bool casc_head_supported(const rsr_refs* refs) { return refs->KS >= 1 && refs->KS <= kMaxHeadSteps; }

hipError_t launch_casc_head(hipStream_t st, const rsr_refs* refs, const SegSrc& seg,
                            const CascadeBuffers& cb, int last) {
    if (!casc_head_supported(refs) || !cb.regions) return hipErrorInvalidValue;
    const int64_t total = seg.total;
    // Spans of whole wave steps, at most kMaxRegions of them; the regions
    // cover slots [0, total) of buffer 1 exactly.
    const int64_t step = static_cast<int64_t>(kWaves) * 32 * head_tiles(refs->KS);
    const int64_t steps = (total + step - 1) / step;
    const int64_t span = (steps + kMaxRegions - 1) / kMaxRegions * step;
    const int grid = static_cast<int>((total + span - 1) / span);
    hipError_t e;
    switch (refs->KS) {
#define RSR_KS_CASE(k) \
    case k: e = head_ks<k>(st, refs, seg, grid, span, cb, last); break;
        RSR_KS_CASE(1) RSR_KS_CASE(2) RSR_KS_CASE(3) RSR_KS_CASE(4) RSR_KS_CASE(5)
        RSR_KS_CASE(6) RSR_KS_CASE(7) RSR_KS_CASE(8) RSR_KS_CASE(9) RSR_KS_CASE(10)
#undef RSR_KS_CASE
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || last) return e;
    hipLaunchKernelGGL(k_casc_gather, dim3(static_cast<unsigned>(grid)), dim3(kBlock), 0, st,
                       cb.regions, span, refs->W, cb.words[1], cb.index[1], cb.stride, cb.words[0],
                       cb.index[0], cb.match[0], cb.stride,
                       reinterpret_cast<unsigned long long*>(cb.counters));
    return hipGetLastError();
}

}  // namespace rsr
