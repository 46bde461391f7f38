// Monte Carlo sampler: 32-bit uniform words compared against integer
// inverse-CDF thresholds, written straight into the packed thermometer layout
// (word-major [W][N]; see rsr.h).
//
// The word of component i is two 16-bit halves at position i mod 8 of two
// Philox4x32-10 blocks (counter word 0 = i div 8, and the same with bit 31
// set).  Its high half decides u >= C unless it equals the high half of C,
// which happens with probability 2^-16 per threshold: only then is the second
// block drawn.  So one Philox block serves eight components, and the result
// is exactly that of comparing the full 32-bit word.
//
// One thread draws one sample; the finished words are stored with coalesced
// 32-bit stores (lanes hold consecutive samples).  The thresholds are
// identical for every thread, so they are read through the scalar cache.
#include "rsr_internal.h"

namespace rsr {
namespace {

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11, section 3.2).
struct Philox4 {
    uint32_t v0, v1, v2, v3;
};

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                 uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t a = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t b = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        // Three-input XORs as one v_bitop3_b32 each (truth table 0x96).
        const uint32_t y0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(b >> 32), c1, k0, 0x96);
        const uint32_t y2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(a >> 32), c3, k1, 0x96);
        c1 = static_cast<uint32_t>(b);
        c3 = static_cast<uint32_t>(a);
        c0 = y0;
        c2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// Half k (0..7) of a block: half (k mod 2) of word (k div 2), low half first.
__device__ __forceinline__ uint32_t half16(const Philox4& b, int k) {
    const uint32_t w = (k >> 1) == 0 ? b.v0 : (k >> 1) == 1 ? b.v1 : (k >> 1) == 2 ? b.v2 : b.v3;
    return (k & 1) ? (w >> 16) : (w & 0xFFFFu);
}

// Draws sample index g (its Philox counter) and stores it as column h of the
// word-major [W][N] array out.  KM1 = K - 1 thermometer planes; thresh and
// half are the model's two forms of the thresholds (rsr_model).
template <int KM1>
__device__ __forceinline__ void draw_sample(const uint64_t* __restrict__ thresh,
                                            const int32_t* __restrict__ half, int n, int PW,
                                            uint32_t key0, uint32_t key1, uint32_t stream_id,
                                            uint64_t g, int64_t h, int64_t N,
                                            uint32_t* __restrict__ out) {
    const uint32_t glo = static_cast<uint32_t>(g), ghi = static_cast<uint32_t>(g >> 32);
    for (int wi = 0; wi < PW; ++wi) {
        uint32_t acc[KM1];
#pragma unroll
        for (int s = 0; s < KM1; ++s) acc[s] = 0;
        const int base = wi * 32;
        const int groups = min(4, (n - base + 7) >> 3);
        // Unrolled over the word's four groups, so every bit position below
        // is a constant.
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q >= groups) break;
            const int i0 = base + q * 8;
            const Philox4 hi = philox4x32_10(static_cast<uint32_t>(i0 >> 3), glo, ghi, stream_id,
                                             key0, key1);
            const int32_t* hq = half + static_cast<int64_t>(i0) * KM1 * 2;
            uint32_t tie = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int32_t u = static_cast<int32_t>(half16(hi, k));
                int32_t th[2 * KM1];
#pragma unroll
                for (int t = 0; t < 2 * KM1; ++t) th[t] = hq[k * KM1 * 2 + t];
#pragma unroll
                for (int s = 0; s < KM1; ++s) {
                    acc[s] |= (u > th[2 * s] ? 1u : 0u) << ((q * 8 + k) & 31);
                    tie |= u == th[2 * s + 1] ? 1u : 0u;
                }
            }
            if (tie) {
                // Some threshold shares this lane's high half: its low half,
                // from the second block, decides.
                const Philox4 lo = philox4x32_10(static_cast<uint32_t>(i0 >> 3) | 0x80000000u,
                                                 glo, ghi, stream_id, key0, key1);
                for (int k = 0; k < 8; ++k) {
                    const int32_t u = static_cast<int32_t>(half16(hi, k));
                    for (int s = 0; s < KM1; ++s) {
                        if (u == hq[(k * KM1 + s) * 2 + 1] &&
                            half16(lo, k) >= (thresh[(i0 + k) * KM1 + s] & 0xFFFFu))
                            acc[s] |= 1u << ((q * 8 + k) & 31);
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < KM1; ++s)
            out[static_cast<int64_t>(s * PW + wi) * N + h] = acc[s];
    }
}

template <int KM1>
__global__ __launch_bounds__(256) void k_sample(const uint64_t* __restrict__ thresh,
                                                const int32_t* __restrict__ half, int n,
                                                int PW, uint32_t key0, uint32_t key1,
                                                uint32_t stream_id, uint64_t first, int64_t N,
                                                uint32_t* __restrict__ out) {
    const int64_t h = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (h >= N) return;
    draw_sample<KM1>(thresh, half, n, PW, key0, key1, stream_id,
                     first + static_cast<uint64_t>(h), h, N, out);
}

// Every sample of every job of a plan segment (same n and K), grid-stride
// over the segment's global index.
template <int KM1>
__global__ __launch_bounds__(256) void k_sample_jobs(const JobDev* __restrict__ jobs,
                                                     const int64_t* __restrict__ offsets,
                                                     int n_jobs, int64_t total, int n, int PW) {
    SegSrc seg{};
    seg.jobs = jobs;
    seg.offsets = offsets;
    seg.n_jobs = n_jobs;
    seg.total = total;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += stride) {
        int j;
        int64_t h;
        seg_locate(seg, g, j, h);
        const JobDev& jd = jobs[j];
        draw_sample<KM1>(jd.thresh, jd.half, n, PW, static_cast<uint32_t>(jd.seed),
                         static_cast<uint32_t>(jd.seed >> 32), jd.stream_id,
                         static_cast<uint64_t>(h), h, jd.N, jd.samples);
    }
}

template <int KM1>
hipError_t launch_k(hipStream_t st, const rsr_model* m, uint64_t seed, uint32_t stream_id,
                    uint64_t first, int64_t N, uint32_t* d_samples) {
    const int threads = 256;
    const int64_t blocks = (N + threads - 1) / threads;
    hipLaunchKernelGGL(k_sample<KM1>, dim3(static_cast<unsigned>(blocks)), dim3(threads), 0, st,
                       m->d_thresh, m->d_half, m->n, plane_words(m->n), static_cast<uint32_t>(seed),
                       static_cast<uint32_t>(seed >> 32), stream_id, first, N, d_samples);
    return hipGetLastError();
}

template <int KM1>
hipError_t launch_jobs_k(hipStream_t st, int n, const JobDev* jobs, const int64_t* offsets,
                         int n_jobs, int64_t total, int grid_cap) {
    int64_t blocks = (total + 255) / 256;
    if (blocks > grid_cap) blocks = grid_cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_sample_jobs<KM1>, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                       jobs, offsets, n_jobs, total, n, plane_words(n));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sample_jobs(hipStream_t st, int n, int K, const JobDev* jobs,
                              const int64_t* offsets, int n_jobs, int64_t total, int grid_cap) {
    switch (K - 1) {
#define RSR_K_CASE(k) \
    case k: return launch_jobs_k<k>(st, n, jobs, offsets, n_jobs, total, grid_cap);
        RSR_K_CASE(1) RSR_K_CASE(2) RSR_K_CASE(3) RSR_K_CASE(4) RSR_K_CASE(5) RSR_K_CASE(6)
        RSR_K_CASE(7) RSR_K_CASE(8) RSR_K_CASE(9) RSR_K_CASE(10) RSR_K_CASE(11) RSR_K_CASE(12)
        RSR_K_CASE(13) RSR_K_CASE(14) RSR_K_CASE(15)
#undef RSR_K_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sample(hipStream_t st, const rsr_model* m, uint64_t seed, uint32_t stream_id,
                         uint64_t first, int64_t N, uint32_t* d_samples) {
    switch (m->K - 1) {
        case 1: return launch_k<1>(st, m, seed, stream_id, first, N, d_samples);
        case 2: return launch_k<2>(st, m, seed, stream_id, first, N, d_samples);
        case 3: return launch_k<3>(st, m, seed, stream_id, first, N, d_samples);
        case 4: return launch_k<4>(st, m, seed, stream_id, first, N, d_samples);
        case 5: return launch_k<5>(st, m, seed, stream_id, first, N, d_samples);
        case 6: return launch_k<6>(st, m, seed, stream_id, first, N, d_samples);
        case 7: return launch_k<7>(st, m, seed, stream_id, first, N, d_samples);
        case 8: return launch_k<8>(st, m, seed, stream_id, first, N, d_samples);
        case 9: return launch_k<9>(st, m, seed, stream_id, first, N, d_samples);
        case 10: return launch_k<10>(st, m, seed, stream_id, first, N, d_samples);
        case 11: return launch_k<11>(st, m, seed, stream_id, first, N, d_samples);
        case 12: return launch_k<12>(st, m, seed, stream_id, first, N, d_samples);
        case 13: return launch_k<13>(st, m, seed, stream_id, first, N, d_samples);
        case 14: return launch_k<14>(st, m, seed, stream_id, first, N, d_samples);
        case 15: return launch_k<15>(st, m, seed, stream_id, first, N, d_samples);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rsr
