// Monte Carlo sampler: Philox4x32-10 words compared against integer
// inverse-CDF thresholds, written straight into the packed thermometer layout
// (word-major [W][N]; see rsr.h).
//
// One thread draws one sample.  A Philox block gives the words of four
// consecutive components, so a 32-component word of every plane takes eight
// blocks; the finished words are stored with coalesced 32-bit stores (lanes
// hold consecutive samples).  The thresholds are identical for every thread,
// so they are read through the scalar cache.
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
        const uint32_t y0 = static_cast<uint32_t>(b >> 32) ^ c1 ^ k0;
        const uint32_t y2 = static_cast<uint32_t>(a >> 32) ^ c3 ^ k1;
        c1 = static_cast<uint32_t>(b);
        c3 = static_cast<uint32_t>(a);
        c0 = y0;
        c2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// Draws sample index g (its Philox counter) and stores it as column h of the
// word-major [W][N] array out.  KM1 = K - 1 thermometer planes.
template <int KM1>
__device__ __forceinline__ void draw_sample(const uint64_t* __restrict__ thresh, int n, int PW,
                                            uint32_t key0, uint32_t key1, uint32_t stream_id,
                                            uint64_t g, int64_t h, int64_t N,
                                            uint32_t* __restrict__ out) {
    const uint32_t glo = static_cast<uint32_t>(g), ghi = static_cast<uint32_t>(g >> 32);
    for (int wi = 0; wi < PW; ++wi) {
        uint32_t acc[KM1];
#pragma unroll
        for (int s = 0; s < KM1; ++s) acc[s] = 0;
        const int base = wi * 32;
        const int groups = min(8, (n - base + 3) >> 2);
        for (int q = 0; q < groups; ++q) {
            const int i0 = base + q * 4;
            const Philox4 u = philox4x32_10(static_cast<uint32_t>(i0 >> 2), glo, ghi, stream_id,
                                            key0, key1);
            const uint32_t words[4] = {u.v0, u.v1, u.v2, u.v3};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int i = i0 + k;
                if (i < n) {
                    const uint64_t w = words[k];
#pragma unroll
                    for (int s = 0; s < KM1; ++s) {
                        const uint32_t bit = (w >= thresh[i * KM1 + s]) ? 1u : 0u;
                        acc[s] |= bit << (i & 31);
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
__global__ __launch_bounds__(256) void k_sample(const uint64_t* __restrict__ thresh, int n,
                                                int PW, uint32_t key0, uint32_t key1,
                                                uint32_t stream_id, uint64_t first, int64_t N,
                                                uint32_t* __restrict__ out) {
    const int64_t h = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (h >= N) return;
    draw_sample<KM1>(thresh, n, PW, key0, key1, stream_id, first + static_cast<uint64_t>(h), h,
                     N, out);
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
        draw_sample<KM1>(jd.thresh, n, PW, static_cast<uint32_t>(jd.seed),
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
                       m->d_thresh, m->n, plane_words(m->n), static_cast<uint32_t>(seed),
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
