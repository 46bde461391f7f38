// Reductions: estimator counts (section 3.3.1) and the score-function
// gradient counts.
//
// k_counts: one pass over flags (and Y) with per-thread counters, a wavefront
// reduction and one 64-bit atomic per counter per wave.
//
// k_grad_bits: a[j][i] = #{h : Y_h = 1 and x_{h,i} >= j} for every thermometer
// bit (plane j, component i).  Block column y = packed word w; each thread
// walks a strided run of samples, keeps 32 per-bit counters of its masked
// words, and the block adds them into a[w][*] with one atomic per bit per
// wave.  Blocks in column 0 also count #{Y = 1}.
// k_grad_finalize: c[i][s] = a[s][i] - a[s+1][i] (a[0][i] = #{Y = 1},
// a[K][i] = 0), G[i][s] = (float)c / ((float)N * p[i][s]).
#include "rsr_internal.h"

namespace rsr {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__global__ __launch_bounds__(kBlock) void k_fill_u64(unsigned long long* p, int64_t count,
                                                     unsigned long long value) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < count) p[i] = value;
}

__global__ __launch_bounds__(kBlock) void k_counts(const uint8_t* __restrict__ flags,
                                                   const uint8_t* __restrict__ Y, int64_t N,
                                                   unsigned long long* __restrict__ out) {
    unsigned long long nL = 0, nU = 0, nu = 0, nb = 0, nuu = 0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t h = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; h < N; h += stride) {
        const uint32_t f = flags[h];
        const uint32_t lo = f & 1u, up = (f >> 1) & 1u;
        nL += lo;
        nU += (!lo && up) ? 1u : 0u;
        const bool unk = !lo && !up;
        nu += unk ? 1u : 0u;
        nb += lo & up;
        if (unk && Y) nuu += Y[h] ? 1u : 0u;
    }
    nL = wave_sum(nL);
    nU = wave_sum(nU);
    nu = wave_sum(nu);
    nb = wave_sum(nb);
    nuu = wave_sum(nuu);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&out[0], nL);
        atomicAdd(&out[1], nU);
        atomicAdd(&out[2], nu);
        atomicAdd(&out[3], nb);
        atomicAdd(&out[4], nuu);
    }
}

__global__ __launch_bounds__(kBlock) void k_grad_bits(const uint32_t* __restrict__ xs,
                                                      const uint8_t* __restrict__ Y, int64_t N,
                                                      unsigned long long* __restrict__ acc,
                                                      int W) {
    const int w = blockIdx.y;
    uint32_t c[32];
#pragma unroll
    for (int b = 0; b < 32; ++b) c[b] = 0;
    uint32_t ny = 0;
    const uint32_t* row = xs + static_cast<int64_t>(w) * N;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t h = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; h < N; h += stride) {
        const uint32_t y = Y[h] ? 0xFFFFFFFFu : 0u;
        ny += y & 1u;
        const uint32_t v = row[h] & y;
#pragma unroll
        for (int b = 0; b < 32; ++b) c[b] += (v >> b) & 1u;
    }
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int b = 0; b < 32; ++b) {
        const uint32_t s = wave_sum32(c[b]);
        if (lane == 0 && s) atomicAdd(&acc[w * 32 + b], static_cast<unsigned long long>(s));
    }
    if (w == 0) {
        const uint32_t s = wave_sum32(ny);
        if (lane == 0 && s) atomicAdd(&acc[W * 32], static_cast<unsigned long long>(s));
    }
}

__global__ __launch_bounds__(kBlock) void k_grad_finalize(const unsigned long long* __restrict__ acc,
                                                          const float* __restrict__ p, int n,
                                                          int K, int PW, int W, int64_t N,
                                                          float* __restrict__ G,
                                                          unsigned long long* __restrict__ counts) {
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= n * K) return;
    const int i = idx / K, s = idx % K;
    auto level_count = [&](int j) -> unsigned long long {
        if (j == 0) return acc[W * 32];
        if (j >= K) return 0ull;
        return acc[((j - 1) * PW + (i >> 5)) * 32 + (i & 31)];
    };
    const unsigned long long cnt = level_count(s) - level_count(s + 1);
    const float pv = p[idx];
    const float g = pv > 0.0f ? static_cast<float>(cnt) / (static_cast<float>(N) * pv) : 0.0f;
    G[idx] = g;
    if (counts) counts[idx] = cnt;
}

}  // namespace

hipError_t launch_fill_u64(hipStream_t st, uint64_t* p, int64_t count, uint64_t value) {
    const dim3 grid(static_cast<unsigned>((count + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_fill_u64, grid, dim3(kBlock), 0, st,
                       reinterpret_cast<unsigned long long*>(p), count,
                       static_cast<unsigned long long>(value));
    return hipGetLastError();
}

hipError_t launch_counts(hipStream_t st, const uint8_t* d_flags, const uint8_t* d_Y, int64_t N,
                         uint64_t* d_counters) {
    int64_t blocks = (N + kBlock * 8 - 1) / (kBlock * 8);
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_counts, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, st, d_flags,
                       d_Y, N, reinterpret_cast<unsigned long long*>(d_counters));
    return hipGetLastError();
}

hipError_t launch_grad(hipStream_t st, const rsr_model* m, const uint32_t* d_samples,
                       const uint8_t* d_Y, int64_t N, uint64_t* d_acc, float* d_G,
                       uint64_t* d_counts) {
    const int PW = plane_words(m->n);
    const int W = (m->K - 1) * PW;
    int64_t bx = (N + kBlock * 16 - 1) / (kBlock * 16);
    if (bx > 512) bx = 512;
    if (bx < 1) bx = 1;
    hipLaunchKernelGGL(k_grad_bits, dim3(static_cast<unsigned>(bx), W), dim3(kBlock), 0, st,
                       d_samples, d_Y, N, reinterpret_cast<unsigned long long*>(d_acc), W);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int total = m->n * m->K;
    hipLaunchKernelGGL(k_grad_finalize, dim3((total + kBlock - 1) / kBlock), dim3(kBlock), 0, st,
                       reinterpret_cast<const unsigned long long*>(d_acc), m->d_p, m->n, m->K, PW,
                       W, N, d_G, reinterpret_cast<unsigned long long*>(d_counts));
    return hipGetLastError();
}

}  // namespace rsr
