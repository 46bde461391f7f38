// Ordered selection of unclassified samples for the Stage-1 loop (section
// 3.4-3.5): the first B sample indices h, in increasing order, whose flags
// have neither the lower nor the upper bit.  Samples are i.i.d., so the
// lowest-index unclassified samples are a uniformly random subset of them,
// and taking them in index order keeps the loop reproducible.
//
// Three passes over contiguous chunks of the flags, one block per chunk:
// count per chunk, exclusive scan of the chunk counts (one block), then each
// chunk writes its unclassified indices at their global ranks below B.
#include "rsr_internal.h"

namespace rsr {
namespace {

constexpr int kPickBlock = 256;
constexpr int kPickWaves = kPickBlock / 64;
constexpr int kMaxPickBlocks = 1024;

__device__ __forceinline__ bool unclassified(const uint8_t* flags, int64_t h, int64_t hi) {
    return h < hi && (flags[h] & 3u) == 0u;
}

__global__ __launch_bounds__(kPickBlock) void k_pick_count(const uint8_t* __restrict__ flags,
                                                           int64_t N, int64_t chunk,
                                                           uint64_t* __restrict__ part) {
    __shared__ uint32_t s_wave[kPickWaves];
    const int64_t lo = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t hi = lo + chunk < N ? lo + chunk : N;
    uint32_t c = 0;
    for (int64_t h = lo + threadIdx.x; h < hi; h += kPickBlock) c += unclassified(flags, h, hi);
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < kPickWaves; ++w) t += s_wave[w];
        part[blockIdx.x] = t;
    }
}

// part[b] becomes the number of unclassified samples before chunk b; *total
// the number in all chunks.
__global__ void k_pick_scan(uint64_t* __restrict__ part, int blocks, uint64_t* __restrict__ total) {
    if (threadIdx.x != 0) return;
    uint64_t run = 0;
    for (int b = 0; b < blocks; ++b) {
        const uint64_t c = part[b];
        part[b] = run;
        run += c;
    }
    *total = run;
}

__global__ __launch_bounds__(kPickBlock) void k_pick_write(const uint8_t* __restrict__ flags,
                                                           int64_t N, int64_t chunk,
                                                           const uint64_t* __restrict__ off,
                                                           int64_t B, int64_t* __restrict__ pick) {
    __shared__ uint32_t s_wave[kPickWaves];
    const int64_t lo = static_cast<int64_t>(blockIdx.x) * chunk;
    const int64_t hi = lo + chunk < N ? lo + chunk : N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t base = off[blockIdx.x];
    for (int64_t tile = lo; tile < hi && base < static_cast<uint64_t>(B); tile += kPickBlock) {
        const int64_t h = tile + threadIdx.x;
        const bool u = unclassified(flags, h, hi);
        const uint64_t mask = __ballot(u);
        if (lane == 0) s_wave[wave] = static_cast<uint32_t>(__popcll(mask));
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int w = 0; w < kPickWaves; ++w) {
            before += w < wave ? s_wave[w] : 0u;
            all += s_wave[w];
        }
        const uint64_t rank =
            base + before + static_cast<uint64_t>(__popcll(mask & ((1ull << lane) - 1ull)));
        if (u && rank < static_cast<uint64_t>(B)) pick[rank] = h;
        base += all;
        __syncthreads();  // s_wave is rewritten by the next tile
    }
}

}  // namespace

hipError_t launch_pick(hipStream_t st, const uint8_t* d_flags, int64_t N, int64_t B,
                       int64_t* d_pick, uint64_t* d_part, uint64_t* d_total) {
    int64_t blocks = (N + 16 * kPickBlock - 1) / (16 * kPickBlock);
    if (blocks > kMaxPickBlocks) blocks = kMaxPickBlocks;
    if (blocks < 1) blocks = 1;
    int64_t chunk = (N + blocks - 1) / blocks;
    chunk = (chunk + kPickBlock - 1) / kPickBlock * kPickBlock;
    const dim3 grid(static_cast<unsigned>(blocks));
    hipLaunchKernelGGL(k_pick_count, grid, dim3(kPickBlock), 0, st, d_flags, N, chunk, d_part);
    hipLaunchKernelGGL(k_pick_scan, dim3(1), dim3(64), 0, st, d_part, static_cast<int>(blocks),
                       d_total);
    if (B > 0)
        hipLaunchKernelGGL(k_pick_write, grid, dim3(kPickBlock), 0, st, d_flags, N, chunk, d_part,
                           B, d_pick);
    return hipGetLastError();
}

}  // namespace rsr
