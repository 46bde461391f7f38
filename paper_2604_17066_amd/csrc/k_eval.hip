// Stage-2 evaluation of the system function on the samples left
// unclassified (section 3.5).
//
// k_label turns flags into Y (lower -> 0, upper -> 1) and appends the indices
// of unclassified samples to a list: one ballot per wave, one atomic per wave
// for the wave's slots.
//
// k_bfs evaluates s-t connectivity at a level on listed samples: one
// wavefront per sample, two node bitmasks in LDS grown from the source and
// from the sink, and edge-parallel sweeps (lane l owns edges l, l+64, ...; an
// edge is usable when the sample's thermometer plane `level` has its bit
// set).  A sweep marks, for each set, the other end of every usable edge with
// exactly one end in it; the search stops when the sets share a node
// (connected) or one of them stops growing (its component is complete, so
// they never meet).  Each sweep marks a new node in both sets or ends the
// search, so there are at most n_nodes sweeps.  The grid
// is sized on the host without knowing the number of unclassified samples
// (it lives on the device), and waves stride over the list.
#include "graph_search.h"

namespace rsr {
namespace {

constexpr int kLabelBlock = 256;
constexpr int kBfsBlock = 256;
constexpr int kWavesPerBfsBlock = kBfsBlock / 64;
constexpr int kMaxNodeWords = RSR_MAX_NODES / 32;

__global__ __launch_bounds__(kLabelBlock) void k_label(SegSrc seg, int32_t* __restrict__ list,
                                                       unsigned long long* __restrict__ counter) {
    const int lane = threadIdx.x & 63;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kLabelBlock;
    // Grid-stride over global indices; the loop bound is wave-uniform.
    for (int64_t g0 = static_cast<int64_t>(blockIdx.x) * kLabelBlock + (threadIdx.x & ~63);
         g0 < seg.total; g0 += stride) {
        const int64_t g = g0 + lane;
        const bool in = g < seg.total;
        int job = 0;
        int64_t h = 0;
        if (in) seg_locate(seg, g, job, h);
        const uint8_t f = in ? seg_flags(seg, job)[h] : 1;
        const bool unknown = (f & 3u) == 0u;
        if (in) seg_Y(seg, job)[h] = (f & 1u) ? 0 : ((f & 2u) ? 1 : 0);
        const uint64_t mask = __ballot(unknown);
        if (mask == 0) continue;
        const int leader = __ffsll(static_cast<unsigned long long>(mask)) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(counter, static_cast<unsigned long long>(__popcll(mask)));
        base = __shfl(base, leader);
        if (unknown) {
            const uint64_t below = mask & ((1ull << lane) - 1ull);
            list[base + __popcll(below)] = static_cast<int32_t>(g);
        }
    }
}

__global__ __launch_bounds__(kBfsBlock) void k_bfs(
    SegSrc seg, int PW, int plane, const uint32_t* __restrict__ edges, int n_edges, int n_nodes,
    int source, int sink, const int32_t* __restrict__ list,
    const unsigned long long* __restrict__ count_ptr, int which,
    unsigned long long* __restrict__ n_evaluated) {
    const int64_t N = seg.total;
    __shared__ uint32_t s_edges[RSR_MAX_BITS];
    __shared__ uint32_t s_reach[kWavesPerBfsBlock][kMaxNodeWords];
    __shared__ uint32_t s_reach_t[kWavesPerBfsBlock][kMaxNodeWords];

    const int64_t total = which == RSR_ALL ? N : static_cast<int64_t>(*count_ptr);
    if (blockIdx.x == 0 && threadIdx.x == 0 && n_evaluated)
        *n_evaluated = static_cast<unsigned long long>(total);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t first = static_cast<int64_t>(blockIdx.x) * kWavesPerBfsBlock;
    if (first >= total) return;  // uniform per block

    for (int e = threadIdx.x; e < n_edges; e += kBfsBlock) s_edges[e] = edges[e];
    __syncthreads();

    const int node_words = (n_nodes + 31) >> 5;
    const int edge_rounds = (n_edges + 63) >> 6;
    uint32_t* reach = s_reach[wave];
    uint32_t* reach_t = s_reach_t[wave];
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kWavesPerBfsBlock;

    for (int64_t j = first + wave; j < total; j += stride) {
        const int64_t g = which == RSR_ALL ? j : static_cast<int64_t>(list[j]);
        int job;
        int64_t h, xstride;
        seg_locate(seg, g, job, h);
        const uint32_t* xs = seg_words(seg, job, xstride);
        // Usable-edge mask of this lane's edges.
        uint64_t usable = 0;
        for (int k = 0; k < edge_rounds; ++k) {
            const int e = lane + 64 * k;
            if (e < n_edges) {
                const uint32_t word = xs[static_cast<int64_t>(plane * PW + (e >> 5)) * xstride + h];
                usable |= static_cast<uint64_t>((word >> (e & 31)) & 1u) << k;
            }
        }
        for (int wd = lane; wd < node_words; wd += 64) reach[wd] = reach_t[wd] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
            reach[source >> 5] = 1u << (source & 31);
            reach_t[sink >> 5] |= 1u << (sink & 31);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        // Two sets grow at once, from the source and from the sink: they
        // meet iff the sample connects s and t, and one that stops growing is
        // a whole component (then they never meet).  Growing from both ends
        // halves the number of sweeps.
        int result = 0;
        while (true) {
            bool changed_s = false, changed_t = false;
            uint64_t todo = usable;
            while (todo) {
                const int k = __ffsll(static_cast<unsigned long long>(todo)) - 1;
                todo &= todo - 1;
                const uint32_t uv = s_edges[lane + 64 * k];
                const uint32_t u = uv & 0xFFFFu, v = uv >> 16;
                const uint32_t su = (__hip_atomic_load(&reach[u >> 5], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WAVEFRONT) >> (u & 31)) & 1u;
                const uint32_t sv = (__hip_atomic_load(&reach[v >> 5], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WAVEFRONT) >> (v & 31)) & 1u;
                const uint32_t tu = (__hip_atomic_load(&reach_t[u >> 5], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WAVEFRONT) >> (u & 31)) & 1u;
                const uint32_t tv = (__hip_atomic_load(&reach_t[v >> 5], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_WAVEFRONT) >> (v & 31)) & 1u;
                if (su != sv) {
                    const uint32_t w = su ? v : u;
                    atomicOr(&reach[w >> 5], 1u << (w & 31));
                    changed_s = true;
                }
                if (tu != tv) {
                    const uint32_t w = tu ? v : u;
                    atomicOr(&reach_t[w >> 5], 1u << (w & 31));
                    changed_t = true;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            bool meet = false;
            for (int wd = lane; wd < node_words; wd += 64)
                meet = meet || (__hip_atomic_load(&reach[wd], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_WAVEFRONT) &
                                __hip_atomic_load(&reach_t[wd], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_WAVEFRONT)) != 0u;
            if (__any(meet)) {
                result = 1;
                break;
            }
            if (!__any(changed_s) || !__any(changed_t)) break;
        }
        if (lane == 0) seg_Y(seg, job)[h] = static_cast<uint8_t>(result);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// Global connectivity (edges work at state >= 1, target S >= level, level 1
// or 2) on the listed samples: one wavefront per sample, the same listing
// and striding as k_bfs, the test of graph_search.h.
__global__ __launch_bounds__(kBfsBlock) void k_global(
    SegSrc seg, const uint32_t* __restrict__ edges, int n_edges, int n_nodes, int level,
    const int32_t* __restrict__ list, const unsigned long long* __restrict__ count_ptr,
    int which, unsigned long long* __restrict__ n_evaluated) {
    extern __shared__ uint32_t lds[];
    const int64_t N = seg.total;
    const int64_t total = which == RSR_ALL ? N : static_cast<int64_t>(*count_ptr);
    if (blockIdx.x == 0 && threadIdx.x == 0 && n_evaluated)
        *n_evaluated = static_cast<unsigned long long>(total);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t first = static_cast<int64_t>(blockIdx.x) * kWavesPerBfsBlock;
    if (first >= total) return;  // uniform per block

    uint32_t* s_edges = lds;
    for (int e = threadIdx.x; e < n_edges; e += kBfsBlock) s_edges[e] = edges[e];
    __syncthreads();
    const graph::GlobalSets g = graph::global_sets(
        lds + n_edges + wave * graph::global_words(n_nodes, n_edges), n_nodes, n_edges);
    const int edge_rounds = (n_edges + 63) >> 6;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kWavesPerBfsBlock;
    for (int64_t j = first + wave; j < total; j += stride) {
        const int64_t g_idx = which == RSR_ALL ? j : static_cast<int64_t>(list[j]);
        int job;
        int64_t h, xstride;
        seg_locate(seg, g_idx, job, h);
        const uint32_t* xs = seg_words(seg, job, xstride);
        uint64_t usable = 0;  // plane 0 = [x >= 1]
        for (int k = 0; k < edge_rounds; ++k) {
            const int e = lane + 64 * k;
            if (e < n_edges) {
                const uint32_t word = xs[static_cast<int64_t>(e >> 5) * xstride + h];
                usable |= static_cast<uint64_t>((word >> (e & 31)) & 1u) << k;
            }
        }
        const bool up = graph::global_at_least(usable, level, s_edges, n_edges, n_nodes, g);
        if (lane == 0) seg_Y(seg, job)[h] = up ? 1 : 0;
        graph::wave_sync();
    }
}

}  // namespace

hipError_t launch_label(hipStream_t st, const SegSrc& seg, int32_t* d_list, uint64_t* d_counter,
                        int grid_cap) {
    int64_t blocks = (seg.total + kLabelBlock - 1) / kLabelBlock;
    if (blocks > grid_cap) blocks = grid_cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_label, dim3(static_cast<unsigned>(blocks)), dim3(kLabelBlock), 0, st, seg,
                       d_list, reinterpret_cast<unsigned long long*>(d_counter));
    return hipGetLastError();
}

hipError_t launch_bfs(hipStream_t st, const rsr_system* sys, const SegSrc& seg,
                      const int32_t* d_list, const uint64_t* d_count, int which,
                      uint64_t* d_n_evaluated, int grid_blocks) {
    const int64_t need = (seg.total + kWavesPerBfsBlock - 1) / kWavesPerBfsBlock;
    int blocks = static_cast<int>(need < grid_blocks ? need : grid_blocks);
    if (blocks < 1) blocks = 1;
    if (sys->kind == RSR_SYS_MAX_FLOW)
        return launch_flow_eval(st, sys, seg, d_list, d_count, which, d_n_evaluated, grid_blocks);
    if (sys->kind == RSR_SYS_GLOBAL_CONNECTIVITY) {
        const size_t lds = sizeof(uint32_t) *
            (static_cast<size_t>(sys->n_edges) +
             kWavesPerBfsBlock * static_cast<size_t>(((sys->n_nodes + 31) >> 5) +
                                                     ((sys->n_edges + 31) >> 5) +
                                                     2 * ((sys->n_nodes + 1) >> 1)));
        hipLaunchKernelGGL(k_global, dim3(blocks), dim3(kBfsBlock), lds, st, seg, sys->d_edges,
                           sys->n_edges, sys->n_nodes, sys->level, d_list,
                           reinterpret_cast<const unsigned long long*>(d_count), which,
                           reinterpret_cast<unsigned long long*>(d_n_evaluated));
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_bfs, dim3(blocks), dim3(kBfsBlock), 0, st, seg, plane_words(sys->n_edges),
                       sys->level - 1, sys->d_edges, sys->n_edges, sys->n_nodes, sys->source,
                       sys->sink, d_list, reinterpret_cast<const unsigned long long*>(d_count),
                       which, reinterpret_cast<unsigned long long*>(d_n_evaluated));
    return hipGetLastError();
}

}  // namespace rsr
