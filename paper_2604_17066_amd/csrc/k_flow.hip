// Single-OD maximum flow with multi-state components (section 2.2: the
// reference states of this system are the d-minimal path and cut vectors):
// edge e carries up to x_e units in either direction, S = the maximum flow
// from source to sink, and the target is S >= d (d = the system level).
//
// One wavefront per sample.  Capacities (u8) and the current flow (i8, > 0
// from edge_u to edge_v) live in the wave's LDS.  Augmenting paths are found
// by edge-parallel sweeps over the residual graph, as the connectivity
// searches do: the unmarked end of an edge is marked when the marked end can
// still push along the edge; the marking edge is recorded as the node's
// parent.  One lane then walks the path from the sink, finds its bottleneck
// and pushes min(bottleneck, d - flow).  The flow is only ever grown up to d,
// so at most d augmentations decide S >= d (every push is at least 1).
//
// The boundary search (section 3.4) keeps the flow of its last evaluation:
// on the survival side, lowering the capacity of an edge that carries less
// than its capacity leaves that flow feasible, so the step is taken with no
// search; otherwise the flow is recomputed from zero at the new capacities,
// and restored from a copy if the step is undone.
#include "graph_search.h"

namespace rsr {
namespace {

constexpr int kFlowBlock = 256;
constexpr int kFlowWaves = kFlowBlock / 64;

using graph::bit;
using graph::fill;
using graph::wave_sync;

struct FlowSets {
    uint32_t* mark;    // [node_words]
    uint16_t* parent;  // [n_nodes]
    uint8_t* cap;      // [n_edges]
    int8_t* flow;      // [n_edges]
    int8_t* saved;     // [n_edges] copy of flow across a trial step
};

__host__ __device__ inline int flow_words(int n_nodes, int n_edges) {
    return ((n_nodes + 31) >> 5) + ((n_nodes + 1) >> 1) + 3 * ((n_edges + 3) >> 2);
}

__device__ inline FlowSets flow_sets(uint32_t* base, int n_nodes, int n_edges) {
    const int node_words = (n_nodes + 31) >> 5, half = (n_nodes + 1) >> 1;
    const int quarter = (n_edges + 3) >> 2;
    FlowSets f;
    f.mark = base;
    f.parent = reinterpret_cast<uint16_t*>(base + node_words);
    f.cap = reinterpret_cast<uint8_t*>(base + node_words + half);
    f.flow = reinterpret_cast<int8_t*>(base + node_words + half + quarter);
    f.saved = reinterpret_cast<int8_t*>(base + node_words + half + 2 * quarter);
    return f;
}

// Spare capacity of edge e in the direction away from node `from`.
__device__ __forceinline__ int spare(const FlowSets& f, int e, uint32_t uv, uint32_t from) {
    const int c = f.cap[e], fl = f.flow[e];
    return (uv & 0xFFFFu) == from ? c - fl : c + fl;
}

// One search for an augmenting path; returns whether the sink was reached.
__device__ bool find_path(const FlowSets& f, const uint32_t* __restrict__ s_edges, int n_edges,
                          int n_nodes, int source, int sink) {
    const int lane = threadIdx.x & 63;
    fill(f.mark, (n_nodes + 31) >> 5, 0u);
    wave_sync();
    if (lane == 0) f.mark[source >> 5] |= 1u << (source & 31);
    wave_sync();
    while (true) {
        bool changed = false;
        for (int e = lane; e < n_edges; e += 64) {
            const uint32_t uv = s_edges[e];
            const uint32_t u = uv & 0xFFFFu, v = uv >> 16;
            const uint32_t mu = bit(f.mark, u), mv = bit(f.mark, v);
            if (mu == mv) continue;
            const uint32_t from = mu ? u : v, to = mu ? v : u;
            if (spare(f, e, uv, from) <= 0) continue;
            f.parent[to] = static_cast<uint16_t>(e);
            atomicOr(&f.mark[to >> 5], 1u << (to & 31));
            changed = true;
        }
        wave_sync();
        if (__builtin_amdgcn_readfirstlane(static_cast<int>(bit(f.mark, sink)))) return true;
        if (!__any(changed)) return false;
    }
}

// Grows the current flow until it reaches `demand` or no augmenting path is
// left; returns min(flow value, demand).  `value` is the current flow value.
__device__ int augment_to(const FlowSets& f, int value, int demand,
                          const uint32_t* __restrict__ s_edges, int n_edges, int n_nodes,
                          int source, int sink) {
    const int lane = threadIdx.x & 63;
    while (value < demand && find_path(f, s_edges, n_edges, n_nodes, source, sink)) {
        int push = 0;
        if (lane == 0) {
            push = demand - value;
            int w = sink;
            for (int steps = 0; w != source && steps < n_nodes; ++steps) {
                const int e = f.parent[w];
                const uint32_t uv = s_edges[e];
                const uint32_t from = graph::other_end(uv, static_cast<uint32_t>(w));
                push = min(push, spare(f, e, uv, from));
                w = static_cast<int>(from);
            }
            w = sink;
            for (int steps = 0; w != source && steps < n_nodes; ++steps) {
                const int e = f.parent[w];
                const uint32_t uv = s_edges[e];
                const uint32_t from = graph::other_end(uv, static_cast<uint32_t>(w));
                f.flow[e] = static_cast<int8_t>(f.flow[e] + ((uv & 0xFFFFu) == from ? push : -push));
                w = static_cast<int>(from);
            }
        }
        push = __shfl(push, 0);
        wave_sync();
        if (push <= 0) break;  // cannot happen on a path the search found
        value += push;
    }
    return value < demand ? value : demand;
}

// Flow value from zero at the current capacities, capped at demand.
__device__ int flow_from_zero(const FlowSets& f, int demand, const uint32_t* __restrict__ s_edges,
                              int n_edges, int n_nodes, int source, int sink) {
    for (int e = threadIdx.x & 63; e < n_edges; e += 64) f.flow[e] = 0;
    wave_sync();
    return augment_to(f, 0, demand, s_edges, n_edges, n_nodes, source, sink);
}

__device__ void load_caps(const FlowSets& f, const uint32_t* xs, int64_t stride, int64_t h,
                          int PW, int K, int n_edges) {
    for (int e = threadIdx.x & 63; e < n_edges; e += 64) {
        int c = 0;
        for (int j = 0; j < K - 1; ++j)
            c += (xs[static_cast<int64_t>(j * PW + (e >> 5)) * stride + h] >> (e & 31)) & 1u;
        f.cap[e] = static_cast<uint8_t>(c);
    }
    wave_sync();
}

__global__ __launch_bounds__(kFlowBlock) void k_flow_eval(
    SegSrc seg, int PW, int K, const uint32_t* __restrict__ edges, int n_edges, int n_nodes,
    int source, int sink, int demand, const int32_t* __restrict__ list,
    const unsigned long long* __restrict__ count_ptr, int which,
    unsigned long long* __restrict__ n_evaluated) {
    extern __shared__ uint32_t lds[];
    const int64_t N = seg.total;
    const int64_t total = which == RSR_ALL ? N : static_cast<int64_t>(*count_ptr);
    if (blockIdx.x == 0 && threadIdx.x == 0 && n_evaluated)
        *n_evaluated = static_cast<unsigned long long>(total);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t first = static_cast<int64_t>(blockIdx.x) * kFlowWaves;
    if (first >= total) return;  // uniform per block

    uint32_t* s_edges = lds;
    for (int e = threadIdx.x; e < n_edges; e += kFlowBlock) s_edges[e] = edges[e];
    __syncthreads();
    const FlowSets f = flow_sets(lds + n_edges + wave * flow_words(n_nodes, n_edges), n_nodes, n_edges);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kFlowWaves;
    for (int64_t j = first + wave; j < total; j += stride) {
        const int64_t g = which == RSR_ALL ? j : static_cast<int64_t>(list[j]);
        int job;
        int64_t h, xstride;
        seg_locate(seg, g, job, h);
        load_caps(f, seg_words(seg, job, xstride), xstride, h, PW, K, n_edges);
        const int v = flow_from_zero(f, demand, s_edges, n_edges, n_nodes, source, sink);
        if (lane == 0) seg_Y(seg, job)[h] = v >= demand ? 1 : 0;
        wave_sync();
    }
}

__global__ __launch_bounds__(kFlowBlock) void k_boundary_flow(
    const uint32_t* __restrict__ xs, int64_t N, int PW, int K, const uint32_t* __restrict__ edges,
    int n_edges, int n_nodes, int source, int sink, int demand, const int64_t* __restrict__ pick,
    int64_t n_pick, uint8_t* __restrict__ rows, uint8_t* __restrict__ side) {
    extern __shared__ uint32_t lds[];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    uint32_t* s_edges = lds;
    for (int e = threadIdx.x; e < n_edges; e += kFlowBlock) s_edges[e] = edges[e];
    __syncthreads();
    const FlowSets f = flow_sets(lds + n_edges + wave * flow_words(n_nodes, n_edges), n_nodes, n_edges);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kFlowWaves;
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * kFlowWaves + wave; j < n_pick; j += stride) {
        const int64_t h = pick[j];
        if (h < 0 || h >= N) {  // not a sample index: reported, nothing read
            if (lane == 0) side[j] = 0xFF;
            continue;
        }
        load_caps(f, xs, N, h, PW, K, n_edges);
        int value = flow_from_zero(f, demand, s_edges, n_edges, n_nodes, source, sink);
        const bool survival = value >= demand;
        for (int i = 0; i < n_edges; ++i) {
            // Walk component i one state at a time; f.cap[i] is its state.
            while (true) {
                const int c = f.cap[i];
                if (survival ? c == 0 : c == K - 1) break;
                if (survival) {
                    const int fl = f.flow[i];
                    if ((fl < 0 ? -fl : fl) < c) {  // the flow still fits: S >= d stays
                        if (lane == 0) f.cap[i] = static_cast<uint8_t>(c - 1);
                        wave_sync();
                        continue;
                    }
                    for (int e = lane; e < n_edges; e += 64) f.saved[e] = f.flow[e];
                    if (lane == 0) f.cap[i] = static_cast<uint8_t>(c - 1);
                    wave_sync();
                    const int v = flow_from_zero(f, demand, s_edges, n_edges, n_nodes, source, sink);
                    if (v >= demand) continue;
                    // Undo: capacity and the flow that went with it.
                    for (int e = lane; e < n_edges; e += 64) f.flow[e] = f.saved[e];
                    if (lane == 0) f.cap[i] = static_cast<uint8_t>(c);
                    wave_sync();
                    break;
                } else {
                    // The current flow stays feasible when a capacity grows.
                    for (int e = lane; e < n_edges; e += 64) f.saved[e] = f.flow[e];
                    if (lane == 0) f.cap[i] = static_cast<uint8_t>(c + 1);
                    wave_sync();
                    const int v = augment_to(f, value, demand, s_edges, n_edges, n_nodes, source, sink);
                    if (v < demand) {
                        value = v;
                        continue;
                    }
                    for (int e = lane; e < n_edges; e += 64) f.flow[e] = f.saved[e];
                    if (lane == 0) f.cap[i] = static_cast<uint8_t>(c);
                    wave_sync();
                    break;
                }
            }
        }
        uint8_t* out = rows + j * static_cast<int64_t>(n_edges);
        for (int e = lane; e < n_edges; e += 64) out[e] = f.cap[e];
        if (lane == 0) side[j] = survival ? 1 : 0;
        wave_sync();
    }
}

}  // namespace

size_t flow_lds_bytes(const rsr_system* sys) {
    return sizeof(uint32_t) * (static_cast<size_t>(sys->n_edges) +
                               kFlowWaves * static_cast<size_t>(flow_words(sys->n_nodes, sys->n_edges)));
}

hipError_t launch_flow_eval(hipStream_t st, const rsr_system* sys, const SegSrc& seg,
                            const int32_t* d_list, const uint64_t* d_count, int which,
                            uint64_t* d_n_evaluated, int grid_blocks) {
    const int64_t need = (seg.total + kFlowWaves - 1) / kFlowWaves;
    int blocks = static_cast<int>(need < grid_blocks ? need : grid_blocks);
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_flow_eval, dim3(blocks), dim3(kFlowBlock), flow_lds_bytes(sys), st, seg,
                       plane_words(sys->n_edges), sys->K, sys->d_edges, sys->n_edges, sys->n_nodes,
                       sys->source, sys->sink, sys->level, d_list,
                       reinterpret_cast<const unsigned long long*>(d_count), which,
                       reinterpret_cast<unsigned long long*>(d_n_evaluated));
    return hipGetLastError();
}

hipError_t launch_boundary_flow(hipStream_t st, const rsr_system* sys, const uint32_t* xs,
                                int64_t N, const int64_t* d_pick, int64_t n_pick, uint8_t* d_rows,
                                uint8_t* d_side, int grid_cap) {
    int64_t blocks = (n_pick + kFlowWaves - 1) / kFlowWaves;
    if (blocks > grid_cap) blocks = grid_cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_boundary_flow, dim3(static_cast<unsigned>(blocks)), dim3(kFlowBlock),
                       flow_lds_bytes(sys), st, xs, N, plane_words(sys->n_edges), sys->K,
                       sys->d_edges, sys->n_edges, sys->n_nodes, sys->source, sys->sink,
                       sys->level, d_pick, n_pick, d_rows, d_side);
    return hipGetLastError();
}

}  // namespace rsr
