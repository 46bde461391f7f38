// Componentwise boundary search (section 3.4) for s-t connectivity at a
// level, many start samples at once: one wavefront per start sample.
//
// The search visits the components (edges) in index order and moves each one
// state at a time towards K-1 (failure start) or 0 (survival start), undoing
// the step that changes the system side.  For this system the side depends
// only on which edges are usable (state >= level), so a component's walk has
// one decisive step: for a failure start, making an unusable edge usable; for
// a survival start, making a usable edge unusable.  Every other step leaves
// the side unchanged and is taken.  The result is therefore fixed by the final
// usable set U':
//   failure start:  x'_i = K-1 if U'_i else level-1   (a maximal failure state)
//   survival start: x'_i = level if U'_i else 0       (a minimal survival state)
//
// The decisive steps are answered with as little graph search as possible:
//  * failure side: R = nodes reachable from s over U (t is not in R).  Making
//    edge (u, v) usable changes R only when exactly one end is in R; then R is
//    grown from the other end on a copy, and the step is undone if t is
//    reached.  Otherwise the step is taken with no search at all.
//  * survival side: a witness s-t path P over U is kept as an edge set.
//    Removing an edge outside P keeps P, so the step is taken with no search.
//    Removing an edge of P needs a new search over U minus the edge: if t is
//    still reached the step is taken and P is replaced by the new tree path,
//    otherwise the step is undone.
//
// Searches are edge-parallel sweeps over the usable edges (lane l owns edges
// l, l+64, ...), marking the unmarked end of every edge with exactly one
// marked end and recording that edge as the node's parent.  All lanes of a
// wave read the marks before any lane writes in the same step, so a parent
// always points at a node marked in an earlier step and the parent chain of
// every marked node ends at s.
#include "graph_search.h"

namespace rsr {
namespace {

using graph::bit;
using graph::fill;
using graph::wave_sync;

constexpr int kBoundaryBlock = 256;
constexpr int kBoundaryWaves = kBoundaryBlock / 64;

// Per-wave LDS working set.
struct WaveSets {
    uint32_t* reach;   // [node_words]
    uint32_t* trial;   // [node_words]
    uint32_t* path;    // [edge_words] witness path edges (survival side)
    uint16_t* parent;  // [n_nodes] edge that marked the node
};

// s-t search from the nodes of `set` over the usable edges; parents recorded
// when `parents`.
__device__ __forceinline__ bool grow(uint32_t* set, uint64_t usable,
                                     const uint32_t* __restrict__ s_edges, int sink,
                                     uint16_t* parent, bool parents) {
    return graph::grow(set, usable, s_edges, sink, parents ? parent : nullptr, nullptr);
}

// Marks the tree path from sink back to source in `path` (one lane walks it;
// a tree path has fewer than n_nodes edges, which also bounds the walk).
__device__ void trace_path(const WaveSets& ws, int edge_words, const uint32_t* __restrict__ s_edges,
                           int n_nodes, int n_edges, int source, int sink) {
    fill(ws.path, edge_words, 0u);
    wave_sync();
    if ((threadIdx.x & 63) == 0) {
        int w = sink;
        for (int steps = 0; w != source && steps < n_nodes; ++steps) {
            const int e = ws.parent[w];
            if (e >= n_edges) break;  // cannot happen for a node marked by this search
            ws.path[e >> 5] |= 1u << (e & 31);
            const uint32_t uv = s_edges[e];
            const int u = static_cast<int>(uv & 0xFFFFu), v = static_cast<int>(uv >> 16);
            w = (u == w) ? v : u;
        }
    }
    wave_sync();
}

__global__ __launch_bounds__(kBoundaryBlock) void k_boundary(
    const uint32_t* __restrict__ xs, int64_t N, int PW, const uint32_t* __restrict__ edges,
    int n_edges, int n_nodes, int source, int sink, int K, int level,
    const int64_t* __restrict__ pick, int64_t n_pick, uint8_t* __restrict__ rows,
    uint8_t* __restrict__ side) {
    extern __shared__ uint32_t lds[];
    const int node_words = (n_nodes + 31) >> 5;
    const int edge_words = (n_edges + 31) >> 5;
    const int parent_words = (n_nodes + 1) >> 1;
    const int per_wave = 2 * node_words + edge_words + parent_words;
    uint32_t* s_edges = lds;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    uint32_t* mine = lds + n_edges + wave * per_wave;
    WaveSets ws{mine, mine + node_words, mine + 2 * node_words,
                reinterpret_cast<uint16_t*>(mine + 2 * node_words + edge_words)};

    for (int e = threadIdx.x; e < n_edges; e += kBoundaryBlock) s_edges[e] = edges[e];
    __syncthreads();

    const int rounds = (n_edges + 63) >> 6;
    const int plane = level - 1;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBoundaryWaves;
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * kBoundaryWaves + wave; j < n_pick;
         j += stride) {
        const int64_t h = pick[j];
        if (h < 0 || h >= N) {  // not a sample index: reported, nothing read
            if (lane == 0) side[j] = 0xFF;
            continue;
        }
        uint64_t usable = 0;
        for (int k = 0; k < rounds; ++k) {
            const int e = lane + 64 * k;
            if (e < n_edges) {
                const uint32_t word = xs[static_cast<int64_t>(plane * PW + (e >> 5)) * N + h];
                usable |= static_cast<uint64_t>((word >> (e & 31)) & 1u) << k;
            }
        }
        // Side of the start sample: one search from s, with parents.
        fill(ws.reach, node_words, 0u);
        wave_sync();
        if (lane == 0) ws.reach[source >> 5] |= 1u << (source & 31);
        wave_sync();
        const bool survival = source == sink || grow(ws.reach, usable, s_edges, sink, ws.parent, true);

        if (!survival) {
            uint32_t* reach = ws.reach;
            uint32_t* trial = ws.trial;
            for (int i = 0; i < n_edges; ++i) {
                const int owner = i & 63, k = i >> 6;
                const uint64_t mine_bits = __shfl(usable, owner);
                if ((mine_bits >> k) & 1u) continue;  // already usable: stays, walks to K-1
                const uint32_t uv = s_edges[i];
                const uint32_t u = uv & 0xFFFFu, v = uv >> 16;
                const uint32_t ru = bit(reach, u), rv = bit(reach, v);
                bool take = true;
                if (ru != rv) {
                    for (int w = lane; w < node_words; w += 64) trial[w] = reach[w];
                    wave_sync();
                    const uint32_t other = ru ? v : u;
                    if (lane == 0) trial[other >> 5] |= 1u << (other & 31);
                    wave_sync();
                    const uint64_t with_i = usable | (lane == owner ? (1ull << k) : 0ull);
                    take = !grow(trial, with_i, s_edges, sink, ws.parent, false);
                    if (take) {
                        uint32_t* t = reach;
                        reach = trial;
                        trial = t;
                    }
                }
                if (take && lane == owner) usable |= 1ull << k;
            }
        } else if (source != sink) {
            trace_path(ws, edge_words, s_edges, n_nodes, n_edges, source, sink);
            for (int i = 0; i < n_edges; ++i) {
                const int owner = i & 63, k = i >> 6;
                const uint64_t mine_bits = __shfl(usable, owner);
                if (!((mine_bits >> k) & 1u)) continue;  // unusable: walks to 0
                bool take = true;
                if (bit(ws.path, static_cast<uint32_t>(i))) {
                    const uint64_t without_i = usable & ~(lane == owner ? (1ull << k) : 0ull);
                    fill(ws.trial, node_words, 0u);
                    wave_sync();
                    if (lane == 0) ws.trial[source >> 5] |= 1u << (source & 31);
                    wave_sync();
                    take = grow(ws.trial, without_i, s_edges, sink, ws.parent, true);
                    if (take) trace_path(ws, edge_words, s_edges, n_nodes, n_edges, source, sink);
                }
                if (take && lane == owner) usable &= ~(1ull << k);
            }
        } else {
            usable = 0;  // s = t: every state survives; the minimal one is all zero
        }

        const uint8_t hi = static_cast<uint8_t>(survival ? level : K - 1);
        const uint8_t lo = static_cast<uint8_t>(survival ? 0 : level - 1);
        uint8_t* out = rows + j * static_cast<int64_t>(n_edges);
        for (int k = 0; k < rounds; ++k) {
            const int e = lane + 64 * k;
            if (e < n_edges) out[e] = ((usable >> k) & 1u) ? hi : lo;
        }
        if (lane == 0) side[j] = survival ? 1 : 0;
        wave_sync();
    }
}

// Global connectivity (edges work at state >= 1; target S >= level, level 1
// or 2): the same walk, with the system function evaluated from scratch at
// every decisive step (a search from node 0, plus the bridge test for level
// 2).  The one shortcut: for level 1 a survival state keeps the spanning tree
// of its last search, and removing an edge outside that tree cannot
// disconnect it.
__global__ __launch_bounds__(kBoundaryBlock) void k_boundary_global(
    const uint32_t* __restrict__ xs, int64_t N, const uint32_t* __restrict__ edges, int n_edges,
    int n_nodes, int K, int level, const int64_t* __restrict__ pick, int64_t n_pick,
    uint8_t* __restrict__ rows, uint8_t* __restrict__ side) {
    extern __shared__ uint32_t lds[];
    const int per_wave = graph::global_words(n_nodes, n_edges);
    uint32_t* s_edges = lds;
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const graph::GlobalSets g = graph::global_sets(lds + n_edges + wave * per_wave, n_nodes, n_edges);

    for (int e = threadIdx.x; e < n_edges; e += kBoundaryBlock) s_edges[e] = edges[e];
    __syncthreads();

    const int rounds = (n_edges + 63) >> 6;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBoundaryWaves;
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * kBoundaryWaves + wave; j < n_pick;
         j += stride) {
        const int64_t h = pick[j];
        if (h < 0 || h >= N) {  // not a sample index: reported, nothing read
            if (lane == 0) side[j] = 0xFF;
            continue;
        }
        uint64_t usable = 0;  // plane 0 = [x >= 1]
        for (int k = 0; k < rounds; ++k) {
            const int e = lane + 64 * k;
            if (e < n_edges) {
                const uint32_t word = xs[static_cast<int64_t>(e >> 5) * N + h];
                usable |= static_cast<uint64_t>((word >> (e & 31)) & 1u) << k;
            }
        }
        // At level 1 the parents of a spanning tree of the usable edges are
        // kept while the state survives.
        const bool tree_mode = level == 1;
        const bool survival =
            graph::global_at_least(usable, level, s_edges, n_edges, n_nodes, g, tree_mode);
        for (int i = 0; i < n_edges; ++i) {
            const int owner = i & 63, k = i >> 6;
            const bool ui = (__shfl(usable, owner) >> k) & 1u;
            if (ui == !survival) continue;  // walks to K-1 (failure) or 0 (survival) unopposed
            const uint64_t flip = lane == owner ? (1ull << k) : 0ull;
            const uint64_t trial = survival ? (usable & ~flip) : (usable | flip);
            bool take;
            if (survival && tree_mode) {
                const uint32_t uv = s_edges[i];
                if (g.parent[uv & 0xFFFFu] != i && g.parent[uv >> 16] != i) {
                    take = true;  // not a tree edge: the tree still spans every node
                } else {
                    take = graph::global_at_least(trial, 1, s_edges, n_edges, n_nodes, g, true);
                    if (!take)  // restore the tree of the current edges
                        graph::global_at_least(usable, 1, s_edges, n_edges, n_nodes, g, true);
                }
            } else {
                const bool after = graph::global_at_least(trial, level, s_edges, n_edges, n_nodes, g);
                take = survival ? after : !after;
            }
            if (take) usable = trial;
        }
        const uint8_t hi = static_cast<uint8_t>(survival ? 1 : K - 1);
        uint8_t* out = rows + j * static_cast<int64_t>(n_edges);
        for (int k = 0; k < rounds; ++k) {
            const int e = lane + 64 * k;
            if (e < n_edges) out[e] = ((usable >> k) & 1u) ? hi : 0;
        }
        if (lane == 0) side[j] = survival ? 1 : 0;
        wave_sync();
    }
}

}  // namespace

size_t boundary_lds_bytes(const rsr_system* sys) {
    if (sys->kind == RSR_SYS_MAX_FLOW) return flow_lds_bytes(sys);
    const int n_nodes = sys->n_nodes, n_edges = sys->n_edges;
    size_t per_wave;
    if (sys->kind == RSR_SYS_GLOBAL_CONNECTIVITY) {
        per_wave = static_cast<size_t>(((n_nodes + 31) >> 5) + ((n_edges + 31) >> 5) +
                                       2 * ((n_nodes + 1) >> 1));
    } else {
        const int node_words = (n_nodes + 31) >> 5;
        const int edge_words = (n_edges + 31) >> 5;
        const int parent_words = (n_nodes + 1) >> 1;
        per_wave = static_cast<size_t>(2 * node_words + edge_words + parent_words);
    }
    return sizeof(uint32_t) * (static_cast<size_t>(n_edges) + kBoundaryWaves * per_wave);
}

hipError_t launch_boundary(hipStream_t st, const rsr_system* sys, const uint32_t* xs, int64_t N,
                           const int64_t* d_pick, int64_t n_pick, uint8_t* d_rows,
                           uint8_t* d_side, int grid_cap) {
    int64_t blocks = (n_pick + kBoundaryWaves - 1) / kBoundaryWaves;
    if (blocks > grid_cap) blocks = grid_cap;
    if (blocks < 1) blocks = 1;
    if (sys->kind == RSR_SYS_MAX_FLOW)
        return launch_boundary_flow(st, sys, xs, N, d_pick, n_pick, d_rows, d_side, grid_cap);
    const size_t lds = boundary_lds_bytes(sys);
    if (sys->kind == RSR_SYS_GLOBAL_CONNECTIVITY)
        hipLaunchKernelGGL(k_boundary_global, dim3(static_cast<unsigned>(blocks)),
                           dim3(kBoundaryBlock), lds, st, xs, N, sys->d_edges, sys->n_edges,
                           sys->n_nodes, sys->K, sys->level, d_pick, n_pick, d_rows, d_side);
    else
        hipLaunchKernelGGL(k_boundary, dim3(static_cast<unsigned>(blocks)), dim3(kBoundaryBlock),
                           lds, st, xs, N, plane_words(sys->n_edges), sys->d_edges, sys->n_edges,
                           sys->n_nodes, sys->source, sys->sink, sys->K, sys->level, d_pick,
                           n_pick, d_rows, d_side);
    return hipGetLastError();
}

}  // namespace rsr
