// Wave-level graph searches over one sample's usable edges, shared by the
// system-function evaluation and the boundary search.  One wavefront works on
// one sample: lane l owns edges l, l+64, ... and holds their usability as bit
// k of a 64-bit mask (edge l + 64 k); node sets are bit arrays in the wave's
// LDS.  A sweep marks the unmarked end of every usable edge with exactly one
// marked end; all lanes read the marks before any lane writes in the same
// step, so a node's recorded parent edge and depth always refer to a node
// marked in an earlier step, and the parent chain of every marked node ends at
// the start node.
#pragma once

#include "rsr_internal.h"

namespace rsr {
namespace graph {

constexpr uint16_t kNoParent = 0xFFFFu;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t bit(const uint32_t* set, uint32_t i) {
    return (__hip_atomic_load(&set[i >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) >>
            (i & 31)) & 1u;
}

__device__ __forceinline__ void fill(uint32_t* set, int words, uint32_t value) {
    for (int w = threadIdx.x & 63; w < words; w += 64) set[w] = value;
}

__device__ __forceinline__ uint32_t other_end(uint32_t uv, uint32_t w) {
    const uint32_t u = uv & 0xFFFFu, v = uv >> 16;
    return u == w ? v : u;
}

// Grows `set` over the usable edges until nothing changes or `stop` (a node,
// or -1 for none) is marked; returns whether `stop` is marked.  With parent
// (and depth) not null, records the marking edge (and depth) of every newly
// marked node.
__device__ inline bool grow(uint32_t* set, uint64_t usable, const uint32_t* __restrict__ s_edges,
                            int stop, uint16_t* parent, uint16_t* depth) {
    const int lane = threadIdx.x & 63;
    while (true) {
        bool changed = false;
        uint64_t todo = usable;
        while (todo) {
            const int k = __ffsll(static_cast<unsigned long long>(todo)) - 1;
            todo &= todo - 1;
            const int e = lane + 64 * k;
            const uint32_t uv = s_edges[e];
            const uint32_t u = uv & 0xFFFFu, v = uv >> 16;
            const uint32_t ru = bit(set, u), rv = bit(set, v);
            if (ru != rv) {
                const uint32_t w = ru ? v : u;
                if (parent) parent[w] = static_cast<uint16_t>(e);
                if (depth) depth[w] = static_cast<uint16_t>(depth[ru ? u : v] + 1);
                atomicOr(&set[w >> 5], 1u << (w & 31));
                changed = true;
            }
        }
        wave_sync();
        if (stop >= 0 && __builtin_amdgcn_readfirstlane(static_cast<int>(bit(set, stop)))) return true;
        if (!__any(changed)) return false;
    }
}

// Number of set bits in the first `words` words of `set` (wave-uniform).
__device__ inline int count(const uint32_t* set, int words) {
    int c = 0;
    for (int w = threadIdx.x & 63; w < words; w += 64) c += __popc(set[w]);
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    return c;
}

// Per-wave LDS working set of the global-connectivity test.
struct GlobalSets {
    uint32_t* reach;    // [node_words]
    uint32_t* covered;  // [edge_words]
    uint16_t* parent;   // [n_nodes]
    uint16_t* depth;    // [n_nodes]
};

__device__ __forceinline__ int global_words(int n_nodes, int n_edges) {
    // reach + covered + parent and depth as 16-bit pairs
    return ((n_nodes + 31) >> 5) + ((n_edges + 31) >> 5) + 2 * ((n_nodes + 1) >> 1);
}

__device__ __forceinline__ GlobalSets global_sets(uint32_t* base, int n_nodes, int n_edges) {
    const int node_words = (n_nodes + 31) >> 5, edge_words = (n_edges + 31) >> 5;
    const int half_words = (n_nodes + 1) >> 1;
    GlobalSets g;
    g.reach = base;
    g.covered = base + node_words;
    g.parent = reinterpret_cast<uint16_t*>(base + node_words + edge_words);
    g.depth = reinterpret_cast<uint16_t*>(base + node_words + edge_words + half_words);
    return g;
}

// Global connectivity of the usable edges: S >= 1 when every node is reached
// from node 0; S >= 2 when, in addition, no usable edge is a bridge.  A
// spanning tree comes from the search (parents and depths); every usable
// non-tree edge (u, v) closes a cycle with the tree path from u to v, and the
// tree edges on no such cycle are exactly the bridges.  Wave-uniform result.
// With keep_tree, the parents of the spanning tree are recorded at level 1
// too (they are always recorded at level 2).
__device__ inline bool global_at_least(uint64_t usable, int level,
                                       const uint32_t* __restrict__ s_edges, int n_edges,
                                       int n_nodes, const GlobalSets& g, bool keep_tree = false) {
    const int lane = threadIdx.x & 63;
    const int node_words = (n_nodes + 31) >> 5, edge_words = (n_edges + 31) >> 5;
    fill(g.reach, node_words, 0u);
    wave_sync();
    if (lane == 0) {
        g.reach[0] = 1u;
        g.parent[0] = kNoParent;
        g.depth[0] = 0;
    }
    wave_sync();
    const bool tree = level >= 2 || keep_tree;
    grow(g.reach, usable, s_edges, -1, tree ? g.parent : nullptr, tree ? g.depth : nullptr);
    if (count(g.reach, node_words) < n_nodes) return false;
    if (level < 2) return true;
    fill(g.covered, edge_words, 0u);
    wave_sync();
    uint64_t todo = usable;
    while (todo) {
        const int k = __ffsll(static_cast<unsigned long long>(todo)) - 1;
        todo &= todo - 1;
        const int e = lane + 64 * k;
        const uint32_t uv = s_edges[e];
        uint32_t a = uv & 0xFFFFu, b = uv >> 16;
        if (g.parent[a] == e || g.parent[b] == e) continue;  // a tree edge
        // Walk both ends up to their lowest common ancestor.
        for (int steps = 0; a != b && steps < 2 * n_nodes; ++steps) {
            if (g.depth[a] < g.depth[b]) {
                const uint32_t t = a;
                a = b;
                b = t;
            }
            const uint32_t pe = g.parent[a];
            if (pe >= static_cast<uint32_t>(n_edges)) break;  // only the root has none
            atomicOr(&g.covered[pe >> 5], 1u << (pe & 31));
            a = other_end(s_edges[pe], a);
        }
    }
    wave_sync();
    bool bridge = false;
    for (int v = lane + 1; v < n_nodes; v += 64) bridge = bridge || !bit(g.covered, g.parent[v]);
    return !__any(bridge);
}

}  // namespace graph
}  // namespace rsr
