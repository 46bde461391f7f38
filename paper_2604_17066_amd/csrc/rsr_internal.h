// Internal declarations shared by the runtime (rsr_api.hip) and the kernel
// translation units.  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/rsr.h"

namespace rsr {

// Packed width helpers (layout documented in rsr.h).
inline int plane_words(int n) { return (n + 31) / 32; }
inline int sample_words(int n, int K) { return (K - 1) * plane_words(n); }

// Row stride of packed reference rows: the word count of the classification
// kernel instantiated for W words (>= W; pad words are zero).
int dom_row_words(int W);

// Reduction shapes (k_reduce.hip): at most this many blocks write partials.
constexpr int kMaxReduceBlocks = 1024;
constexpr int kMaxGradBlocks = 64;
// Largest k-step count of the matrix-core form (n (K-1) <= 1280 bits).
constexpr int kMaxMfmaSteps = 20;

struct Workspace {
    uint64_t* counters = nullptr;      // 16 u64 device counters
    uint64_t* count_part = nullptr;    // [kMaxReduceBlocks][8] u64 partial counts
    int32_t* list = nullptr;           // unknown-sample index list
    int64_t list_cap = 0;
    uint32_t* grad_part = nullptr;     // [RSR_MAX_BITS * kMaxGradBlocks + kMaxGradBlocks] u32
    uint64_t* host_counts = nullptr;   // pinned, 16 u64
};

}  // namespace rsr

struct rsr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    rsr::Workspace ws;
    int cu_count = 0;
};

struct rsr_model {
    rsr_ctx* ctx = nullptr;
    int n = 0, K = 0;
    uint64_t* d_thresh = nullptr;  // [n][K-1]
    float* d_p = nullptr;          // [n][K] fp32 copy of the probabilities
};

struct rsr_refs {
    rsr_ctx* ctx = nullptr;
    int n = 0, K = 0, W = 0, WR = 0;  // WR = packed row stride in words
    int64_t R_L = 0, R_U = 0;
    uint32_t* d_lower_nbits = nullptr;  // [R_L][WR]: NOT t(r), pad bits 0
    uint32_t* d_upper_bits = nullptr;   // [R_U][WR]: t(r)
    // Matrix-core operands (k_dom_mfma.hip); absent when KS > kMaxMfmaSteps.
    int KS = 0;                          // 64-wide k-steps: ceil(32 W / 64)
    int TL = 0, TU = 0;                  // 16-row tiles per side
    int8_t* d_lower_frag = nullptr;      // [TL][KS][64 lanes][16]: NOT t(r) as 0/1 bytes
    int32_t* d_lower_cinit = nullptr;    // [TL * 16]: 0 (row) or 1 (pad row)
    int8_t* d_upper_frag = nullptr;      // [TU][KS][64][16]: t(r) as 0/1 bytes
    int32_t* d_upper_cinit = nullptr;    // [TU * 16]: -|t(r)| (row) or 1 (pad row)
};

struct rsr_system {
    rsr_ctx* ctx = nullptr;
    int n_nodes = 0, n_edges = 0, K = 0, level = 0, source = 0, sink = 0;
    uint32_t* d_edges = nullptr;  // [n_edges] packed (u | v << 16)
};

namespace rsr {

// Kernel launchers (each returns the hipError_t of the launch).
hipError_t launch_sample(hipStream_t st, const rsr_model* m, uint64_t seed, uint32_t stream_id,
                         uint64_t first, int64_t N, uint32_t* d_samples);
hipError_t launch_dom_bits(hipStream_t st, const rsr_refs* refs, const uint32_t* d_samples,
                           int64_t N, int mode, uint8_t* d_flags, uint32_t* d_match);
hipError_t launch_dom_mfma(hipStream_t st, const rsr_refs* refs, const uint32_t* d_samples,
                           int64_t N, int mode, uint8_t* d_flags, uint32_t* d_match);
hipError_t launch_label(hipStream_t st, const uint8_t* d_flags, int64_t N, int which,
                        uint8_t* d_Y, int32_t* d_list, uint64_t* d_counter);
hipError_t launch_bfs(hipStream_t st, const rsr_system* sys, const uint32_t* d_samples,
                      int64_t N, const int32_t* d_list, const uint64_t* d_count, int which,
                      uint8_t* d_Y, uint64_t* d_n_evaluated, int grid_blocks);
hipError_t launch_fill_u64(hipStream_t st, uint64_t* p, int64_t count, uint64_t value);
hipError_t launch_counts(hipStream_t st, const uint8_t* d_flags, const uint8_t* d_Y, int64_t N,
                         uint64_t* d_counters, uint64_t* d_partial);
hipError_t launch_grad(hipStream_t st, const rsr_model* m, const uint32_t* d_samples,
                       const uint8_t* d_Y, int64_t N, uint32_t* d_partial, float* d_G,
                       uint64_t* d_counts);
hipError_t launch_copy_u64(hipStream_t st, const uint64_t* src, uint64_t* dst, int count);

}  // namespace rsr
