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
constexpr int kMaxMfmaSteps = 20;   // int8 form: 64 k per step, 1280 bits
constexpr int kMaxMfma4Steps = 10;  // FP4 form: 128 k per step, 1280 bits

// Every device and pinned-host allocation of the library goes through these
// two, so that rsr_debug_fail_alloc can make a chosen one fail.
hipError_t dev_malloc(void** p, size_t bytes);
hipError_t host_malloc(void** p, size_t bytes);
template <class T>
inline hipError_t dev_malloc(T** p, size_t bytes) {
    return dev_malloc(reinterpret_cast<void**>(p), bytes);
}
template <class T>
inline hipError_t host_malloc(T** p, size_t bytes) {
    return host_malloc(reinterpret_cast<void**>(p), bytes);
}

// Staging of a host-callback system function (rsr_callback.hip): gathered
// sample words and system-function results on the device and in pinned host
// memory, grown on demand.
struct CallbackStage {
    uint32_t* d_words = nullptr;  // [count][W] sample-major
    uint32_t* h_words = nullptr;  // pinned copy
    int64_t words_cap = 0;
    uint8_t* d_bytes = nullptr;   // [count] results / [count][n] rows
    uint8_t* h_bytes = nullptr;   // pinned copy
    int64_t bytes_cap = 0;
    int64_t* h_index = nullptr;   // pinned [count] picks
    int64_t index_cap = 0;
};

struct Workspace {
    uint64_t* counters = nullptr;      // 16 u64 device counters
    uint64_t* count_part = nullptr;    // [kMaxReduceBlocks][8] u64 partial counts
    int32_t* list = nullptr;           // unknown-sample index list
    int64_t list_cap = 0;
    uint32_t* grad_part = nullptr;     // [RSR_MAX_BITS * kMaxGradBlocks + kMaxGradBlocks] u32
    uint64_t* host_counts = nullptr;   // pinned, 16 u64
    uint64_t* host_counts_dev = nullptr;  // the device address of host_counts
    uint64_t estimate_seq = 0;         // last sequence number of rsr_estimate's counts
    uint64_t* casc_counters = nullptr; // [16] per-round cascade counters
    uint32_t* casc_words = nullptr;    // 2 x [W][N] u32 (cascade)
    int32_t* casc_index = nullptr;     // 2 x [N] i32 indices, then 2 x [N] u32 match words
    int64_t casc_words_cap = 0, casc_index_cap = 0;
    uint32_t* casc_state = nullptr;    // persistent cascade state (counts, items, barrier, tickets)
    int64_t casc_state_cap = 0;        // in u32 words
    CallbackStage cb;
};

}  // namespace rsr

struct rsr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    rsr::Workspace ws;
    int cu_count = 0;
    std::string arch;  // gcnArchName of the device
    void* noalloc_scratch = nullptr;  // this device's address of rsr_noalloc.hip's scratch
};

struct rsr_model {
    rsr_ctx* ctx = nullptr;
    int n = 0, K = 0;
    // One device allocation holds the four arrays below, one pinned host
    // buffer of the same layout stages their updates.
    void* d_mem = nullptr;
    void* h_stage = nullptr;
    size_t mem_bytes = 0;
    hipEvent_t staged = nullptr;   // recorded after the last staged upload
    uint64_t* d_thresh = nullptr;  // [n][K-1]
    double* d_p64 = nullptr;       // [n][K] the probabilities as given
    // Sampler form of the thresholds, [ceil(n/8)*8][K-1] pairs (gt, eq) of
    // int32 on the high 16 bits of the uniform word u: u >= C is decided true
    // by (u >> 16) > gt, and needs the low half only when (u >> 16) == eq.
    // Padding components never set a bit (gt = INT32_MAX, eq = -1).
    int32_t* d_half = nullptr;
    float* d_p = nullptr;          // [n][K] fp32 copy of the probabilities
};

struct rsr_refs {
    rsr_ctx* ctx = nullptr;
    int n = 0, K = 0, W = 0, WR = 0;  // WR = packed row stride in words
    int64_t R_L = 0, R_U = 0;
    bool consistent = false;            // no upper row lies below a lower row
    uint32_t* d_lower_nbits = nullptr;  // [R_L][WR]: NOT t(r), pad bits 0
    uint32_t* d_upper_bits = nullptr;   // [R_U][WR]: t(r)
    // Matrix-core operands (k_dom_mfma.hip); absent when KS > kMaxMfmaSteps.
    int KS = 0;                          // 64-wide k-steps: ceil(32 W / 64)
    int TL = 0, TU = 0;                  // 16-row tiles per side
    int8_t* d_lower_frag = nullptr;      // [TL][KS][64 lanes][16]: NOT t(r) as 0/1 bytes
    int32_t* d_lower_cinit = nullptr;    // [TL * 16]: -1 (row) or 0 (pad row)
    int8_t* d_upper_frag = nullptr;      // [TU][KS][64][16]: -t(r) as 0/-1 bytes
    int32_t* d_upper_cinit = nullptr;    // [TU * 16]: |t(r)| - 1 (row) or 0 (pad row)
    // FP4 form: 128-wide k-steps, nibbles 0x2 (+1) / 0xA (-1), float starts.
    int KS4 = 0;                          // ceil(32 W / 128)
    int8_t* d_lower_frag4 = nullptr;      // [TL][KS4][64][16]: NOT t(r) as +1 nibbles
    float* d_lower_cinit4 = nullptr;      // [TL * 16]: -0.5 (row) or +0.5 (pad row)
    int8_t* d_upper_frag4 = nullptr;      // [TU][KS4][64][16]: t(r) as -1 nibbles
    float* d_upper_cinit4 = nullptr;      // [TU * 16]: |t(r)| - 0.5 (row) or +0.5 (pad row)
    // FP4 form on 32-row tiles (k_dom_fp4x32): KS steps of 64 k; lane l of a
    // step holds row l % 32, packed word 2 s + l / 32 as +1 nibbles (NOT
    // t(r) for lower rows, t(r) for upper rows); ceil(R / 32) tiles per side.
    int8_t* d_lower_frag32 = nullptr;     // [ceil(R_L/32)][KS][64][16]
    int8_t* d_upper_frag32 = nullptr;     // [ceil(R_U/32)][KS][64][16]
};

struct rsr_system {
    rsr_ctx* ctx = nullptr;
    int kind = RSR_SYS_ST_CONNECTIVITY;
    int n_nodes = 0, n_edges = 0, K = 0, level = 0, source = 0, sink = 0;
    uint32_t* d_edges = nullptr;  // [n_edges] packed (u | v << 16); graph systems only
    // RSR_SYS_HOST_CALLBACK: the system state of a state vector, on the host.
    int32_t (*phi)(const uint8_t* x, int32_t n, void* user) = nullptr;
    void* user = nullptr;
};

namespace rsr {

// Device-side record of one job of a batched plan.
struct JobDev {
    const uint64_t* thresh;  // [n][K-1]
    const int32_t* half;     // rsr_model::d_half
    const float* p;          // [n][K]
    uint32_t* samples;       // [W][N]
    uint8_t* flags;          // [N]
    uint8_t* Y;              // [N]
    float* G;                // [n][K] or nullptr
    int64_t N;
    uint64_t seed;
    uint32_t stream_id;
    int32_t n, K;
    int64_t g_off;           // offset of this job's gradient in a plan's gather buffer
};

// Where a kernel finds its samples: one job (jobs == nullptr: samples / N /
// flags / Y), or the jobs of a plan segment, addressed by a global index g in
// [0, total) with offsets[j] = first g of job j.
struct SegSrc {
    const uint32_t* samples;
    int64_t N;
    uint8_t* flags;
    uint8_t* Y;
    const JobDev* jobs;
    const int64_t* offsets;  // [n_jobs + 1]
    int32_t n_jobs;
    int64_t total;
};

inline SegSrc single_src(const uint32_t* samples, int64_t N, uint8_t* flags, uint8_t* Y) {
    SegSrc s{};
    s.samples = samples;
    s.N = N;
    s.flags = flags;
    s.Y = Y;
    s.total = N;
    return s;
}

#ifdef __HIPCC__
// Job j and sample h of global index g (binary search over the job offsets).
__device__ __forceinline__ void seg_locate(const SegSrc& s, int64_t g, int& j, int64_t& h) {
    if (!s.jobs) {
        j = 0;
        h = g;
        return;
    }
    int lo = 0, hi = s.n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s.offsets[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    j = lo;
    h = g - s.offsets[lo];
}
__device__ __forceinline__ const uint32_t* seg_words(const SegSrc& s, int j, int64_t& stride) {
    if (!s.jobs) {
        stride = s.N;
        return s.samples;
    }
    stride = s.jobs[j].N;
    return s.jobs[j].samples;
}
__device__ __forceinline__ uint8_t* seg_flags(const SegSrc& s, int j) {
    return s.jobs ? s.jobs[j].flags : s.flags;
}
__device__ __forceinline__ uint8_t* seg_Y(const SegSrc& s, int j) {
    return s.jobs ? s.jobs[j].Y : s.Y;
}
#endif

// Ping-pong buffers of the LABEL-mode cascade (k_dom_cascade): compacted
// sample words [W][N] and original indices [N], plus one counter per round.
struct CascadeBuffers {
    static constexpr int kMaxRounds = 12;
    // Most output regions of the matrix-core round 0 (one per block).
    static constexpr int kMaxRegions = 2048;
    // u64 words of the counters allocation: 16 round counters, then
    // kMaxRegions u32 region counts.
    static constexpr int kCounterU64 = 16 + kMaxRegions / 2;
    uint32_t* words[2] = {nullptr, nullptr};  // [W][stride] each
    int32_t* index[2] = {nullptr, nullptr};   // [stride] each
    uint32_t* match[2] = {nullptr, nullptr};  // [stride] each: match bits of split rounds
    int64_t stride = 0;                       // capacity in samples (>= total)
    uint64_t* counters = nullptr;  // [kMaxRounds], zeroed before the first round
    uint32_t* regions = nullptr;   // [kMaxRegions] (k_casc_head)
};

// Round boundaries of the cascade: rows [0, first), [first, first*growth), ...
// Rounds of more than split_rows rows (after round 0) are split into
// rows / split_rows chunks taken by different waves.
struct CascadeShape {
    int first = 32;
    int growth = 5;
    int split_rows = 128;
    // Rounds after round 0 in the FP4 matrix-core form (needs refs->KS4 > 0).
    bool mfma_tail = false;
    // Round 0 in the FP4 32 x 32 form (k_casc_head) when first == 32 and
    // casc_head_supported(refs); otherwise on the vector ALU.
    bool mfma_head = false;
    // Most chunks of a split round (1..1024); 0 takes the built-in caps.
    int max_chunks = 0;
};

// Default shape with the matrix-core tail (measured on graph2: matrix-core
// rounds favour smaller first rounds, faster growth and larger chunks).
inline CascadeShape mfma_tail_shape() {
    CascadeShape s;
    s.first = 16;
    s.growth = 6;
    s.split_rows = 256;
    s.mfma_tail = true;
    return s;
}

// Default shape with every round in the matrix-core form: round 0 is one
// 32-row tile per side.
inline CascadeShape mfma_head_shape() {
    CascadeShape s;
    s.first = 32;
    s.growth = 6;
    s.split_rows = 256;
    s.mfma_tail = true;
    s.mfma_head = true;
    return s;
}

// Shape with the matrix-core tail for many rows: growth 8 reaches the last
// row in fewer rounds, and larger chunks keep each split round's waves busy.
inline CascadeShape mfma_wide_shape() {
    CascadeShape s;
    s.first = 16;
    s.growth = 8;
    s.split_rows = 512;
    s.mfma_tail = true;
    return s;
}

// Rows per side from which the automatic LABEL form takes mfma_wide_shape
// (measured on MI355X on the three-state levels of graph2 and on 4.4e4 to 2e5
// reference rows: 0.79 to 0.99 of the persistent cascade's time and 0.80 to
// 0.96 of mfma_tail_shape's; on graph2's 1e4 rows per side mfma_tail_shape is
// the faster by 18%).
constexpr int64_t kWideRows = 16384;

// Largest refs->KS (64-wide k-steps) of the matrix-core round 0.
constexpr int kMaxHeadSteps = 10;

// Kernel launchers (each returns the hipError_t of the launch).
hipError_t launch_sample(hipStream_t st, const rsr_model* m, uint64_t seed, uint32_t stream_id,
                         uint64_t first, int64_t N, uint32_t* d_samples);
hipError_t launch_dom_bits(hipStream_t st, const rsr_refs* refs, const uint32_t* d_samples,
                           int64_t N, int mode, uint8_t* d_flags, uint32_t* d_match);
hipError_t launch_dom_cascade(hipStream_t st, const rsr_refs* refs, const SegSrc& seg,
                              const CascadeBuffers& cb, const CascadeShape& shape, int grid_cap);
// `cus` (the device's CU count) picks the sample tiles per wave for the grid.
hipError_t launch_dom_mfma(hipStream_t st, const rsr_refs* refs, const uint32_t* d_samples,
                           int64_t N, int mode, bool fp4, int cus, uint8_t* d_flags,
                           uint32_t* d_match);
// A whole cascade round (test, flags, compaction) in the FP4 matrix-core form
// (k_dom_mfma.hip); src_count null means host_count samples.
hipError_t launch_casc_mfma_round(hipStream_t st, const rsr_refs* refs, const SegSrc& seg,
                                  const uint32_t* csrc, int64_t cstride, const int32_t* src_idx,
                                  const unsigned long long* src_count, int64_t host_count,
                                  int64_t max_count, int l0, int l1, int u0, int u1, int grid_cap,
                                  uint32_t* dst, int32_t* dst_idx, uint32_t* dst_match,
                                  int64_t dst_stride, unsigned long long* dst_count, int last);
// Split-round test of the cascade in the FP4 matrix-core form (k_dom_mfma.hip).
hipError_t launch_casc_mfma(hipStream_t st, const rsr_refs* refs, const uint32_t* csrc,
                            int64_t cstride, const unsigned long long* src_count, int64_t max_count,
                            int l0, int l1, int u0, int u1, int chunks, int grid_cap,
                            uint32_t* match);
// The persistent LABEL cascade (k_cascade_persist.hip): a popcount round-0
// launch, then the FP4 32 x 32 rounds in one cooperative launch.  cb.stride
// is at least casc_persist_stride(refs, seg.total, cus); d_state holds
// casc_persist_state_words(cb.stride, refs->KS) u32, zero on entry (left
// nonzero); *d_err becomes 1 if a grid barrier timed out.
hipError_t launch_casc_persist(hipStream_t st, const rsr_refs* refs, const SegSrc& seg,
                               const CascadeBuffers& cb, const CascadeShape& shape,
                               unsigned* d_state, unsigned long long* d_err, int cus);
int64_t casc_persist_state_words(int64_t stride, int KS);
// Compact-buffer capacity (cb.stride) the persistent cascade needs for N
// samples: N plus the slack of its per-block output regions.
int64_t casc_persist_stride(const rsr_refs* refs, int64_t N, int cus);
// Whether the persistent cascade is built for the handle's width.
bool casc_persist_supported(const rsr_refs* refs);
// Time limit of the persistent cascade's grid barriers (ticks of the 100 MHz
// real-time counter; < 0: the default, 10 s).
void set_barrier_timeout(int64_t ticks);
// Round 0 of the cascade in the FP4 32 x 32 form (k_casc_head.hip): rows
// [0, 32) of both sides over all samples of seg; flags the decided samples
// (all samples when last) and packs the others into cb.words[0] / index[0] /
// match[0], their number in cb.counters[0] (through regions of cb.words[1]).
bool casc_head_supported(const rsr_refs* refs);
hipError_t launch_casc_head(hipStream_t st, const rsr_refs* refs, const SegSrc& seg,
                            const CascadeBuffers& cb, int last);
hipError_t launch_label(hipStream_t st, const SegSrc& seg, int32_t* d_list, uint64_t* d_counter,
                        int grid_cap);
hipError_t launch_bfs(hipStream_t st, const rsr_system* sys, const SegSrc& seg,
                      const int32_t* d_list, const uint64_t* d_count, int which,
                      uint64_t* d_n_evaluated, int grid_blocks);
hipError_t launch_fill_u64(hipStream_t st, uint64_t* p, int64_t count, uint64_t value);
size_t boundary_lds_bytes(const rsr_system* sys);
size_t flow_lds_bytes(const rsr_system* sys);
hipError_t launch_flow_eval(hipStream_t st, const rsr_system* sys, const SegSrc& seg,
                            const int32_t* d_list, const uint64_t* d_count, int which,
                            uint64_t* d_n_evaluated, int grid_blocks);
hipError_t launch_boundary_flow(hipStream_t st, const rsr_system* sys, const uint32_t* xs,
                                int64_t N, const int64_t* d_pick, int64_t n_pick, uint8_t* d_rows,
                                uint8_t* d_side, int grid_cap);
// rsr_refs_create; without matrix_operands the MFMA fragments are not built
// (the handle then serves the popcount and cascade forms only).
rsr_status refs_create(rsr_ctx* ctx, int32_t n, int32_t K, const uint8_t* lower, int64_t R_L,
                       const uint8_t* upper, int64_t R_U, bool matrix_operands, rsr_refs** out);
// First B unclassified samples in index order -> d_pick; *d_total = all of
// them.  d_part: at least 1024 u64 of scratch.
hipError_t launch_pick(hipStream_t st, const uint8_t* d_flags, int64_t N, int64_t B,
                       int64_t* d_pick, uint64_t* d_part, uint64_t* d_total);
hipError_t launch_boundary(hipStream_t st, const rsr_system* sys, const uint32_t* xs, int64_t N,
                           const int64_t* d_pick, int64_t n_pick, uint8_t* d_rows,
                           uint8_t* d_side, int grid_cap);
// With a job table (jobs != nullptr) the reductions run once per job in one
// launch; N must then be the largest job size (it sizes the grid), counters
// receive [n_jobs][8] and the gradient partials need n_jobs * (W * bx * 32 +
// bx) u32 with bx = grad_blocks(N).
hipError_t launch_counts(hipStream_t st, const uint8_t* d_flags, const uint8_t* d_Y, int64_t N,
                         uint64_t* d_counters, uint64_t* d_partial, const JobDev* jobs = nullptr,
                         int n_jobs = 1);
// One job's counts in one launch (flags and Y 16-byte aligned); d_ticket is a
// zero-initialised u32 the kernel leaves at zero.
// out[0..4] = n_L, n_U, n_u, n_both, n_u_up and out[5] = *d_carry (0 when
// d_carry is NULL); out may be pinned host memory (its device address).  A
// nonzero seq is stored into out[6] after them (system-scope release).
hipError_t launch_counts_vec(hipStream_t st, const uint8_t* d_flags, const uint8_t* d_Y, int64_t N,
                             uint64_t* out, uint64_t* d_partial, uint32_t* d_ticket,
                             const uint64_t* d_carry, uint64_t seq);
int64_t grad_blocks(int64_t N);
hipError_t launch_grad(hipStream_t st, int n, int K, const float* d_p, const uint32_t* d_samples,
                       const uint8_t* d_Y, int64_t N, uint32_t* d_partial, float* d_G,
                       uint64_t* d_counts, const JobDev* jobs = nullptr, int n_jobs = 1);
hipError_t launch_gather_G(hipStream_t st, const JobDev* jobs, int n_jobs, int nK, float* out);
// Binary Birnbaum importance I[i] = c1 / (N p1) - c0 / (N p0), fp64 then
// rounded to fp32 (k_reduce.hip); d_partial as for launch_grad.
hipError_t launch_importance(hipStream_t st, int n, const double* d_p64, const uint32_t* d_samples,
                             const uint8_t* d_Y, int64_t N, uint32_t* d_partial, float* d_I);

// Scratch of rsr_eval_unknown_noalloc (rsr_noalloc.hip): a file-scope device
// array holding a counter and a list of up to kNoAllocMaxSamples indices.
constexpr int64_t kNoAllocMaxSamples = int64_t{1} << 22;
constexpr int RSR_MAX_DEVICES = 64;
// This device's address of the array, looked up once per device.
hipError_t noalloc_scratch(int device, void** out);

// Error recording shared by the translation units of the ABI.
inline rsr_status set_error(rsr_ctx* ctx, rsr_status st, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return st;
}
inline rsr_status hip_error(rsr_ctx* ctx, hipError_t e, const char* what) {
    return set_error(ctx, e == hipErrorOutOfMemory ? RSR_ENOMEM : RSR_EHIP,
                     std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
}
// Grows the context's unknown-sample list to at least N entries.
rsr_status ensure_list(rsr_ctx* ctx, int64_t N);
// Host-callback system function (rsr_callback.hip): Stage-2 evaluation and
// the componentwise boundary search with Phi evaluated on the host.
rsr_status eval_callback(rsr_ctx* ctx, const rsr_system* sys, const uint32_t* d_samples, int64_t N,
                         const uint8_t* d_flags, int which, uint8_t* d_Y, uint64_t* d_n_evaluated);
rsr_status boundary_callback(rsr_ctx* ctx, const rsr_system* sys, const uint32_t* d_samples,
                             int64_t N, const int64_t* d_pick, int64_t n_pick, uint8_t* d_rows,
                             uint8_t* d_side);
hipError_t launch_sample_jobs(hipStream_t st, int n, int K, const JobDev* jobs,
                              const int64_t* offsets, int n_jobs, int64_t total, int grid_cap);
hipError_t launch_copy_u64(hipStream_t st, const uint64_t* src, uint64_t* dst, int count);

}  // namespace rsr
