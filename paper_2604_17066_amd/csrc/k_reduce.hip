// Reductions: estimator counts (section 3.3.1) and the score-function
// gradient counts.
//
// Blocks write partial sums to a workspace, which are added in a fixed order
// (integers: the results do not depend on scheduling either way).
//
// k_counts: one pass over flags (and Y) with per-thread counters, wavefront
// and block reductions, one partial row per block; k_counts_final adds rows.
// k_counts_vec: the same for one job in one launch, 16 flags per load; the
// last block to finish (one ticket atomic per block) adds the rows.
//
// k_grad_bits: a[j][i] = #{h : Y_h = 1 and x_{h,i} >= j} for every thermometer
// bit (plane j, component i).  Block column y = packed word w; each thread
// walks a strided run of samples (about 64), counts the 32 bit positions of
// its Y-masked words in bit-sliced form and then in 32 plain counters; the
// block reduces them to one partial row.  Blocks in column 0 also count
// #{Y = 1}.
// k_grad_finalize: c[i][s] = a[s][i] - a[s+1][i] (a[0][i] = #{Y = 1},
// a[K][i] = 0), G[i][s] = (float)c / ((float)N * p[i][s]).
#include "rsr_internal.h"

namespace rsr {
namespace {

constexpr int kBlock = 256;
// 16-flag chunks per thread of k_counts_vec: more blocks spread the pass over
// more CUs, fewer blocks take fewer same-address ticket atomics.
constexpr int kCountsChunks = 4;

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sum over the wave with DPP moves (no LDS round trips): shifts within each
// row of 16 lanes leave the row's sum in its lane 15, two row broadcasts carry
// it up, and lane 63 holds the total, which is read into a scalar.  Every
// lane of the wave must be active.
__device__ __forceinline__ uint32_t wave_sum32(uint32_t v) {
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x111, 0xF, 0xF, true));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x112, 0xF, 0xF, true));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x114, 0xF, 0xF, true));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x118, 0xF, 0xF, true));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x142, 0xA, 0xF, false));
    v += static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x143, 0xC, 0xF, false));
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 63));
}

__global__ __launch_bounds__(kBlock) void k_fill_u64(unsigned long long* p, int64_t count,
                                                     unsigned long long value) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (i < count) p[i] = value;
}

__global__ __launch_bounds__(kBlock) void k_counts(const uint8_t* __restrict__ flags,
                                                   const uint8_t* __restrict__ Y, int64_t N,
                                                   unsigned long long* __restrict__ partial,
                                                   const JobDev* __restrict__ jobs) {
    // partial[job][block][0..4] = this block's n_L, n_U, n_u, n_both, n_u_up;
    // with a job table, blockIdx.y selects the job.
    if (jobs) {
        const JobDev& jd = jobs[blockIdx.y];
        flags = jd.flags;
        Y = jd.Y;
        N = jd.N;
        partial += static_cast<int64_t>(blockIdx.y) * gridDim.x * 8;
    }
    uint32_t nL = 0, nU = 0, nu = 0, nb = 0, nuu = 0;
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
    __shared__ uint32_t red[kBlock / 64][5];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    nL = wave_sum32(nL);
    nU = wave_sum32(nU);
    nu = wave_sum32(nu);
    nb = wave_sum32(nb);
    nuu = wave_sum32(nuu);
    if (lane == 0) {
        red[wave][0] = nL;
        red[wave][1] = nU;
        red[wave][2] = nu;
        red[wave][3] = nb;
        red[wave][4] = nuu;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        unsigned long long s = 0;
        for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
        partial[static_cast<int64_t>(blockIdx.x) * 8 + threadIdx.x] = s;
    }
}

// Counts of flags in the SWAR form: four one-byte flags per 32-bit word (bit 0
// lower, bit 1 upper), and Y bytes reduced to bit 0 of each byte (nonzero).
__device__ __forceinline__ void count_word(uint32_t w, uint32_t y, uint32_t (&c)[5]) {
    const uint32_t lo = w & 0x01010101u, up = (w >> 1) & 0x01010101u;
    const uint32_t unk = ~(lo | up) & 0x01010101u;
    const uint32_t ynz = ((((y & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | y) >> 7) & 0x01010101u;
    c[0] += __popc(lo);
    c[1] += __popc(up & ~lo);
    c[2] += __popc(unk);
    c[3] += __popc(lo & up);
    c[4] += __popc(unk & ynz);
}

// The counts of k_counts for one job in one launch: 16 flags (and Y bytes)
// per 16-byte load (both arrays 16-byte aligned), per-block partials, and the
// last block to finish (a ticket counter, left at zero again) adds them into
// out[0..4] and copies *carry (0 when carry is NULL) into out[5].  out may be
// pinned host memory.  When seq is not 0 the last block then stores seq into
// out[6], ordered after out[0..5] at system scope, so that a host polling
// out[6] may read the counts before the kernel is seen to end.
__global__ __launch_bounds__(kBlock) void k_counts_vec(const uint8_t* __restrict__ flags,
                                                       const uint8_t* __restrict__ Y, int64_t N,
                                                       unsigned long long* __restrict__ partial,
                                                       unsigned long long* __restrict__ out,
                                                       unsigned int* __restrict__ ticket,
                                                       const unsigned long long* __restrict__ carry,
                                                       unsigned long long seq) {
    uint32_t c[5] = {0, 0, 0, 0, 0};
    const int64_t chunks = N >> 4;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; k < chunks;
         k += stride) {
        const uint4 f = reinterpret_cast<const uint4*>(flags)[k];
        const uint4 y = Y ? reinterpret_cast<const uint4*>(Y)[k] : make_uint4(0, 0, 0, 0);
        count_word(f.x, y.x, c);
        count_word(f.y, y.y, c);
        count_word(f.z, y.z, c);
        count_word(f.w, y.w, c);
    }
    if (blockIdx.x == 0)
        for (int64_t h = (chunks << 4) + threadIdx.x; h < N; h += kBlock) {
            const uint32_t f = flags[h];
            const uint32_t lo = f & 1u, up = (f >> 1) & 1u, unk = (lo | up) ^ 1u;
            c[0] += lo;
            c[1] += up & (lo ^ 1u);
            c[2] += unk;
            c[3] += lo & up;
            c[4] += (unk && Y && Y[h]) ? 1u : 0u;
        }
    __shared__ uint32_t red[kBlock / 64][5];
    __shared__ bool is_last;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const uint32_t v = wave_sum32(c[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        unsigned long long v = 0;
        for (int w = 0; w < kBlock / 64; ++w) v += red[w][threadIdx.x];
        partial[static_cast<int64_t>(blockIdx.x) * 8 + threadIdx.x] = v;
        // The writer itself makes its partial visible device-wide before the
        // ticket is taken.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int done = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL,
                                                         __HIP_MEMORY_SCOPE_AGENT);
        is_last = done == gridDim.x - 1;
    }
    __syncthreads();
    if (!is_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    unsigned long long v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < static_cast<int>(gridDim.x); b += kBlock)
        for (int k = 0; k < 5; ++k) v[k] += partial[static_cast<int64_t>(b) * 8 + k];
    __shared__ unsigned long long red64[kBlock / 64][5];
    for (int k = 0; k < 5; ++k) {
        v[k] = wave_sum(v[k]);
        if (lane == 0) red64[wave][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        unsigned long long sum = 0;
        for (int w = 0; w < kBlock / 64; ++w) sum += red64[w][threadIdx.x];
        out[threadIdx.x] = sum;
    }
    if (threadIdx.x == 5) out[5] = carry ? *carry : 0ull;
    if (threadIdx.x == 0) __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // Host memory: the stores reach it before the kernel is seen to end.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    if (seq == 0) return;
    // Every writer of out[0..5] has passed its release before the barrier.
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(&out[6], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Sums the per-block partials of k_counts into out[0..4] (one block per job).
__global__ __launch_bounds__(kBlock) void k_counts_final(const unsigned long long* __restrict__ partial,
                                                         int blocks,
                                                         unsigned long long* __restrict__ out) {
    partial += static_cast<int64_t>(blockIdx.x) * blocks * 8;
    out += static_cast<int64_t>(blockIdx.x) * 8;
    __shared__ unsigned long long red[kBlock / 64][5];
    unsigned long long v[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < blocks; b += kBlock)
        for (int k = 0; k < 5; ++k) v[k] += partial[static_cast<int64_t>(b) * 8 + k];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k = 0; k < 5; ++k) {
        v[k] = wave_sum(v[k]);
        if (lane == 0) red[wave][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        unsigned long long s = 0;
        for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Bit-sliced counters: bit b of s[l] is bit l of this thread's running count
// of Y-masked words with bit b set, so one added word costs a few bitwise
// operations for all 32 positions at once (two words enter a full adder at
// level 0, whose carry ripples up).  With kSliceBits levels a thread counts
// up to 127 words; words arrive in batches of kBatch (all loads of a batch in
// flight together), and after kChunkBatches batches (120 words) the slices
// are added into plain per-bit counters and cleared.
constexpr int kSliceBits = 7;
constexpr int kBatch = 8;
constexpr int kChunkBatches = ((1 << kSliceBits) - 1) / kBatch;

__device__ __forceinline__ void slice_add2(uint32_t (&s)[kSliceBits], uint32_t a, uint32_t b) {
    // Full adder at level 0 as two v_bitop3_b32: sum = a ^ b ^ s0 (truth
    // table 0x96), carry = majority(a, b, s0) (0xE8).
    uint32_t carry = __builtin_amdgcn_bitop3_b32(a, b, s[0], 0xE8);
    s[0] = __builtin_amdgcn_bitop3_b32(a, b, s[0], 0x96);
#pragma unroll
    for (int l = 1; l < kSliceBits; ++l) {
        const uint32_t next = s[l] & carry;
        s[l] ^= carry;
        carry = next;
    }
}

__device__ __forceinline__ void add_batch(uint32_t (&s)[kSliceBits], const uint32_t (&wv)[kBatch],
                                          const uint8_t (&yv)[kBatch], uint32_t& ny) {
#pragma unroll
    for (int q = 0; q < kBatch; q += 2) {
        const uint32_t ya = yv[q] ? 0xFFFFFFFFu : 0u;
        const uint32_t yb = yv[q + 1] ? 0xFFFFFFFFu : 0u;
        ny += (ya & 1u) + (yb & 1u);
        slice_add2(s, wv[q] & ya, wv[q + 1] & yb);
    }
}

// Per-bit masked counts of one packed word column, written as per-block
// partials: partial[(w * gridDim.x + bx) * 32 + b]; column 0 blocks also write
// #{Y = 1} to ypart[bx].  Each thread takes samples h0, h0 + stride, ...
// (coalesced across the wave).
__global__ __launch_bounds__(kBlock) void k_grad_bits(const uint32_t* __restrict__ xs,
                                                      const uint8_t* __restrict__ Y, int64_t N,
                                                      uint32_t* __restrict__ partial,
                                                      uint32_t* __restrict__ ypart,
                                                      const JobDev* __restrict__ jobs,
                                                      int64_t job_stride) {
    // With a job table, blockIdx.z selects the job; its partials start at
    // job * job_stride (u32).
    if (jobs) {
        const JobDev& jd = jobs[blockIdx.z];
        xs = jd.samples;
        Y = jd.Y;
        N = jd.N;
        partial += static_cast<int64_t>(blockIdx.z) * job_stride;
        ypart += static_cast<int64_t>(blockIdx.z) * job_stride;
    }
    const int w = blockIdx.y;
    uint32_t c[32];
#pragma unroll
    for (int b = 0; b < 32; ++b) c[b] = 0;
    uint32_t ny = 0;
    const uint32_t* row = xs + static_cast<int64_t>(w) * N;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    // Rows 16-byte aligned (N a multiple of 4): four consecutive samples per
    // 16-byte load and their Y bytes per 32-bit load, four loads of each in
    // flight per batch.
    const bool quads = (N & 3) == 0 && (reinterpret_cast<uintptr_t>(xs) & 15u) == 0 &&
                       (reinterpret_cast<uintptr_t>(Y) & 3u) == 0;
    if (quads) {
        constexpr int kQuads = 4;                                // per batch: 16 words
        constexpr int kChunkQuadBatches = ((1 << kSliceBits) - 1) / (4 * kQuads);
        const uint4* rowq = reinterpret_cast<const uint4*>(row);
        const uint32_t* yq = reinterpret_cast<const uint32_t*>(Y);
        const int64_t NQ = N >> 2;
        int64_t q = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
        while (q < NQ) {
            uint32_t sl[kSliceBits];
#pragma unroll
            for (int l = 0; l < kSliceBits; ++l) sl[l] = 0;
            for (int k = 0; k < kChunkQuadBatches && q < NQ; ++k) {
                uint4 xv[kQuads];
                uint32_t yv4[kQuads];
#pragma unroll
                for (int i = 0; i < kQuads; ++i) {
                    const int64_t qi = q + i * stride;
                    xv[i] = qi < NQ ? rowq[qi] : make_uint4(0, 0, 0, 0);
                    yv4[i] = qi < NQ ? yq[qi] : 0u;
                }
#pragma unroll
                for (int i = 0; i < kQuads; i += 2) {
                    const uint32_t wv[kBatch] = {xv[i].x,     xv[i].y,     xv[i].z,     xv[i].w,
                                                 xv[i + 1].x, xv[i + 1].y, xv[i + 1].z, xv[i + 1].w};
                    uint8_t yb[kBatch];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        yb[t] = static_cast<uint8_t>(yv4[i] >> (8 * t));
                        yb[4 + t] = static_cast<uint8_t>(yv4[i + 1] >> (8 * t));
                    }
                    add_batch(sl, wv, yb, ny);
                }
                q += kQuads * stride;
            }
#pragma unroll
            for (int b = 0; b < 32; ++b) {
                uint32_t v = 0;
#pragma unroll
                for (int l = 0; l < kSliceBits; ++l) v += ((sl[l] >> b) & 1u) << l;
                c[b] += v;
            }
        }
    }
    int64_t h = quads ? N : static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    while (h < N) {
        uint32_t sl[kSliceBits];
#pragma unroll
        for (int l = 0; l < kSliceBits; ++l) sl[l] = 0;
        int k = 0;
        // Whole batches in range: unconditional loads, all in flight at once.
        for (; k < kChunkBatches && h + (kBatch - 1) * stride < N; ++k) {
            uint32_t wv[kBatch];
            uint8_t yv[kBatch];
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                wv[q] = row[h + q * stride];
                yv[q] = Y[h + q * stride];
            }
            add_batch(sl, wv, yv, ny);
            h += kBatch * stride;
        }
        // The thread's last, partial batch.
        if (k < kChunkBatches && h < N) {
            uint32_t wv[kBatch];
            uint8_t yv[kBatch];
#pragma unroll
            for (int q = 0; q < kBatch; ++q) {
                const int64_t hq = h + q * stride;
                wv[q] = hq < N ? row[hq] : 0u;
                yv[q] = hq < N ? Y[hq] : 0;
            }
            add_batch(sl, wv, yv, ny);
            h += kBatch * stride;
        }
#pragma unroll
        for (int b = 0; b < 32; ++b) {
            uint32_t v = 0;
#pragma unroll
            for (int l = 0; l < kSliceBits; ++l) v += ((sl[l] >> b) & 1u) << l;
            c[b] += v;
        }
    }
    __shared__ uint32_t red[kBlock / 64][33];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int b = 0; b < 32; ++b) {
        const uint32_t s = wave_sum32(c[b]);
        if (lane == 0) red[wave][b] = s;
    }
    const uint32_t sy = wave_sum32(ny);
    if (lane == 0) red[wave][32] = sy;
    __syncthreads();
    if (threadIdx.x < 33) {
        uint32_t s = 0;
        for (int k = 0; k < kBlock / 64; ++k) s += red[k][threadIdx.x];
        if (threadIdx.x < 32)
            partial[(static_cast<int64_t>(w) * gridDim.x + blockIdx.x) * 32 + threadIdx.x] = s;
        else if (w == 0)
            ypart[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kBlock) void k_grad_finalize(const uint32_t* __restrict__ partial,
                                                          const uint32_t* __restrict__ ypart,
                                                          int bx, const float* __restrict__ p,
                                                          int n, int K, int PW, int64_t N,
                                                          float* __restrict__ G,
                                                          unsigned long long* __restrict__ counts,
                                                          const JobDev* __restrict__ jobs,
                                                          int64_t job_stride) {
    if (jobs) {
        const JobDev& jd = jobs[blockIdx.y];
        p = jd.p;
        N = jd.N;
        G = jd.G;
        counts = nullptr;
        partial += static_cast<int64_t>(blockIdx.y) * job_stride;
        ypart += static_cast<int64_t>(blockIdx.y) * job_stride;
        if (!G) return;
    }
    // One wavefront per (i, s); its lanes add the per-block partials.
    const int lane = threadIdx.x & 63;
    const int idx = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (idx >= n * K) return;
    const int i = idx / K, s = idx % K;
    // a(j) = #{h : Y_h = 1 and x_{h,i} >= j}; a(0) = #{Y = 1}; a(K) = 0.
    auto level_count = [&](int j) -> unsigned long long {
        unsigned long long t = 0;
        if (j == 0) {
            for (int b = lane; b < bx; b += 64) t += ypart[b];
        } else if (j < K) {
            const int w = (j - 1) * PW + (i >> 5);
            const uint32_t* col = partial + static_cast<int64_t>(w) * bx * 32 + (i & 31);
            for (int b = lane; b < bx; b += 64) t += col[static_cast<int64_t>(b) * 32];
        }
        return wave_sum(t);
    };
    const unsigned long long cnt = level_count(s) - level_count(s + 1);
    if (lane == 0) {
        const float pv = p[idx];
        const float g = pv > 0.0f ? static_cast<float>(cnt) / (static_cast<float>(N) * pv) : 0.0f;
        G[idx] = g;
        if (counts) counts[idx] = cnt;
    }
}

// Binary Birnbaum importance from the same partials (K = 2, one plane): one
// wavefront per component i adds a(0) = #{Y = 1} and a(1) = #{Y = 1, x_i = 1};
// c1 = a(1), c0 = a(0) - a(1), and I[i] = c1 / (N p1) - c0 / (N p0) with both
// quotients in fp64 (0 where p = 0), the difference rounded once to fp32.
__global__ __launch_bounds__(kBlock) void k_importance_finalize(
    const uint32_t* __restrict__ partial, const uint32_t* __restrict__ ypart, int bx,
    const double* __restrict__ p, int n, int64_t N, float* __restrict__ I) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    if (i >= n) return;
    unsigned long long a0 = 0, a1 = 0;
    const uint32_t* col = partial + static_cast<int64_t>(i >> 5) * bx * 32 + (i & 31);
    for (int b = lane; b < bx; b += 64) {
        a0 += ypart[b];
        a1 += col[static_cast<int64_t>(b) * 32];
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    if (lane == 0) {
        const double Nd = static_cast<double>(N);
        const double p0 = p[2 * i], p1 = p[2 * i + 1];
        const double g1 = p1 > 0.0 ? static_cast<double>(a1) / (Nd * p1) : 0.0;
        const double g0 = p0 > 0.0 ? static_cast<double>(a0 - a1) / (Nd * p0) : 0.0;
        I[i] = static_cast<float>(g1 - g0);
    }
}

// Copies every job's gradient into one buffer (out + job.g_off), so a plan
// returns all gradients with a single device-to-host copy.
__global__ __launch_bounds__(kBlock) void k_gather_G(const JobDev* __restrict__ jobs, int nK,
                                                     float* __restrict__ out) {
    const JobDev& jd = jobs[blockIdx.y];
    const int idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx < nK && jd.G) out[jd.g_off + idx] = jd.G[idx];
}

}  // namespace

hipError_t launch_gather_G(hipStream_t st, const JobDev* jobs, int n_jobs, int nK, float* out) {
    hipLaunchKernelGGL(k_gather_G, dim3((nK + kBlock - 1) / kBlock, n_jobs), dim3(kBlock), 0, st,
                       jobs, nK, out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(hipStream_t st, uint64_t* p, int64_t count, uint64_t value) {
    const dim3 grid(static_cast<unsigned>((count + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_fill_u64, grid, dim3(kBlock), 0, st,
                       reinterpret_cast<unsigned long long*>(p), count,
                       static_cast<unsigned long long>(value));
    return hipGetLastError();
}

hipError_t launch_counts(hipStream_t st, const uint8_t* d_flags, const uint8_t* d_Y, int64_t N,
                         uint64_t* d_counters, uint64_t* d_partial, const JobDev* jobs,
                         int n_jobs) {
    int64_t blocks = (N + kBlock * 16 - 1) / (kBlock * 16);
    if (blocks > kMaxReduceBlocks) blocks = kMaxReduceBlocks;
    if (blocks < 1) blocks = 1;
    const int nj = jobs ? n_jobs : 1;
    hipLaunchKernelGGL(k_counts, dim3(static_cast<unsigned>(blocks), nj), dim3(kBlock), 0, st,
                       d_flags, d_Y, N, reinterpret_cast<unsigned long long*>(d_partial), jobs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_counts_final, dim3(nj), dim3(kBlock), 0, st,
                       reinterpret_cast<const unsigned long long*>(d_partial),
                       static_cast<int>(blocks), reinterpret_cast<unsigned long long*>(d_counters));
    return hipGetLastError();
}

hipError_t launch_counts_vec(hipStream_t st, const uint8_t* d_flags, const uint8_t* d_Y, int64_t N,
                             uint64_t* out, uint64_t* d_partial, uint32_t* d_ticket,
                             const uint64_t* d_carry, uint64_t seq) {
    int64_t blocks = ((N >> 4) + kBlock * kCountsChunks - 1) / (kBlock * kCountsChunks);
    if (blocks > kMaxReduceBlocks) blocks = kMaxReduceBlocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_counts_vec, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0, st,
                       d_flags, d_Y, N, reinterpret_cast<unsigned long long*>(d_partial),
                       reinterpret_cast<unsigned long long*>(out), d_ticket,
                       reinterpret_cast<const unsigned long long*>(d_carry),
                       static_cast<unsigned long long>(seq));
    return hipGetLastError();
}

hipError_t launch_importance(hipStream_t st, int n, const double* d_p64, const uint32_t* d_samples,
                             const uint8_t* d_Y, int64_t N, uint32_t* d_partial, float* d_I) {
    const int W = plane_words(n);
    const int64_t bx = grad_blocks(N);
    uint32_t* ypart = d_partial + static_cast<int64_t>(W) * bx * 32;
    hipLaunchKernelGGL(k_grad_bits, dim3(static_cast<unsigned>(bx), W, 1), dim3(kBlock), 0, st,
                       d_samples, d_Y, N, d_partial, ypart, nullptr, int64_t{0});
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int waves_per_block = kBlock / 64;
    hipLaunchKernelGGL(k_importance_finalize, dim3((n + waves_per_block - 1) / waves_per_block),
                       dim3(kBlock), 0, st, d_partial, ypart, static_cast<int>(bx), d_p64, n, N,
                       d_I);
    return hipGetLastError();
}

int64_t grad_blocks(int64_t N) {
    // About 64 samples per thread, at most kMaxGradBlocks blocks per word column.
    int64_t bx = (N + kBlock * 64 - 1) / (kBlock * 64);
    if (bx > kMaxGradBlocks) bx = kMaxGradBlocks;
    if (bx < 1) bx = 1;
    return bx;
}

hipError_t launch_grad(hipStream_t st, int n, int K, const float* d_p, const uint32_t* d_samples,
                       const uint8_t* d_Y, int64_t N, uint32_t* d_partial, float* d_G,
                       uint64_t* d_counts, const JobDev* jobs, int n_jobs) {
    const int PW = plane_words(n);
    const int W = (K - 1) * PW;
    const int64_t bx = grad_blocks(N);
    const int64_t job_stride = static_cast<int64_t>(W) * bx * 32 + bx;
    const int nj = jobs ? n_jobs : 1;
    uint32_t* ypart = d_partial + static_cast<int64_t>(W) * bx * 32;
    hipLaunchKernelGGL(k_grad_bits, dim3(static_cast<unsigned>(bx), W, nj), dim3(kBlock), 0, st,
                       d_samples, d_Y, N, d_partial, ypart, jobs, job_stride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int total = n * K;
    const int waves_per_block = kBlock / 64;
    hipLaunchKernelGGL(k_grad_finalize, dim3((total + waves_per_block - 1) / waves_per_block, nj),
                       dim3(kBlock), 0, st,
                       d_partial, ypart, static_cast<int>(bx), d_p, n, K, PW, N, d_G,
                       reinterpret_cast<unsigned long long*>(d_counts), jobs, job_stride);
    return hipGetLastError();
}

}  // namespace rsr
