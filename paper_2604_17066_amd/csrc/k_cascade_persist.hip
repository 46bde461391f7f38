// Persistent LABEL cascade on a consistent reference set (no upper row below
// a lower row, which valid reference sets of section 2.2 always are): each
// sample stops at its first match on either side, which decides its label
// (Algorithm 1).  Rows are stored by increasing size, so most samples match
// among the first rows; round r covers rows [bound[r], bound[r+1]) of both
// sides.
//
//   round 0 (k_casc_r0, vector ALU, on the samples where they are): block b
//     takes a contiguous span of samples; each lane tests S of them at a time
//     against the round's rows with a per-wave early exit (casc_popcount.h),
//     flags the matched ones and appends the others to region b of the
//     compact buffer (the span's own slots).
//   rounds 1.. (k_casc_persist, one cooperative launch, FP4 matrix core on
//     32 x 32 x 64 tiles, dom_fp4x32.h): work items are (group of G samples,
//     chunk of the round's row tiles), one per wavefront at a time, with no
//     block synchronisation inside a round; the row fragments are read
//     straight from memory (a round's rows stay in L2), the next tile's while
//     the current one's products run.  With one chunk a wave flags and
//     compacts its group itself; with several, each wave ORs its matches into
//     the samples' match words and takes a ticket on the group, and the wave
//     that takes the last ticket flags and compacts the group.  The last round
//     flags every remaining sample (0 = unclassified).
//
// Same-address device atomics serialise (about 12 ns each on MI355X), so the
// compaction uses none: every block appends to its own region through an LDS
// counter and stores its count at the end of the round, and the next round
// reads the regions through a prefix sum of the counts (a binary search per
// sample).  A grid barrier separates the rounds; its arrivals are spread over
// up to 64 counters and only the last arrival of each reaches the top
// counter.  It waits with a time limit, and a block that exceeds it sets the
// error flag and leaves, so the kernel always ends.  The grid never exceeds
// the blocks that can be resident at once (cooperative launch).
#include "casc_popcount.h"
#include "dom_fp4x32.h"

namespace rsr {
namespace {

using namespace mf;
using namespace casc;


constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kMaxRounds = CascadeBuffers::kMaxRounds;
// Most regions (blocks) of one round: bounds both grids.
constexpr int kMaxRegions = 2048;
// Chunks of fewer row tiles than this (per side) are not worth their sample
// loads.
constexpr int kMinChunkTiles = 4;
// Barrier time limit in ticks of the 100 MHz real-time counter (10 s);
// rsr_debug_barrier_timeout changes it for tests of the time-out path.
constexpr uint64_t kBarrierTimeout = 1000000000ull;
uint64_t g_barrier_ticks = kBarrierTimeout;
// Barrier: kBarGroups arrival counters, the top counter and the generation,
// each on its own 128-byte line (32 u32).
constexpr int kBarGroups = 64;
constexpr int kLine = 32;

// Sample tiles (32 samples) per wave in the matrix-core rounds.
// (Measured on the multi-state level, 10 k-steps: two tiles 0.29 ms, one
// 0.31 ms.)
constexpr int casc_tiles32(int KS) { return KS <= 10 ? 2 : 1; }

// Register sets of a wave's read-ahead ring of A fragments (one tile read
// ahead; three sets measured no faster).
constexpr int kRing = 2;

// Samples per lane in round 0.
constexpr int r0_samples(int W) { return W <= 12 ? 4 : (W <= 24 ? 2 : 1); }

// Layout of the state buffer (u32 words), all zero on entry.
struct StateLayout {
    int64_t cnt = 0;    // [kMaxRounds][kMaxRegions] samples kept per region
    int64_t cap = 0;    // [kMaxRounds] region capacity (samples) of each round's output
    int64_t ngrid = 0;  // [kMaxRounds] regions written by each round
    int64_t bar = 0;    // barrier: kBarGroups + 2 lines
    int64_t done = 0;   // group tickets
    int64_t total = 0;  // words
    StateLayout() = default;
    explicit StateLayout(int64_t groups) {
        cnt = 0;
        cap = cnt + static_cast<int64_t>(kMaxRounds) * kMaxRegions;
        ngrid = cap + kMaxRounds;
        bar = (ngrid + kMaxRounds + kLine - 1) / kLine * kLine;
        done = bar + static_cast<int64_t>(kBarGroups + 2) * kLine;
        total = done + groups;
    }
};

struct PersistArgs {
    SegSrc seg;                      // the samples and the flags
    const v4i* low32;                // FP4 32-row tiles
    const v4i* up32;
    int64_t R_L, R_U;
    int n, PW, W;
    int rounds;
    int bound[kMaxRounds + 1];
    uint32_t* words[2];              // compact buffers [W][stride], by round parity
    int32_t* index[2];
    uint32_t* match[2];
    int64_t stride;
    uint32_t* state;                 // StateLayout
    StateLayout L;
    unsigned long long* err;         // set to 1 when a barrier times out
    uint64_t timeout;                // barrier time limit (real-time counter ticks)
};

// ---- round 0 -----------------------------------------------------------------

// Block b takes samples [b * span, (b + 1) * span) and appends the undecided
// ones to the same slots of buffer 1 (its region), its count to cnt0[b];
// block 0 also stores the region layout (capacity span, gridDim.x regions).
template <int W, int S>
__global__ __launch_bounds__(kBlock) void k_casc_r0(SegSrc seg, int w_real,
                                                    const uint32_t* __restrict__ low_n, int l1,
                                                    const uint32_t* __restrict__ up_b, int u1,
                                                    uint32_t* __restrict__ dst,
                                                    int32_t* __restrict__ dst_idx,
                                                    uint32_t* __restrict__ dst_match,
                                                    int64_t dst_stride, int64_t span,
                                                    uint32_t* __restrict__ state, int64_t cap_at,
                                                    int64_t ngrid_at, int last) {
    __shared__ int s_counts[S * kWaves];
    __shared__ uint32_t s_rows[2 * tile_rows<W>() * W];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t begin = static_cast<int64_t>(blockIdx.x) * span;
    const int64_t end = begin + span < seg.total ? begin + span : seg.total;
    int64_t kept = 0;  // block-uniform
    // Block-uniform loop (test_rows synchronises the block).
    for (int64_t b0 = begin; b0 < end; b0 += static_cast<int64_t>(kBlock) * S) {
        const int64_t j0 = b0 + static_cast<int64_t>(wave) * 64 * S;
        uint32_t x[S][W];
        bool valid[S];
        int64_t gg[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            gg[s] = j0 + s * 64 + lane;
            valid[s] = gg[s] < end;
            int job = 0;
            int64_t at = 0, stride = 0;
            const uint32_t* base = nullptr;
            if (valid[s]) {
                seg_locate(seg, gg[s], job, at);
                base = seg_words(seg, job, stride);
            }
#pragma unroll
            for (int w = 0; w < W; ++w) {
                x[s][w] = (valid[s] && w < w_real) ? base[w * stride + at] : 0u;
            }
        }
        uint32_t mnL[S], mnU[S];
#pragma unroll
        for (int s = 0; s < S; ++s) mnL[s] = mnU[s] = 0xFFFFFFFFu;
        test_rows<W, S, kBlock>(x, valid, low_n, 0, l1, up_b, 0, u1, mnL, mnU, s_rows);
        bool carry[S];
        uint64_t mask[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bool hit = mnL[s] == 0u || mnU[s] == 0u;
            if (valid[s] && (hit || last)) {
                int job;
                int64_t h;
                seg_locate(seg, gg[s], job, h);
                seg_flags(seg, job)[h] = static_cast<uint8_t>(mnL[s] == 0u ? 1 : (mnU[s] == 0u ? 2 : 0));
            }
            carry[s] = !last && valid[s] && !hit;
            mask[s] = __ballot(carry[s]);
            if (lane == 0) s_counts[s * kWaves + wave] = __popcll(mask[s]);
        }
        __syncthreads();
        // Exclusive prefix of the (s, wave) counts (LDS broadcasts).
        int before[S], tot = 0;
        for (int k = 0; k < S * kWaves; ++k) {
            const int c = s_counts[k];
#pragma unroll
            for (int s = 0; s < S; ++s)
                if (k == s * kWaves + wave) before[s] = tot;
            tot += c;
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (carry[s]) {
                const int64_t slot = begin + kept + before[s] +
                                     __popcll(mask[s] & ((1ull << lane) - 1ull));
                dst_idx[slot] = static_cast<int32_t>(gg[s]);
                dst_match[slot] = 0u;
#pragma unroll
                for (int w = 0; w < W; ++w)
                    if (w < w_real) dst[w * dst_stride + slot] = x[s][w];
            }
        }
        kept += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        state[blockIdx.x] = static_cast<uint32_t>(kept);
        if (blockIdx.x == 0) {
            state[cap_at] = static_cast<uint32_t>(span);
            state[ngrid_at] = gridDim.x;
        }
    }
}

// ---- rounds 1.. -----------------------------------------------------------------

// Grid barrier with a time limit; returns false (and sets *err) when it timed
// out or another block already did.  Every thread of every block calls it.
// The counters only grow: at the barrier of generation k, group counter g
// completes at (k + 1) times its blocks and the top counter at (k + 1) times
// the groups.  A release fence before the arrival writes this block's earlier
// stores back from its L2 (the L2s of the XCDs are not coherent); an acquire
// fence after the barrier drops stale lines.
__device__ bool grid_sync(uint32_t* bar, unsigned long long* err, uint64_t timeout) {
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const unsigned nblocks = gridDim.x;
        const unsigned groups = nblocks < static_cast<unsigned>(kBarGroups) ? nblocks : kBarGroups;
        const unsigned grp = blockIdx.x % groups;
        const unsigned in_grp = (nblocks - 1 - grp) / groups + 1;
        uint32_t* sub = bar + grp * kLine;
        uint32_t* top = bar + kBarGroups * kLine;
        uint32_t* gen_p = bar + (kBarGroups + 1) * kLine;
        const unsigned gen = __hip_atomic_load(gen_p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        bool released = false;
        if (__hip_atomic_fetch_add(sub, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 ==
                in_grp * (gen + 1) &&
            __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1 ==
                groups * (gen + 1)) {
            __hip_atomic_fetch_add(gen_p, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            released = true;
        }
        if (!released) {
            const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
            while (__hip_atomic_load(gen_p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (__builtin_amdgcn_s_memrealtime() - t0 > timeout) {
                    ok = 0;
                    __hip_atomic_store(err, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0ull) ok = 0;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// Exclusive prefix sum over the block of one value per thread; *total gets
// the block's sum.  Every thread calls it.
__device__ uint32_t block_scan(uint32_t v, uint32_t* s_wave, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d);
        if (lane >= d) inc += y;
    }
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    uint32_t before = 0, sum = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
        const uint32_t c = s_wave[k];
        if (k < wave) before += c;
        sum += c;
    }
    *total = sum;
    __syncthreads();
    return before + inc - v;
}

// Physical slot of virtual position p of a round's input: region j holds
// prefix[j + 1] - prefix[j] samples from slot j * cap.
__device__ __forceinline__ int64_t region_slot(const uint32_t* prefix, int nreg, int64_t cap,
                                               int64_t p) {
    int lo = 0, hi = nreg - 1;  // the last j with prefix[j] <= p
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (static_cast<int64_t>(prefix[mid]) <= p) lo = mid;
        else hi = mid - 1;
    }
    return static_cast<int64_t>(lo) * cap + (p - static_cast<int64_t>(prefix[lo]));
}

// One wave's pass over a range of 32-row tiles of one side (rows past `rows`
// from the range's first tile are padding).  The tiles' A fragments are read
// straight from memory into a ring of R register sets, R - 1 tiles ahead of
// the products.  The read-ahead is unconditional (past the last tile it
// reads the last tile again): a conditional load would make the compiler's
// wait counts cover both paths, i.e. wait for the tile just requested.
// acc[t] keeps the signed minimum over this lane's rows (negative = some row
// matched).  The wave leaves once every live sample is decided.
template <int KS, int MT, int R>
__device__ __forceinline__ void wave_pass(const v4i (&bf)[MT][KS], const v4i* __restrict__ frag,
                                          int64_t rows, int (&acc)[MT], const bool (&live)[MT]) {
    if (rows <= 0) return;
    const int lane = threadIdx.x & 63, half = lane >> 5;
    const int tiles = __builtin_amdgcn_readfirstlane(static_cast<int>((rows + 31) / 32));
    const int last_rows = static_cast<int>(rows - 32 * static_cast<int64_t>(tiles - 1));
    const v16f start = v16f{} - 0.5f;
    v4i ring[R][KS];
#pragma unroll
    for (int k = 0; k < R - 1; ++k) {
        const int64_t tk = k < tiles ? k : tiles - 1;
#pragma unroll
        for (int s = 0; s < KS; ++s) ring[k][s] = frag[(tk * KS + s) * 64 + lane];
    }
    bool stop = false;
    for (int t0 = 0; !stop; t0 += R) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int t = t0 + k;
            if (stop) break;
            const int64_t tn = t + R - 1 < tiles ? t + R - 1 : tiles - 1;
#pragma unroll
            for (int s = 0; s < KS; ++s)
                ring[(k + R - 1) % R][s] = frag[(tn * KS + s) * 64 + lane];
            const bool more = t + 1 < tiles;
            v16f r[MT];
#pragma unroll
            for (int s = 0; s < KS; ++s)
#pragma unroll
                for (int m = 0; m < MT; ++m) r[m] = mfma32_step(ring[k][s], bf[m][s], s == 0 ? start : r[m]);
            bool done = true;
#pragma unroll
            for (int m = 0; m < MT; ++m) {
                acc[m] = more ? fold32<false>(r[m], acc[m]) : fold32_last<false>(r[m], acc[m], last_rows, half);
                done = done && (!live[m] || min(acc[m], __shfl_xor(acc[m], 32)) < 0);
            }
            if (!more || __all(done)) stop = true;
        }
    }
}

template <int W, int KS>
__global__ __launch_bounds__(kBlock) void k_casc_persist(PersistArgs a) {
    constexpr int MT = casc_tiles32(KS);
    constexpr int G = 32 * MT;  // samples per wave item
    constexpr int RING = kRing;
    constexpr int kPer = kMaxRegions / kBlock;
    __shared__ uint32_t s_prefix[kMaxRegions + 1];
    __shared__ uint32_t s_wave[kWaves];
    __shared__ unsigned s_out;
    // The wave index is uniform: readfirstlane lets the item loop and its
    // branches run on the scalar unit.
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t gwave = static_cast<int64_t>(blockIdx.x) * kWaves + wave;
    const int64_t nwaves = static_cast<int64_t>(gridDim.x) * kWaves;
    const uint64_t below32 = (1ull << (lane & 31)) - 1ull;
    uint32_t* st = a.state;
    for (int r = 1; r < a.rounds; ++r) {
        const bool last = r + 1 == a.rounds;
        if (r > 1 && !grid_sync(st + a.L.bar, a.err, a.timeout)) return;
        // Regions of this round's input (written by round r - 1) and the
        // prefix sum of their counts, in LDS.
        const int nreg = static_cast<int>(st[a.L.ngrid + r - 1]);
        const int64_t in_cap = static_cast<int64_t>(st[a.L.cap + r - 1]);
        {
            const uint32_t* in_cnt = st + a.L.cnt + static_cast<int64_t>(r - 1) * kMaxRegions;
            uint32_t v[kPer], sum = 0;
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int j = threadIdx.x * kPer + k;
                v[k] = j < nreg ? in_cnt[j] : 0u;
                sum += v[k];
            }
            uint32_t all;
            uint32_t run = block_scan(sum, s_wave, &all);
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                s_prefix[threadIdx.x * kPer + k] = run;
                run += v[k];
            }
            if (threadIdx.x == 0) {
                s_prefix[kMaxRegions] = all;
                s_out = 0;
            }
            __syncthreads();
        }
        const int64_t n_in = static_cast<int64_t>(s_prefix[kMaxRegions]);
        // Every block reads the same counts: all leave together.
        if (n_in == 0) return;
        const int lo = a.bound[r], hi = a.bound[r + 1];
        const int in = r & 1, out = in ^ 1;
        const uint32_t* src_w = a.words[in];
        const int32_t* src_i = a.index[in];
        uint32_t* src_m = a.match[in];
        // Tile ranges of the round's rows (32-row tiles; a tile may reach rows
        // of a neighbouring round, which on a consistent set only repeats or
        // anticipates a decision).
        const int64_t lcl0 = lo < a.R_L ? lo : a.R_L, lcl1 = hi < a.R_L ? hi : a.R_L;
        const int64_t ucl0 = lo < a.R_U ? lo : a.R_U, ucl1 = hi < a.R_U ? hi : a.R_U;
        const int lt0 = static_cast<int>(lcl0 / 32), lt1 = static_cast<int>((lcl1 + 31) / 32);
        const int ut0 = static_cast<int>(ucl0 / 32), ut1 = static_cast<int>((ucl1 + 31) / 32);
        const int TLr = lt1 > lt0 ? lt1 - lt0 : 0, TUr = ut1 > ut0 ? ut1 - ut0 : 0;
        const int tmax = TLr > TUr ? TLr : TUr;
        const int64_t groups = (n_in + G - 1) / G;
        // Chunks: as many as keep the items within one per wave.
        int64_t chunks = nwaves / groups;
        const int64_t cmax = tmax / kMinChunkTiles > 1 ? tmax / kMinChunkTiles : 1;
        if (chunks > cmax) chunks = cmax;
        if (chunks < 1) chunks = 1;
        const int64_t items = groups * chunks;
        // Output regions: a wave item compacts at most one group of G.
        const int64_t out_cap = static_cast<int64_t>(kWaves) * ((items + nwaves - 1) / nwaves) * G;
        const int64_t out_base = static_cast<int64_t>(blockIdx.x) * out_cap;
        // An item's samples: lane l holds virtual positions gbase + 32 t +
        // l % 32 and their words 2 s + l / 32, with the sample's index (read
        // unconditionally from clamped positions: see wave_pass).  A second
        // item read ahead does not help: loads complete in issue order, so
        // the first tile's wait would cover it too.
        struct Held {
            uint32_t raw[MT][KS];
            int64_t slot[MT];
            int32_t idx[MT];
            bool valid[MT];
        };
        auto fetch = [&](int64_t item, Held& h) {
            const int64_t gbase = (item / chunks) * G;
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                const int64_t p = gbase + 32 * t + (lane & 31);
                h.valid[t] = p < n_in;
                h.slot[t] = region_slot(s_prefix, nreg, in_cap, p < n_in ? p : n_in - 1);
                h.idx[t] = src_i[h.slot[t]];
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    const int w = 2 * s + (lane >> 5);
                    const uint32_t v = src_w[(w < a.W ? w : a.W - 1) * a.stride + h.slot[t]];
                    h.raw[t][s] = (h.valid[t] && w < a.W) ? v : 0u;
                }
            }
        };
        for (int64_t item = gwave; item < items; item += nwaves) {
            Held cur;
            fetch(item, cur);
            const int64_t g = item / chunks, c = item % chunks;
            const int cl0 = lt0 + static_cast<int>((TLr * c) / chunks);
            const int cl1 = lt0 + static_cast<int>((TLr * (c + 1)) / chunks);
            const int cu0 = ut0 + static_cast<int>((TUr * c) / chunks);
            const int cu1 = ut0 + static_cast<int>((TUr * (c + 1)) / chunks);
            const int64_t rl = cl1 > cl0 ? (32ll * cl1 < a.R_L ? 32ll * cl1 : a.R_L) - 32ll * cl0 : 0;
            const int64_t ru = cu1 > cu0 ? (32ll * cu1 < a.R_U ? 32ll * cu1 : a.R_U) - 32ll * cu0 : 0;
            v4i bf[MT][KS];
#pragma unroll
            for (int t = 0; t < MT; ++t)
#pragma unroll
                for (int s = 0; s < KS; ++s) bf[t][s] = expand_word_fp4(cur.raw[t][s]);
            int accL[MT], accU[MT];
            bool lowered[MT], todo[MT];
#pragma unroll
            for (int t = 0; t < MT; ++t) accL[t] = accU[t] = 0;
            wave_pass<KS, MT, RING>(bf, a.low32 + static_cast<int64_t>(cl0) * KS * 64, rl, accL, cur.valid);
            bool any_left = false;
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                lowered[t] = min(accL[t], __shfl_xor(accL[t], 32)) < 0;
                todo[t] = cur.valid[t] && !lowered[t];
                any_left = any_left || todo[t];
            }
            if (__any(any_left)) {
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    const v4i m = expand_word_fp4(valid_word(2 * s + (lane >> 5), a.n, a.PW, a.W));
#pragma unroll
                    for (int t = 0; t < MT; ++t) bf[t][s] ^= m;
                }
                wave_pass<KS, MT, RING>(bf, a.up32 + static_cast<int64_t>(cu0) * KS * 64, ru, accU, todo);
            }
            uint32_t bits[MT];
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                const int m = min(accU[t], __shfl_xor(accU[t], 32));
                bits[t] = lowered[t] ? 1u : (m < 0 ? 2u : 0u);
            }
            bool resolve = true;
            if (chunks > 1) {
                // The match words are only touched by device-scope atomics
                // until the group is resolved, which act at the device's
                // coherence point: the wave waits for its ORs to return (the
                // empty asm consumes their results) before it takes its
                // ticket, so the wave that takes the last ticket sees them all.
                uint32_t dep = 0;
                if (lane < 32) {
#pragma unroll
                    for (int t = 0; t < MT; ++t)
                        if (cur.valid[t] && bits[t])
                            dep |= __hip_atomic_fetch_or(&src_m[cur.slot[t]], bits[t], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                }
                asm volatile("" ::"v"(dep) : "memory");
                unsigned fin = 0;
                if (lane == 0) {
                    uint32_t* ticket_p = st + a.L.done + g;
                    const unsigned ticket = __hip_atomic_fetch_add(ticket_p, 1u, __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT);
                    fin = ticket + 1 == static_cast<unsigned>(chunks) ? 1u : 0u;
                    if (fin) __hip_atomic_store(ticket_p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                resolve = __shfl(fin, 0) != 0u;
                if (resolve) {
#pragma unroll
                    for (int t = 0; t < MT; ++t)
                        bits[t] = cur.valid[t] ? __hip_atomic_load(&src_m[cur.slot[t]], __ATOMIC_RELAXED,
                                                                   __HIP_MEMORY_SCOPE_AGENT)
                                               : 0u;
                }
            }
            if (resolve) {
                // Flags of the group's decided samples (all of them in the
                // last round; lanes 0..31) and compaction of the others into
                // this block's region from the held words: lanes l and l + 32
                // write the words 2 s and 2 s + 1 of their sample.
#pragma unroll
                for (int t = 0; t < MT; ++t) {
                    const uint32_t b = cur.valid[t] ? bits[t] : 0u;
                    if (lane < 32 && cur.valid[t] && (b || last)) {
                        int job;
                        int64_t h;
                        seg_locate(a.seg, cur.idx[t], job, h);
                        seg_flags(a.seg, job)[h] = static_cast<uint8_t>((b & 1u) ? 1 : ((b & 2u) ? 2 : 0));
                    }
                    if (last) continue;
                    const bool carry = cur.valid[t] && b == 0u;
                    const uint64_t mask = __ballot(carry && lane < 32);
                    if (mask == 0) continue;
                    unsigned base = 0;
                    if (lane == 0) base = atomicAdd(&s_out, static_cast<unsigned>(__popcll(mask)));
                    base = __shfl(base, 0);
                    if (carry) {
                        const int64_t o = out_base + base + __popcll(mask & below32);
                        if (lane < 32) {
                            a.index[out][o] = cur.idx[t];
                            a.match[out][o] = 0u;
                        }
#pragma unroll
                        for (int s = 0; s < KS; ++s) {
                            const int w = 2 * s + (lane >> 5);
                            if (w < a.W) a.words[out][w * a.stride + o] = cur.raw[t][s];
                        }
                    }
                }
            }
        }
        if (last) break;
        // This block's count and (block 0) the round's region layout, stored
        // before the next barrier.
        __syncthreads();
        if (threadIdx.x == 0) {
            st[a.L.cnt + static_cast<int64_t>(r) * kMaxRegions + blockIdx.x] = s_out;
            if (blockIdx.x == 0) {
                st[a.L.cap + r] = static_cast<uint32_t>(out_cap);
                st[a.L.ngrid + r] = gridDim.x;
            }
        }
    }
}

template <int W, int KS>
int per_cu_wk() {
    static int per_cu = -1;
    if (per_cu < 0) {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_casc_persist<W, KS>, kBlock, 0) != hipSuccess)
            b = 0;
        per_cu = b;
    }
    return per_cu;
}

template <int W, int KS>
hipError_t launch_wk(hipStream_t st, PersistArgs& args, int grid) {
    void* kargs[] = {&args};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_casc_persist<W, KS>),
                                      dim3(static_cast<unsigned>(grid)), dim3(kBlock), kargs, 0, st);
}

template <int W>
hipError_t launch_r0(hipStream_t st, const SegSrc& seg, const rsr_refs* refs, const PersistArgs& a,
                     int grid0, int64_t span) {
    constexpr int S = r0_samples(W);
    const int l1 = static_cast<int>(a.bound[1] < refs->R_L ? a.bound[1] : refs->R_L);
    const int u1 = static_cast<int>(a.bound[1] < refs->R_U ? a.bound[1] : refs->R_U);
    hipLaunchKernelGGL((k_casc_r0<W, S>), dim3(static_cast<unsigned>(grid0)), dim3(kBlock), 0, st, seg,
                       refs->W, refs->d_lower_nbits, l1, refs->d_upper_bits, u1, a.words[1],
                       a.index[1], a.match[1], a.stride, span, a.state, a.L.cap, a.L.ngrid,
                       a.rounds == 1 ? 1 : 0);
    return hipGetLastError();
}

// Blocks that can be resident at once (0 when the width has no kernel).
int resident_blocks(const rsr_refs* refs, int cus) {
    int per_cu = 0;
    switch (refs->WR * 100 + refs->KS) {
#define RSR_WK_CASE(w, k) \
    case w * 100 + k: per_cu = per_cu_wk<w, k>(); break;
        RSR_WK_CASE(1, 1) RSR_WK_CASE(2, 1) RSR_WK_CASE(3, 2) RSR_WK_CASE(4, 2) RSR_WK_CASE(5, 3)
        RSR_WK_CASE(6, 3) RSR_WK_CASE(8, 4) RSR_WK_CASE(10, 5) RSR_WK_CASE(12, 6)
        RSR_WK_CASE(16, 7) RSR_WK_CASE(16, 8) RSR_WK_CASE(20, 9) RSR_WK_CASE(20, 10)
        RSR_WK_CASE(24, 11) RSR_WK_CASE(24, 12) RSR_WK_CASE(32, 13) RSR_WK_CASE(32, 14)
        RSR_WK_CASE(32, 15) RSR_WK_CASE(32, 16) RSR_WK_CASE(40, 17) RSR_WK_CASE(40, 18)
        RSR_WK_CASE(40, 19) RSR_WK_CASE(40, 20)
#undef RSR_WK_CASE
        default: return 0;
    }
    return per_cu * cus;
}

int group_size(int KS) { return 32 * casc_tiles32(KS); }

}  // namespace

void set_barrier_timeout(int64_t ticks) {
    g_barrier_ticks = ticks < 0 ? kBarrierTimeout : static_cast<uint64_t>(ticks);
}

bool casc_persist_supported(const rsr_refs* refs) {
    return refs->KS > 0 && resident_blocks(refs, 1) > 0;
}

// Grid of the persistent launch for N samples: the resident blocks, at most
// kMaxRegions, and no more than the samples can keep busy.
int casc_persist_grid(const rsr_refs* refs, int64_t N, int cus) {
    int64_t grid = resident_blocks(refs, cus);
    if (grid > kMaxRegions) grid = kMaxRegions;
    const int64_t want = (N + static_cast<int64_t>(kWaves) * group_size(refs->KS) - 1) /
                         (static_cast<int64_t>(kWaves) * group_size(refs->KS));
    if (grid > want) grid = want;
    return static_cast<int>(grid);
}

// Compact-buffer capacity for N samples: a round after round 0 keeps at most
// its input plus one group per wave of slack in its regions.
int64_t casc_persist_stride(const rsr_refs* refs, int64_t N, int cus) {
    const int64_t G = group_size(refs->KS);
    return N + (static_cast<int64_t>(casc_persist_grid(refs, N, cus)) * kWaves + 1) * G;
}

int64_t casc_persist_state_words(int64_t stride, int KS) {
    const int64_t G = group_size(KS);
    return StateLayout((stride + G - 1) / G).total;
}

hipError_t launch_casc_persist(hipStream_t st, const rsr_refs* refs, const SegSrc& seg,
                               const CascadeBuffers& cb, const CascadeShape& shape,
                               unsigned* d_state, unsigned long long* d_err, int cus) {
    if (shape.first < 1 || shape.growth < 2 || refs->KS == 0) return hipErrorInvalidValue;
    const int64_t total = seg.total;
    const int grid = casc_persist_grid(refs, total, cus);
    if (grid < 1 || cb.stride < casc_persist_stride(refs, total, cus)) return hipErrorInvalidValue;
    PersistArgs a{};
    a.seg = seg;
    a.low32 = reinterpret_cast<const v4i*>(refs->d_lower_frag32);
    a.up32 = reinterpret_cast<const v4i*>(refs->d_upper_frag32);
    a.R_L = refs->R_L;
    a.R_U = refs->R_U;
    a.n = refs->n;
    a.PW = plane_words(refs->n);
    a.W = refs->W;
    const int64_t n_max = refs->R_L > refs->R_U ? refs->R_L : refs->R_U;
    int64_t lo = 0, hi = shape.first;
    int r = 0;
    for (;; ++r) {
        const bool last = hi >= n_max || r + 1 >= kMaxRounds;
        if (last) hi = n_max;
        a.bound[r] = static_cast<int>(lo);
        a.bound[r + 1] = static_cast<int>(hi);
        if (last) break;
        lo = hi;
        hi *= shape.growth;
    }
    a.rounds = r + 1;
    for (int k = 0; k < 2; ++k) {
        a.words[k] = cb.words[k];
        a.index[k] = cb.index[k];
        a.match[k] = cb.match[k];
    }
    a.stride = cb.stride;
    a.state = d_state;
    a.err = d_err;
    a.timeout = g_barrier_ticks;
    a.L = StateLayout((cb.stride + group_size(refs->KS) - 1) / group_size(refs->KS));
    // Round 0: contiguous spans of whole block steps, at most kMaxRegions.
    const int64_t step = static_cast<int64_t>(kBlock) * r0_samples(refs->WR);
    const int64_t steps = (total + step - 1) / step;
    const int64_t span = (steps + kMaxRegions - 1) / kMaxRegions * step;
    const int grid0 = static_cast<int>((total + span - 1) / span);
    hipError_t e;
    switch (refs->WR) {
#define RSR_W_CASE(w) \
    case w: e = launch_r0<w>(st, seg, refs, a, grid0, span); break;
        RSR_W_CASE(1) RSR_W_CASE(2) RSR_W_CASE(3) RSR_W_CASE(4) RSR_W_CASE(5) RSR_W_CASE(6)
        RSR_W_CASE(8) RSR_W_CASE(10) RSR_W_CASE(12) RSR_W_CASE(16) RSR_W_CASE(20)
        RSR_W_CASE(24) RSR_W_CASE(32) RSR_W_CASE(40)
#undef RSR_W_CASE
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess || a.rounds == 1) return e;
    switch (refs->WR * 100 + refs->KS) {
#define RSR_WK_CASE(w, k) \
    case w * 100 + k: return launch_wk<w, k>(st, a, grid);
        RSR_WK_CASE(1, 1) RSR_WK_CASE(2, 1) RSR_WK_CASE(3, 2) RSR_WK_CASE(4, 2) RSR_WK_CASE(5, 3)
        RSR_WK_CASE(6, 3) RSR_WK_CASE(8, 4) RSR_WK_CASE(10, 5) RSR_WK_CASE(12, 6)
        RSR_WK_CASE(16, 7) RSR_WK_CASE(16, 8) RSR_WK_CASE(20, 9) RSR_WK_CASE(20, 10)
        RSR_WK_CASE(24, 11) RSR_WK_CASE(24, 12) RSR_WK_CASE(32, 13) RSR_WK_CASE(32, 14)
        RSR_WK_CASE(32, 15) RSR_WK_CASE(32, 16) RSR_WK_CASE(40, 17) RSR_WK_CASE(40, 18)
        RSR_WK_CASE(40, 19) RSR_WK_CASE(40, 20)
#undef RSR_WK_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rsr
