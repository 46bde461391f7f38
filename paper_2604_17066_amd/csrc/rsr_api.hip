// C ABI of the RSR Stage-2 library (declared in include/rsr.h): argument
// validation, handle construction (threshold computation, reference-row
// packing, graph upload), workspace management and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "rsr_internal.h"

using rsr::plane_words;
using rsr::sample_words;

namespace rsr {

// Allocations left before the injected failure (rsr_debug_fail_alloc); < 0:
// none armed.
static int64_t g_fail_countdown = -1;

static bool injected_failure() {
    if (g_fail_countdown < 0) return false;
    if (g_fail_countdown == 0) {
        g_fail_countdown = -1;
        return true;
    }
    --g_fail_countdown;
    return false;
}

hipError_t dev_malloc(void** p, size_t bytes) {
    if (injected_failure()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

hipError_t host_malloc(void** p, size_t bytes) {
    if (injected_failure()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipHostMalloc(p, bytes, hipHostMallocDefault);
}

rsr_status ensure_list(rsr_ctx* ctx, int64_t N) {
    if (ctx->ws.list_cap >= N) return RSR_OK;
    if (ctx->ws.list) {
        hipError_t e = hipFree(ctx->ws.list);
        ctx->ws.list = nullptr;
        ctx->ws.list_cap = 0;
        if (e != hipSuccess) return hip_error(ctx, e, "hipFree(unknown list)");
    }
    hipError_t e = dev_malloc(&ctx->ws.list, sizeof(int32_t) * static_cast<size_t>(N));
    if (e != hipSuccess) return hip_error(ctx, e, "unknown-sample list");
    ctx->ws.list_cap = N;
    return RSR_OK;
}

}  // namespace rsr

namespace {

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            changed = hipSetDevice(dev) == hipSuccess;
        }
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

rsr_status fail(rsr_ctx* ctx, rsr_status st, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return st;
}

rsr_status hip_fail(rsr_ctx* ctx, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    return fail(ctx, e == hipErrorOutOfMemory ? RSR_ENOMEM : RSR_EHIP, m);
}

#define RSR_HIP(ctx, call)                                  \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

rsr_status validate_probs(rsr_ctx* ctx, int32_t n, int32_t K, const double* p) {
    if (n <= 0 || K < 2) return fail(ctx, RSR_EINVAL, "n must be > 0 and K >= 2");
    if (K > RSR_MAX_K) return fail(ctx, RSR_EUNSUPPORTED, "K exceeds RSR_MAX_K");
    if (static_cast<int64_t>(n) * (K - 1) > RSR_MAX_BITS)
        return fail(ctx, RSR_EUNSUPPORTED, "n*(K-1) exceeds RSR_MAX_BITS");
    if (!p) return fail(ctx, RSR_EINVAL, "p is NULL");
    for (int32_t i = 0; i < n; ++i) {
        double sum = 0.0;
        for (int32_t s = 0; s < K; ++s) {
            const double v = p[static_cast<size_t>(i) * K + s];
            if (!std::isfinite(v) || v < 0.0 || v > 1.0)
                return fail(ctx, RSR_EINVAL,
                            "p[" + std::to_string(i) + "][" + std::to_string(s) + "] not in [0,1]");
            sum += v;
        }
        if (std::fabs(sum - 1.0) > 1e-9)
            return fail(ctx, RSR_EINVAL, "row " + std::to_string(i) + " of p does not sum to 1");
    }
    return RSR_OK;
}

// Inverse-CDF thresholds: C[i][s-1] = min(floor(2^32 * cumulative), 2^32),
// with the cumulative probability summed left to right in fp64.
void compute_thresholds(int32_t n, int32_t K, const double* p, uint64_t* C) {
    const double two32 = 4294967296.0;
    for (int32_t i = 0; i < n; ++i) {
        double cum = 0.0;
        for (int32_t s = 1; s < K; ++s) {
            cum = cum + p[static_cast<size_t>(i) * K + (s - 1)];
            const double f = std::floor(cum * two32);
            uint64_t c = 0;
            if (f >= two32)
                c = 4294967296ull;
            else if (f > 0.0)
                c = static_cast<uint64_t>(f);
            C[static_cast<size_t>(i) * (K - 1) + (s - 1)] = c;
        }
    }
}


// A reference set is consistent when no upper row lies below a lower row:
// then no sample can be dominated on both sides and the LABEL cascade may stop
// at the first match.  Checked once on the device with the classification
// kernels themselves (upper rows as samples against the lower rows): the FP4
// form when the handle has matrix-core operands (0.72 against 7.15 ms for the
// popcount form at 2.5e4 rows of 590 bits per side; its 2.5e4 samples fill a
// fifth of the CUs), else the popcount form.  Synchronous.
rsr_status check_consistency(rsr_ctx* ctx, rsr_refs* refs, const std::vector<uint32_t>& up) {
    refs->consistent = true;
    if (refs->R_L == 0 || refs->R_U == 0) return RSR_OK;
    const int64_t RU = refs->R_U;
    const int W = refs->W, WR = refs->WR;
    std::vector<uint32_t> cols(static_cast<size_t>(W) * RU);
    for (int64_t r = 0; r < RU; ++r)
        for (int w = 0; w < W; ++w) cols[static_cast<size_t>(w) * RU + r] = up[r * WR + w];
    uint32_t* d_cols = nullptr;
    uint8_t* d_flags = nullptr;
    hipError_t e = rsr::dev_malloc(&d_cols, sizeof(uint32_t) * cols.size());
    if (e == hipSuccess) e = rsr::dev_malloc(&d_flags, static_cast<size_t>(RU));
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_cols, cols.data(), sizeof(uint32_t) * cols.size(),
                           hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) {
        rsr_refs lower_only = *refs;
        lower_only.R_U = 0;
        lower_only.TU = 0;
        lower_only.d_upper_bits = nullptr;
        lower_only.d_upper_frag = nullptr;
        lower_only.d_upper_frag4 = nullptr;
        lower_only.d_upper_frag32 = nullptr;
        lower_only.d_upper_cinit = nullptr;
        lower_only.d_upper_cinit4 = nullptr;
        e = refs->KS > 0 ? rsr::launch_dom_mfma(ctx->stream, &lower_only, d_cols, RU, RSR_LABEL, true,
                                                ctx->cu_count, d_flags, nullptr)
                         : rsr::launch_dom_bits(ctx->stream, &lower_only, d_cols, RU, RSR_LABEL,
                                                d_flags, nullptr);
    }
    std::vector<uint8_t> fl(static_cast<size_t>(RU));
    if (e == hipSuccess)
        e = hipMemcpyAsync(fl.data(), d_flags, fl.size(), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (d_cols) (void)hipFree(d_cols);
    if (d_flags) (void)hipFree(d_flags);
    if (e != hipSuccess) return hip_fail(ctx, e, "reference consistency check");
    for (uint8_t f : fl)
        if (f & 1u) {
            refs->consistent = false;
            break;
        }
    return RSR_OK;
}

// Byte offsets of a model's device arrays in its single allocation (and in
// its pinned staging buffer): thresholds u64 [n][K-1], probabilities f64
// [n][K], sampler threshold halves i32 [ceil(n/8)*8][K-1][2], probabilities
// f32 [n][K].  Every offset is a multiple of 8.
struct ModelLayout {
    size_t thresh, p64, half, p32, total;
    ModelLayout(int n, int K) {
        const size_t nn = static_cast<size_t>(n), k1 = static_cast<size_t>(K - 1);
        const size_t n_pad = (nn + 7) / 8 * 8;
        thresh = 0;
        p64 = thresh + sizeof(uint64_t) * nn * k1;
        half = p64 + sizeof(double) * nn * K;
        p32 = half + sizeof(int32_t) * n_pad * k1 * 2;
        total = p32 + sizeof(float) * nn * K;
    }
};

// The host images of a model's arrays (p already validated).  The sampler
// form of a threshold C is a pair (gt, eq) on the high 16 bits of a uniform
// word u: u >= C is true when (u >> 16) > gt and needs the low half only when
// (u >> 16) == eq; padding components never set a bit.
void fill_model_stage(const ModelLayout& L, int n, int K, const double* p, void* stage) {
    char* base = static_cast<char*>(stage);
    uint64_t* C = reinterpret_cast<uint64_t*>(base + L.thresh);
    compute_thresholds(n, K, p, C);
    std::memcpy(base + L.p64, p, sizeof(double) * static_cast<size_t>(n) * K);
    int32_t* half = reinterpret_cast<int32_t*>(base + L.half);
    const size_t n_pad = (static_cast<size_t>(n) + 7) / 8 * 8;
    for (size_t i = 0; i < n_pad; ++i)
        for (int s = 0; s < K - 1; ++s) {
            int32_t gt = 0x7FFFFFFF, eq = -1;
            if (i < static_cast<size_t>(n)) {
                const uint64_t c = C[i * (K - 1) + s];
                const int32_t ch = static_cast<int32_t>(c >> 16);
                const bool low_zero = (c & 0xFFFFu) == 0;
                gt = low_zero ? ch - 1 : ch;
                eq = low_zero ? -1 : ch;
            }
            half[(i * (K - 1) + s) * 2] = gt;
            half[(i * (K - 1) + s) * 2 + 1] = eq;
        }
    float* pf = reinterpret_cast<float*>(base + L.p32);
    for (size_t i = 0; i < static_cast<size_t>(n) * K; ++i) pf[i] = static_cast<float>(p[i]);
}

rsr_status ensure_cascade(rsr_ctx* ctx, int W, int64_t N, int64_t state_words = 0) {
    const int64_t words = 2 * static_cast<int64_t>(W) * N, idx = 4 * N;
    if (ctx->ws.casc_state_cap < state_words) {
        if (ctx->ws.casc_state) RSR_HIP(ctx, hipFree(ctx->ws.casc_state));
        ctx->ws.casc_state = nullptr;
        ctx->ws.casc_state_cap = 0;
        // Rounded to whole u64 (the state is cleared 8 bytes at a time).
        const int64_t cap = (state_words + 1) / 2 * 2;
        RSR_HIP(ctx, rsr::dev_malloc(&ctx->ws.casc_state, sizeof(uint32_t) * static_cast<size_t>(cap)));
        ctx->ws.casc_state_cap = cap;
    }
    if (ctx->ws.casc_words_cap < words) {
        if (ctx->ws.casc_words) RSR_HIP(ctx, hipFree(ctx->ws.casc_words));
        ctx->ws.casc_words = nullptr;
        ctx->ws.casc_words_cap = 0;
        RSR_HIP(ctx, rsr::dev_malloc(&ctx->ws.casc_words, sizeof(uint32_t) * static_cast<size_t>(words)));
        ctx->ws.casc_words_cap = words;
    }
    if (ctx->ws.casc_index_cap < idx) {
        if (ctx->ws.casc_index) RSR_HIP(ctx, hipFree(ctx->ws.casc_index));
        ctx->ws.casc_index = nullptr;
        ctx->ws.casc_index_cap = 0;
        RSR_HIP(ctx, rsr::dev_malloc(&ctx->ws.casc_index, sizeof(int32_t) * static_cast<size_t>(idx)));
        ctx->ws.casc_index_cap = idx;
    }
    return RSR_OK;
}

}  // namespace

extern "C" {

const char* rsr_status_str(rsr_status s) {
    switch (s) {
        case RSR_OK: return "RSR_OK";
        case RSR_EINVAL: return "RSR_EINVAL";
        case RSR_ENOMEM: return "RSR_ENOMEM";
        case RSR_EHIP: return "RSR_EHIP";
        case RSR_EUNSUPPORTED: return "RSR_EUNSUPPORTED";
    }
    return "unknown status";
}

const char* rsr_last_error(const rsr_ctx* ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

size_t rsr_words(int32_t n, int32_t K) {
    if (n <= 0 || K < 2) return 0;
    return static_cast<size_t>(sample_words(n, K));
}

rsr_status rsr_thresholds(int32_t n, int32_t K, const double* p, uint64_t* C) {
    rsr_status st = validate_probs(nullptr, n, K, p);
    if (st != RSR_OK) return st;
    if (!C) return RSR_EINVAL;
    compute_thresholds(n, K, p, C);
    return RSR_OK;
}

rsr_status rsr_ctx_create(int device, void* hip_stream, rsr_ctx** out) {
    if (!out) return RSR_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return RSR_EHIP;
    if (device < 0 || device >= count) return RSR_EINVAL;
    rsr_ctx* ctx = new (std::nothrow) rsr_ctx();
    if (!ctx) return RSR_ENOMEM;
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    DeviceGuard g(device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete ctx;
        return RSR_EHIP;
    }
    ctx->cu_count = prop.multiProcessorCount;
    ctx->arch = prop.gcnArchName;
    rsr_status st = RSR_OK;
    if (rsr::dev_malloc(&ctx->ws.counters, sizeof(uint64_t) * 16) != hipSuccess ||
        rsr::dev_malloc(&ctx->ws.casc_counters,
                        sizeof(uint64_t) * rsr::CascadeBuffers::kCounterU64) != hipSuccess ||
        rsr::dev_malloc(&ctx->ws.count_part, sizeof(uint64_t) * rsr::kMaxReduceBlocks * 8) != hipSuccess ||
        rsr::dev_malloc(&ctx->ws.grad_part, sizeof(uint32_t) * (static_cast<size_t>(RSR_MAX_BITS) + 1) *
                                                rsr::kMaxGradBlocks) != hipSuccess ||
        rsr::host_malloc(&ctx->ws.host_counts, sizeof(uint64_t) * 16) != hipSuccess)
        st = RSR_ENOMEM;
    if (st == RSR_OK && hipHostGetDevicePointer(reinterpret_cast<void**>(&ctx->ws.host_counts_dev),
                                                ctx->ws.host_counts, 0) != hipSuccess)
        st = RSR_EHIP;
    if (st == RSR_OK && rsr::noalloc_scratch(device, &ctx->noalloc_scratch) != hipSuccess)
        st = RSR_EHIP;
    // counters[15] is the ticket of the one-launch counts kernel, which
    // expects it at zero and leaves it there.
    if (st == RSR_OK && hipMemset(ctx->ws.counters, 0, sizeof(uint64_t) * 16) != hipSuccess)
        st = RSR_EHIP;
    if (st != RSR_OK) {
        rsr_ctx_destroy(ctx);
        return st;
    }
    *out = ctx;
    return RSR_OK;
}

rsr_status rsr_ctx_destroy(rsr_ctx* ctx) {
    if (!ctx) return RSR_EINVAL;
    DeviceGuard g(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    if (ctx->ws.counters) (void)hipFree(ctx->ws.counters);
    if (ctx->ws.casc_counters) (void)hipFree(ctx->ws.casc_counters);
    if (ctx->ws.casc_words) (void)hipFree(ctx->ws.casc_words);
    if (ctx->ws.casc_index) (void)hipFree(ctx->ws.casc_index);
    if (ctx->ws.casc_state) (void)hipFree(ctx->ws.casc_state);
    if (ctx->ws.list) (void)hipFree(ctx->ws.list);
    if (ctx->ws.count_part) (void)hipFree(ctx->ws.count_part);
    if (ctx->ws.grad_part) (void)hipFree(ctx->ws.grad_part);
    if (ctx->ws.host_counts) (void)hipHostFree(ctx->ws.host_counts);
    const rsr::CallbackStage& cb = ctx->ws.cb;
    if (cb.d_words) (void)hipFree(cb.d_words);
    if (cb.d_bytes) (void)hipFree(cb.d_bytes);
    if (cb.h_words) (void)hipHostFree(cb.h_words);
    if (cb.h_bytes) (void)hipHostFree(cb.h_bytes);
    if (cb.h_index) (void)hipHostFree(cb.h_index);
    delete ctx;
    return RSR_OK;
}

// ---- handles ---------------------------------------------------------------

rsr_status rsr_model_create(rsr_ctx* ctx, int32_t n, int32_t K, const double* p,
                            rsr_model** out) {
    if (!ctx || !out) return RSR_EINVAL;
    *out = nullptr;
    rsr_status st = validate_probs(ctx, n, K, p);
    if (st != RSR_OK) return st;
    DeviceGuard g(ctx->device);
    rsr_model* m = new (std::nothrow) rsr_model();
    if (!m) return fail(ctx, RSR_ENOMEM, "host allocation");
    m->ctx = ctx;
    m->n = n;
    m->K = K;
    const ModelLayout L(n, K);
    m->mem_bytes = L.total;
    hipError_t e = rsr::dev_malloc(&m->d_mem, L.total);
    if (e == hipSuccess) e = rsr::host_malloc(&m->h_stage, L.total);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&m->staged, hipEventDisableTiming);
    if (e != hipSuccess) {
        rsr_model_destroy(m);
        return hip_fail(ctx, e, "rsr_model_create allocation");
    }
    char* base = static_cast<char*>(m->d_mem);
    m->d_thresh = reinterpret_cast<uint64_t*>(base + L.thresh);
    m->d_p64 = reinterpret_cast<double*>(base + L.p64);
    m->d_half = reinterpret_cast<int32_t*>(base + L.half);
    m->d_p = reinterpret_cast<float*>(base + L.p32);
    fill_model_stage(L, n, K, p, m->h_stage);
    e = hipMemcpyAsync(m->d_mem, m->h_stage, L.total, hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipEventRecord(m->staged, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(m->staged);
    if (e != hipSuccess) {
        rsr_model_destroy(m);
        return hip_fail(ctx, e, "rsr_model_create upload");
    }
    *out = m;
    return RSR_OK;
}

rsr_status rsr_model_update(rsr_model* m, const double* p) {
    if (!m) return RSR_EINVAL;
    rsr_ctx* ctx = m->ctx;
    rsr_status st = validate_probs(ctx, m->n, m->K, p);
    if (st != RSR_OK) return st;
    DeviceGuard g(ctx->device);
    // The previous upload must have left the staging buffer before it is
    // overwritten (normally long done: any synchronising call since then
    // has waited for it).
    RSR_HIP(ctx, hipEventSynchronize(m->staged));
    fill_model_stage(ModelLayout(m->n, m->K), m->n, m->K, p, m->h_stage);
    RSR_HIP(ctx, hipMemcpyAsync(m->d_mem, m->h_stage, m->mem_bytes, hipMemcpyHostToDevice,
                                ctx->stream));
    RSR_HIP(ctx, hipEventRecord(m->staged, ctx->stream));
    return RSR_OK;
}

rsr_status rsr_model_destroy(rsr_model* m) {
    if (!m) return RSR_EINVAL;
    DeviceGuard g(m->ctx->device);
    if (m->staged) {
        (void)hipEventSynchronize(m->staged);
        (void)hipEventDestroy(m->staged);
    }
    if (m->d_mem) (void)hipFree(m->d_mem);
    if (m->h_stage) (void)hipHostFree(m->h_stage);
    delete m;
    return RSR_OK;
}

}  // extern "C"

namespace rsr {

rsr_status refs_create(rsr_ctx* ctx, int32_t n, int32_t K, const uint8_t* lower, int64_t R_L,
                       const uint8_t* upper, int64_t R_U, bool matrix_operands, rsr_refs** out) {
    if (!ctx || !out) return RSR_EINVAL;
    *out = nullptr;
    if (n <= 0 || K < 2) return fail(ctx, RSR_EINVAL, "n must be > 0 and K >= 2");
    if (K > RSR_MAX_K || static_cast<int64_t>(n) * (K - 1) > RSR_MAX_BITS)
        return fail(ctx, RSR_EUNSUPPORTED, "n*(K-1) exceeds RSR_MAX_BITS or K > RSR_MAX_K");
    if (R_L < 0 || R_U < 0) return fail(ctx, RSR_EINVAL, "negative row count");
    if ((R_L > 0 && !lower) || (R_U > 0 && !upper))
        return fail(ctx, RSR_EINVAL, "NULL reference rows with a non-zero count");
    for (int64_t k = 0; k < R_L * n; ++k)
        if (lower[k] >= K) return fail(ctx, RSR_EINVAL, "lower reference state >= K");
    for (int64_t k = 0; k < R_U * n; ++k)
        if (upper[k] >= K) return fail(ctx, RSR_EINVAL, "upper reference state >= K");
    DeviceGuard g(ctx->device);
    const int PW = plane_words(n);
    const int W = sample_words(n, K);
    const int WR = rsr::dom_row_words(W);
    if (WR < 0) return fail(ctx, RSR_EUNSUPPORTED, "packed width not supported");
    // Valid-bit mask per packed word (pad bits of each plane are 0).
    std::vector<uint32_t> valid(W, 0u);
    for (int j = 1; j < K; ++j)
        for (int i = 0; i < n; ++i) valid[(j - 1) * PW + i / 32] |= 1u << (i % 32);
    auto pack = [&](const uint8_t* row, uint32_t* dst, bool complement) {
        for (int w = 0; w < WR; ++w) dst[w] = 0u;
        for (int j = 1; j < K; ++j)
            for (int i = 0; i < n; ++i)
                if (row[i] >= j) dst[(j - 1) * PW + i / 32] |= 1u << (i % 32);
        if (complement)
            for (int w = 0; w < W; ++w) dst[w] = ~dst[w] & valid[w];
    };
    std::vector<uint32_t> lo(static_cast<size_t>(R_L) * WR), up(static_cast<size_t>(R_U) * WR);
    for (int64_t r = 0; r < R_L; ++r) pack(lower + r * n, lo.data() + r * WR, true);
    for (int64_t r = 0; r < R_U; ++r) pack(upper + r * n, up.data() + r * WR, false);
    // Store rows by increasing number of violation bits (stable): a row with
    // fewer constrained components dominates a larger region, so the LABEL
    // cascade finds most matches among the first rows.  Results do not depend
    // on the order.
    auto sort_rows = [&](std::vector<uint32_t>& rows, int64_t R) {
        std::vector<int64_t> order(R);
        std::vector<int> weight(R);
        for (int64_t r = 0; r < R; ++r) {
            order[r] = r;
            int c = 0;
            for (int w = 0; w < W; ++w) c += __builtin_popcount(rows[r * WR + w]);
            weight[r] = c;
        }
        std::stable_sort(order.begin(), order.end(),
                         [&](int64_t a, int64_t b) { return weight[a] < weight[b]; });
        std::vector<uint32_t> sorted(rows.size());
        for (int64_t r = 0; r < R; ++r)
            std::copy(rows.begin() + order[r] * WR, rows.begin() + (order[r] + 1) * WR,
                      sorted.begin() + r * WR);
        rows.swap(sorted);
    };
    sort_rows(lo, R_L);
    sort_rows(up, R_U);

    // Matrix-core operands: fragment-ordered bytes and accumulator starts,
    // chosen so that a row matches exactly when its accumulator is negative.
    // Lower rows: bytes NOT t(r) in {0, 1}, start -1, so the result is
    // |t(x) & ~t(r)| - 1.  Upper rows: bytes -t(r) in {0, -1}, start
    // |t(r)| - 1, so the result is |t(r) & ~t(x)| - 1.  Pad rows and pad
    // tiles are all zero: result 0, never a match.
    const int KS = (W * 32 + 63) / 64;
    const bool with_mfma = matrix_operands && KS <= rsr::kMaxMfmaSteps;
    const int TL = static_cast<int>((R_L + 15) / 16), TU = static_cast<int>((R_U + 15) / 16);
    const int KS4 = (W * 32 + 127) / 128;
    std::vector<int8_t> lof, upf;
    std::vector<int32_t> loc, upc;
    std::vector<uint8_t> lof4, upf4, lof32, upf32;
    std::vector<float> loc4, upc4;
    if (with_mfma) {
        auto frag = [&](const uint32_t* words, int64_t r, int8_t value, std::vector<int8_t>& dst) {
            const int64_t T = r / 16;
            const int rr = static_cast<int>(r % 16);
            for (int k = 0; k < W * 32; ++k) {
                if (!((words[k / 32] >> (k % 32)) & 1u)) continue;
                const int s = k / 64, o = k % 64;
                const int lane = (o / 16) * 16 + rr;
                dst[((static_cast<size_t>(T) * KS + s) * 64 + lane) * 16 + (o % 16)] = value;
            }
        };
        lof.assign(static_cast<size_t>(TL) * KS * 1024, 0);
        upf.assign(static_cast<size_t>(TU) * KS * 1024, 0);
        loc.assign(static_cast<size_t>(TL) * 16, 0);
        upc.assign(static_cast<size_t>(TU) * 16, 0);
        for (int64_t r = 0; r < R_L; ++r) {
            frag(lo.data() + r * WR, r, 1, lof);
            loc[r] = -1;
        }
        for (int64_t r = 0; r < R_U; ++r) {
            frag(up.data() + r * WR, r, -1, upf);
            int pop = 0;
            for (int w = 0; w < W; ++w) pop += __builtin_popcount(up[r * WR + w]);
            upc[r] = pop - 1;
        }
        // FP4 operands: 128 k per step; lane (group g, row rr) holds nibbles
        // j = 0..31 for k = 128 s + 32 g + j, two per byte, low nibble first.
        auto frag4 = [&](const uint32_t* words, int64_t r, uint8_t nib, std::vector<uint8_t>& dst) {
            const int64_t T = r / 16;
            const int rr = static_cast<int>(r % 16);
            for (int k = 0; k < W * 32; ++k) {
                if (!((words[k / 32] >> (k % 32)) & 1u)) continue;
                const int s = k / 128, o = k % 128;
                const int lane = (o / 32) * 16 + rr, j = o % 32;
                dst[((static_cast<size_t>(T) * KS4 + s) * 64 + lane) * 16 + j / 2] |=
                    static_cast<uint8_t>(nib << (4 * (j % 2)));
            }
        };
        lof4.assign(static_cast<size_t>(TL) * KS4 * 1024, 0);
        upf4.assign(static_cast<size_t>(TU) * KS4 * 1024, 0);
        loc4.assign(static_cast<size_t>(TL) * 16, 0.5f);
        upc4.assign(static_cast<size_t>(TU) * 16, 0.5f);
        for (int64_t r = 0; r < R_L; ++r) {
            frag4(lo.data() + r * WR, r, 0x2, lof4);  // +1.0
            loc4[r] = -0.5f;
        }
        for (int64_t r = 0; r < R_U; ++r) {
            frag4(up.data() + r * WR, r, 0xA, upf4);  // -1.0
            upc4[r] = static_cast<float>(upc[r]) + 0.5f;  // |t(r)| - 0.5
        }
        // FP4 operands on 32-row tiles: 64 k per step; lane (half h, row rr)
        // holds nibbles j = 0..31 for k = 64 s + 32 h + j.  Both sides are +1
        // nibbles (NOT t(r) for lower rows, t(r) for upper rows); the kernel
        // starts every row at -1/2 and contracts upper rows with the
        // complemented samples.
        auto frag32 = [&](const uint32_t* words, int64_t r, std::vector<uint8_t>& dst) {
            const int64_t T = r / 32;
            const int rr = static_cast<int>(r % 32);
            for (int k = 0; k < W * 32; ++k) {
                if (!((words[k / 32] >> (k % 32)) & 1u)) continue;
                const int s = k / 64, o = k % 64;
                const int lane = (o / 32) * 32 + rr, j = o % 32;
                dst[((static_cast<size_t>(T) * KS + s) * 64 + lane) * 16 + j / 2] |=
                    static_cast<uint8_t>(0x2 << (4 * (j % 2)));
            }
        };
        const int64_t TL32 = (R_L + 31) / 32, TU32 = (R_U + 31) / 32;
        lof32.assign(static_cast<size_t>(TL32) * KS * 1024, 0);
        upf32.assign(static_cast<size_t>(TU32) * KS * 1024, 0);
        for (int64_t r = 0; r < R_L; ++r) frag32(lo.data() + r * WR, r, lof32);
        for (int64_t r = 0; r < R_U; ++r) frag32(up.data() + r * WR, r, upf32);
    }

    rsr_refs* refs = new (std::nothrow) rsr_refs();
    if (!refs) return fail(ctx, RSR_ENOMEM, "host allocation");
    refs->ctx = ctx;
    refs->n = n;
    refs->K = K;
    refs->W = W;
    refs->WR = WR;
    refs->R_L = R_L;
    refs->R_U = R_U;
    hipError_t e = hipSuccess;
    auto upload = [&](void** dst, const void* src, size_t bytes) {
        if (e != hipSuccess || bytes == 0) return;
        e = rsr::dev_malloc(dst, bytes);
        if (e == hipSuccess) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    };
    upload(reinterpret_cast<void**>(&refs->d_lower_nbits), lo.data(), sizeof(uint32_t) * lo.size());
    upload(reinterpret_cast<void**>(&refs->d_upper_bits), up.data(), sizeof(uint32_t) * up.size());
    if (with_mfma) {
        refs->KS = KS;
        refs->TL = TL;
        refs->TU = TU;
        upload(reinterpret_cast<void**>(&refs->d_lower_frag), lof.data(), lof.size());
        upload(reinterpret_cast<void**>(&refs->d_lower_cinit), loc.data(), sizeof(int32_t) * loc.size());
        upload(reinterpret_cast<void**>(&refs->d_upper_frag), upf.data(), upf.size());
        upload(reinterpret_cast<void**>(&refs->d_upper_cinit), upc.data(), sizeof(int32_t) * upc.size());
        upload(reinterpret_cast<void**>(&refs->d_lower_frag32), lof32.data(), lof32.size());
        upload(reinterpret_cast<void**>(&refs->d_upper_frag32), upf32.data(), upf32.size());
        refs->KS4 = KS4;
        upload(reinterpret_cast<void**>(&refs->d_lower_frag4), lof4.data(), lof4.size());
        upload(reinterpret_cast<void**>(&refs->d_lower_cinit4), loc4.data(), sizeof(float) * loc4.size());
        upload(reinterpret_cast<void**>(&refs->d_upper_frag4), upf4.data(), upf4.size());
        upload(reinterpret_cast<void**>(&refs->d_upper_cinit4), upc4.data(), sizeof(float) * upc4.size());
    }
    if (e != hipSuccess) {
        rsr_refs_destroy(refs);
        return hip_fail(ctx, e, "rsr_refs_create upload");
    }
    rsr_status st = check_consistency(ctx, refs, up);
    if (st != RSR_OK) {
        rsr_refs_destroy(refs);
        return st;
    }
    *out = refs;
    return RSR_OK;
}

}  // namespace rsr

extern "C" {

rsr_status rsr_refs_consistent(const rsr_refs* refs, int32_t* out) {
    if (!refs || !out) return RSR_EINVAL;
    *out = refs->consistent ? 1 : 0;
    return RSR_OK;
}

rsr_status rsr_refs_create(rsr_ctx* ctx, int32_t n, int32_t K, const uint8_t* lower, int64_t R_L,
                           const uint8_t* upper, int64_t R_U, rsr_refs** out) {
    return rsr::refs_create(ctx, n, K, lower, R_L, upper, R_U, true, out);
}

rsr_status rsr_refs_destroy(rsr_refs* refs) {
    if (!refs) return RSR_EINVAL;
    DeviceGuard g(refs->ctx->device);
    if (refs->d_lower_nbits) (void)hipFree(refs->d_lower_nbits);
    if (refs->d_upper_bits) (void)hipFree(refs->d_upper_bits);
    if (refs->d_lower_frag) (void)hipFree(refs->d_lower_frag);
    if (refs->d_lower_cinit) (void)hipFree(refs->d_lower_cinit);
    if (refs->d_upper_frag) (void)hipFree(refs->d_upper_frag);
    if (refs->d_upper_cinit) (void)hipFree(refs->d_upper_cinit);
    if (refs->d_lower_frag4) (void)hipFree(refs->d_lower_frag4);
    if (refs->d_lower_cinit4) (void)hipFree(refs->d_lower_cinit4);
    if (refs->d_upper_frag4) (void)hipFree(refs->d_upper_frag4);
    if (refs->d_upper_cinit4) (void)hipFree(refs->d_upper_cinit4);
    if (refs->d_lower_frag32) (void)hipFree(refs->d_lower_frag32);
    if (refs->d_upper_frag32) (void)hipFree(refs->d_upper_frag32);
    delete refs;
    return RSR_OK;
}

rsr_status rsr_system_create(rsr_ctx* ctx, const rsr_system_desc* d, rsr_system** out) {
    if (!ctx || !out || !d) return RSR_EINVAL;
    *out = nullptr;
    if (d->kind == RSR_SYS_HOST_CALLBACK) {
        if (!d->phi) return fail(ctx, RSR_EINVAL, "RSR_SYS_HOST_CALLBACK without phi");
        if (d->n_edges <= 0 || d->K < 2) return fail(ctx, RSR_EINVAL, "n must be > 0 and K >= 2");
        if (d->K > RSR_MAX_K || static_cast<int64_t>(d->n_edges) * (d->K - 1) > RSR_MAX_BITS)
            return fail(ctx, RSR_EUNSUPPORTED, "n*(K-1) exceeds RSR_MAX_BITS or K > RSR_MAX_K");
        if (d->level < 1) return fail(ctx, RSR_EINVAL, "level must be >= 1");
        rsr_system* s = new (std::nothrow) rsr_system();
        if (!s) return fail(ctx, RSR_ENOMEM, "host allocation");
        s->ctx = ctx;
        s->kind = d->kind;
        s->n_edges = d->n_edges;
        s->K = d->K;
        s->level = d->level;
        s->phi = d->phi;
        s->user = d->user;
        *out = s;
        return RSR_OK;
    }
    if (d->kind != RSR_SYS_ST_CONNECTIVITY && d->kind != RSR_SYS_GLOBAL_CONNECTIVITY &&
        d->kind != RSR_SYS_MAX_FLOW)
        return fail(ctx, RSR_EINVAL, "unknown system kind");
    const bool global = d->kind == RSR_SYS_GLOBAL_CONNECTIVITY;
    const bool flow = d->kind == RSR_SYS_MAX_FLOW;
    if (d->n_nodes < 2 || d->n_edges <= 0 || d->K < 2 || !d->edge_u || !d->edge_v)
        return fail(ctx, RSR_EINVAL, "bad graph size or NULL edge arrays");
    if (d->n_nodes > RSR_MAX_NODES || d->K > RSR_MAX_K ||
        static_cast<int64_t>(d->n_edges) * (d->K - 1) > RSR_MAX_BITS)
        return fail(ctx, RSR_EUNSUPPORTED, "graph exceeds RSR_MAX_NODES / RSR_MAX_BITS");
    if (global) {
        if (d->level < 1 || d->level > 2) return fail(ctx, RSR_EINVAL, "level not in 1..2");
        // Edge list plus four waves' node sets, parents and depths in 64 KB of LDS.
        const int64_t words = d->n_edges + 4ll * (((d->n_nodes + 31) >> 5) + ((d->n_edges + 31) >> 5) +
                                                   2 * ((d->n_nodes + 1) >> 1));
        if (words * 4 > 64 * 1024)
            return fail(ctx, RSR_EUNSUPPORTED, "graph too large for the global-connectivity search");
    } else {
        if (d->source < 0 || d->source >= d->n_nodes || d->sink < 0 || d->sink >= d->n_nodes ||
            d->source == d->sink)
            return fail(ctx, RSR_EINVAL, "source/sink out of range or equal");
        if (flow ? (d->level < 1 || d->level > 255) : (d->level < 1 || d->level > d->K - 1))
            return fail(ctx, RSR_EINVAL, flow ? "demand not in 1..255" : "level not in 1..K-1");
        if (flow) {
            // Edge list plus four waves' marks, parents, capacities and flows in 64 KB.
            const int64_t words = d->n_edges + 4ll * (((d->n_nodes + 31) >> 5) + ((d->n_nodes + 1) >> 1) +
                                                       3 * ((d->n_edges + 3) >> 2));
            if (words * 4 > 64 * 1024)
                return fail(ctx, RSR_EUNSUPPORTED, "graph too large for the max-flow search");
        }
    }
    std::vector<uint32_t> packed(d->n_edges);
    for (int e = 0; e < d->n_edges; ++e) {
        const int32_t u = d->edge_u[e], v = d->edge_v[e];
        if (u < 0 || u >= d->n_nodes || v < 0 || v >= d->n_nodes)
            return fail(ctx, RSR_EINVAL, "edge endpoint out of range");
        packed[e] = static_cast<uint32_t>(u) | (static_cast<uint32_t>(v) << 16);
    }
    DeviceGuard g(ctx->device);
    rsr_system* s = new (std::nothrow) rsr_system();
    if (!s) return fail(ctx, RSR_ENOMEM, "host allocation");
    s->ctx = ctx;
    s->kind = d->kind;
    s->n_nodes = d->n_nodes;
    s->n_edges = d->n_edges;
    s->K = d->K;
    s->level = d->level;
    s->source = global ? 0 : d->source;
    s->sink = global ? 0 : d->sink;
    hipError_t e = rsr::dev_malloc(&s->d_edges, sizeof(uint32_t) * packed.size());
    if (e == hipSuccess)
        e = hipMemcpy(s->d_edges, packed.data(), sizeof(uint32_t) * packed.size(),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        rsr_system_destroy(s);
        return hip_fail(ctx, e, "rsr_system_create upload");
    }
    *out = s;
    return RSR_OK;
}

rsr_status rsr_system_destroy(rsr_system* s) {
    if (!s) return RSR_EINVAL;
    DeviceGuard g(s->ctx->device);
    if (s->d_edges) (void)hipFree(s->d_edges);
    delete s;
    return RSR_OK;
}

// ---- hot path ----------------------------------------------------------------

rsr_status rsr_sample(rsr_ctx* ctx, const rsr_model* model, uint64_t seed, uint32_t stream_id,
                      uint64_t first_sample, int64_t N, uint32_t* d_samples) {
    if (!ctx) return RSR_EINVAL;
    if (!model || !d_samples) return fail(ctx, RSR_EINVAL, "NULL model or d_samples");
    if (N <= 0) return fail(ctx, RSR_EINVAL, "N must be > 0");
    DeviceGuard g(ctx->device);
    RSR_HIP(ctx, rsr::launch_sample(ctx->stream, model, seed, stream_id, first_sample, N, d_samples));
    return RSR_OK;
}

rsr_status rsr_classify(rsr_ctx* ctx, const rsr_refs* refs, const uint32_t* d_samples, int64_t N,
                        int32_t mode, int32_t form, uint8_t* d_flags, uint32_t* d_match) {
    if (!ctx) return RSR_EINVAL;
    if (!refs || !d_samples || !d_flags) return fail(ctx, RSR_EINVAL, "NULL argument");
    if (N <= 0) return fail(ctx, RSR_EINVAL, "N must be > 0");
    if (mode != RSR_LABEL && mode != RSR_COUNT) return fail(ctx, RSR_EINVAL, "bad mode");
    if (form != RSR_AUTO && form != RSR_POPCOUNT && form != RSR_MFMA && form != RSR_MFMA_FP4 &&
        form != RSR_PERSIST)
        return fail(ctx, RSR_EINVAL, "bad form");
    if (refs->ctx->device != ctx->device) return fail(ctx, RSR_EINVAL, "refs on another device");
    DeviceGuard g(ctx->device);
    if ((form == RSR_MFMA && refs->KS == 0) ||
        ((form == RSR_MFMA_FP4 || form == RSR_PERSIST) && refs->KS4 == 0))
        return fail(ctx, RSR_EUNSUPPORTED, "matrix-core form needs n*(K-1) <= 1280");
    if (form == RSR_PERSIST &&
        (mode != RSR_LABEL || !refs->consistent || N > 0x7FFFFFFFll || !rsr::casc_persist_supported(refs)))
        return fail(ctx, RSR_EUNSUPPORTED,
                    "the persistent cascade takes LABEL mode on consistent rows, N <= 2^31-1");
    uint32_t* match = mode == RSR_COUNT ? d_match : nullptr;
    // RSR_AUTO: the cascade for LABEL on consistent rows (each sample stops at
    // its first match); otherwise the FP4 matrix-core form, which makes the
    // most tests per second in both modes; popcount beyond 1280 bits.
    if (form == RSR_AUTO && refs->KS4 > 0 && (mode == RSR_COUNT || !refs->consistent))
        form = RSR_MFMA_FP4;
    const bool matrix = form == RSR_MFMA || form == RSR_MFMA_FP4;
    if (mode == RSR_LABEL && !matrix && refs->consistent && N <= 0x7FFFFFFFll) {
        // RSR_PERSIST runs the rounds after round 0 in one persistent
        // launch; the automatic and popcount forms run one launch per round.
        const int64_t n_max = refs->R_L > refs->R_U ? refs->R_L : refs->R_U;
        const bool persist = form == RSR_PERSIST;
        const int64_t stride = persist ? rsr::casc_persist_stride(refs, N, ctx->cu_count) : N;
        const int64_t state_words = persist ? rsr::casc_persist_state_words(stride, refs->KS) : 0;
        rsr_status st = ensure_cascade(ctx, refs->W, stride, state_words);
        if (st != RSR_OK) return st;
        rsr::CascadeBuffers cb;
        cb.words[0] = ctx->ws.casc_words;
        cb.words[1] = ctx->ws.casc_words + static_cast<int64_t>(refs->W) * stride;
        cb.index[0] = ctx->ws.casc_index;
        cb.index[1] = ctx->ws.casc_index + stride;
        cb.match[0] = reinterpret_cast<uint32_t*>(ctx->ws.casc_index + 2 * stride);
        cb.match[1] = reinterpret_cast<uint32_t*>(ctx->ws.casc_index + 3 * stride);
        cb.stride = stride;
        cb.counters = ctx->ws.casc_counters;
        cb.regions = reinterpret_cast<uint32_t*>(ctx->ws.casc_counters + 16);
        // The automatic form runs the rounds after round 0 in the FP4
        // matrix-core form when the handle has its operands, with faster
        // growing rounds from kWideRows rows per side on; the popcount form
        // stays popcount.
        const rsr::CascadeShape shape = form != RSR_AUTO || refs->KS4 == 0 ? rsr::CascadeShape{}
                                        : n_max >= rsr::kWideRows        ? rsr::mfma_wide_shape()
                                                                         : rsr::mfma_tail_shape();
        if (persist) {
            RSR_HIP(ctx, rsr::launch_fill_u64(ctx->stream, reinterpret_cast<uint64_t*>(ctx->ws.casc_state),
                                              (state_words + 1) / 2, 0));
            RSR_HIP(ctx, rsr::launch_casc_persist(ctx->stream, refs,
                                                  rsr::single_src(d_samples, N, d_flags, nullptr), cb,
                                                  rsr::mfma_head_shape(), ctx->ws.casc_state,
                                                  reinterpret_cast<unsigned long long*>(ctx->ws.counters + 14),
                                                  ctx->cu_count));
            return RSR_OK;
        }
        RSR_HIP(ctx, rsr::launch_fill_u64(ctx->stream, cb.counters, rsr::CascadeBuffers::kMaxRounds, 0));
        RSR_HIP(ctx, rsr::launch_dom_cascade(ctx->stream, refs,
                                             rsr::single_src(d_samples, N, d_flags, nullptr), cb,
                                             shape, ctx->cu_count * 8));
        return RSR_OK;
    }
    if (matrix)
        RSR_HIP(ctx, rsr::launch_dom_mfma(ctx->stream, refs, d_samples, N, mode,
                                          form == RSR_MFMA_FP4, ctx->cu_count, d_flags,
                                          match));
    else
        RSR_HIP(ctx, rsr::launch_dom_bits(ctx->stream, refs, d_samples, N, mode, d_flags, match));
    return RSR_OK;
}

rsr_status rsr_eval_unknown(rsr_ctx* ctx, const rsr_system* sys, const uint32_t* d_samples,
                            int64_t N, const uint8_t* d_flags, int32_t which, uint8_t* d_Y,
                            uint64_t* d_n_evaluated) {
    if (!ctx) return RSR_EINVAL;
    if (!sys || !d_samples || !d_Y) return fail(ctx, RSR_EINVAL, "NULL argument");
    if (N <= 0 || N > 0x7FFFFFFFll) return fail(ctx, RSR_EINVAL, "N must be in 1..2^31-1");
    if (which != RSR_UNKNOWN_ONLY && which != RSR_ALL) return fail(ctx, RSR_EINVAL, "bad which");
    if (which == RSR_UNKNOWN_ONLY && !d_flags)
        return fail(ctx, RSR_EINVAL, "d_flags is NULL with RSR_UNKNOWN_ONLY");
    DeviceGuard g(ctx->device);
    if (sys->kind == RSR_SYS_HOST_CALLBACK)
        return rsr::eval_callback(ctx, sys, d_samples, N, d_flags, which, d_Y, d_n_evaluated);
    uint64_t* counter = ctx->ws.counters + 8;
    const rsr::SegSrc seg = rsr::single_src(d_samples, N, const_cast<uint8_t*>(d_flags), d_Y);
    if (which == RSR_UNKNOWN_ONLY) {
        rsr_status st = rsr::ensure_list(ctx, N);
        if (st != RSR_OK) return st;
        RSR_HIP(ctx, rsr::launch_fill_u64(ctx->stream, counter, 1, 0));
        RSR_HIP(ctx, rsr::launch_label(ctx->stream, seg, ctx->ws.list, counter, ctx->cu_count * 16));
    }
    RSR_HIP(ctx, rsr::launch_bfs(ctx->stream, sys, seg, ctx->ws.list, counter, which,
                                 d_n_evaluated, ctx->cu_count * 8));
    return RSR_OK;
}

rsr_status rsr_boundary_search(rsr_ctx* ctx, const rsr_system* sys, const uint32_t* d_samples,
                               int64_t N, const int64_t* d_pick, int64_t n_pick,
                               uint8_t* d_rows, uint8_t* d_side) {
    if (!ctx) return RSR_EINVAL;
    if (n_pick < 0) return fail(ctx, RSR_EINVAL, "n_pick must be >= 0");
    if (n_pick == 0) return RSR_OK;
    if (!sys || !d_samples || !d_pick || !d_rows || !d_side)
        return fail(ctx, RSR_EINVAL, "NULL argument");
    if (N <= 0 || N > 0x7FFFFFFFll) return fail(ctx, RSR_EINVAL, "N must be in 1..2^31-1");
    if (sys->kind == RSR_SYS_HOST_CALLBACK) {
        DeviceGuard g(ctx->device);
        return rsr::boundary_callback(ctx, sys, d_samples, N, d_pick, n_pick, d_rows, d_side);
    }
    if (rsr::boundary_lds_bytes(sys) > 64 * 1024)
        return fail(ctx, RSR_EUNSUPPORTED, "graph too large for the boundary search");
    DeviceGuard g(ctx->device);
    RSR_HIP(ctx, rsr::launch_boundary(ctx->stream, sys, d_samples, N, d_pick, n_pick, d_rows,
                                      d_side, ctx->cu_count * 8));
    return RSR_OK;
}

rsr_status rsr_estimate(rsr_ctx* ctx, const uint8_t* d_flags, const uint8_t* d_Y, int64_t N,
                        rsr_estimate_t* out) {
    if (!ctx) return RSR_EINVAL;
    if (!d_flags || !out) return fail(ctx, RSR_EINVAL, "NULL argument");
    if (N <= 0) return fail(ctx, RSR_EINVAL, "N must be > 0");
    DeviceGuard g(ctx->device);
    const bool aligned = (reinterpret_cast<uintptr_t>(d_flags) & 15u) == 0 &&
                         (reinterpret_cast<uintptr_t>(d_Y) & 15u) == 0;
    // host_counts[0..4] receive the counts and host_counts[5] the persistent
    // cascade's time-out flag (counters[14]); the one-launch kernel writes
    // them into the pinned buffer itself, the other path through a copy.
    uint64_t* c = ctx->ws.host_counts;
    if (aligned) {
        // The kernel's last block stores this call's sequence number into
        // c[6] after the counts (system-scope release), once every earlier
        // kernel of the stream and every other block of its own have ended:
        // the host returns as soon as it sees it, instead of waiting for the
        // end-of-kernel signal.  Past 10 ms of polling (a long queue ahead of
        // the counts) it synchronises the stream.
        const uint64_t seq = ++ctx->ws.estimate_seq;
        __atomic_store_n(&c[6], uint64_t{0}, __ATOMIC_RELAXED);
        RSR_HIP(ctx, rsr::launch_counts_vec(ctx->stream, d_flags, d_Y, N, ctx->ws.host_counts_dev,
                                            ctx->ws.count_part,
                                            reinterpret_cast<uint32_t*>(ctx->ws.counters + 15),
                                            ctx->ws.counters + 14, seq));
        const auto t0 = std::chrono::steady_clock::now();
        bool seen = false;
        for (uint32_t it = 1;; ++it) {
            if (__atomic_load_n(&c[6], __ATOMIC_ACQUIRE) == seq) {
                seen = true;
                break;
            }
            if ((it & 255u) == 0 &&
                std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(10))
                break;
        }
        if (!seen) RSR_HIP(ctx, hipStreamSynchronize(ctx->stream));
    } else {
        RSR_HIP(ctx, rsr::launch_counts(ctx->stream, d_flags, d_Y, N, ctx->ws.counters,
                                        ctx->ws.count_part));
        RSR_HIP(ctx, hipMemcpyAsync(c, ctx->ws.counters, sizeof(uint64_t) * 16,
                                    hipMemcpyDeviceToHost, ctx->stream));
        RSR_HIP(ctx, hipStreamSynchronize(ctx->stream));
        c[5] = c[14];
    }
    if (c[5] != 0) {
        // A persistent cascade since the last check could not synchronise its
        // blocks in time: its flags are not to be trusted.
        RSR_HIP(ctx, rsr::launch_fill_u64(ctx->stream, ctx->ws.counters + 14, 1, 0));
        return fail(ctx, RSR_EHIP, "a persistent classification timed out at a grid barrier");
    }
    out->n_L = c[0];
    out->n_U = c[1];
    out->n_u = c[2];
    out->n_both = c[3];
    out->n_u_up = c[4];
    out->N = static_cast<uint64_t>(N);
    const double Nd = static_cast<double>(N);
    out->p_L = static_cast<double>(out->n_L) / Nd;
    out->p_U = static_cast<double>(out->n_U) / Nd;
    out->p_u = static_cast<double>(out->n_u) / Nd;
    if (!d_Y) {
        out->P = out->se = out->cov = std::nan("");
        return RSR_OK;
    }
    const double P = static_cast<double>(out->n_U + out->n_u_up) / Nd;
    out->P = P;
    out->se = std::sqrt(P * (1.0 - P) / Nd);
    out->cov = P > 0.0 ? std::sqrt((1.0 - P) / (Nd * P)) : HUGE_VAL;
    return RSR_OK;
}

rsr_status rsr_grad(rsr_ctx* ctx, const rsr_model* model, const uint32_t* d_samples,
                    const uint8_t* d_Y, int64_t N, float* d_G, uint64_t* d_counts) {
    if (!ctx) return RSR_EINVAL;
    if (!model || !d_samples || !d_Y || !d_G) return fail(ctx, RSR_EINVAL, "NULL argument");
    if (N <= 0) return fail(ctx, RSR_EINVAL, "N must be > 0");
    DeviceGuard g(ctx->device);
    RSR_HIP(ctx, rsr::launch_grad(ctx->stream, model->n, model->K, model->d_p, d_samples, d_Y, N,
                                  ctx->ws.grad_part, d_G, d_counts));
    return RSR_OK;
}

rsr_status rsr_importance(rsr_ctx* ctx, const rsr_model* model, const uint32_t* d_samples,
                          const uint8_t* d_Y, int64_t N, float* d_I) {
    if (!ctx) return RSR_EINVAL;
    if (!model || !d_samples || !d_Y || !d_I) return fail(ctx, RSR_EINVAL, "NULL argument");
    if (N <= 0) return fail(ctx, RSR_EINVAL, "N must be > 0");
    if (model->K != 2) return fail(ctx, RSR_EINVAL, "the Birnbaum importance needs K = 2");
    DeviceGuard g(ctx->device);
    RSR_HIP(ctx, rsr::launch_importance(ctx->stream, model->n, model->d_p64, d_samples, d_Y, N,
                                        ctx->ws.grad_part, d_I));
    return RSR_OK;
}

rsr_status rsr_debug_barrier_timeout(int64_t ticks) {
    rsr::set_barrier_timeout(ticks);
    return RSR_OK;
}

rsr_status rsr_debug_fail_alloc(int64_t after) {
    rsr::g_fail_countdown = after < 0 ? -1 : after;
    return RSR_OK;
}

}  // extern "C"
