// Stage 1 of the RSR workflow (section 3.5, fig. rsr_alg): alternate sample
// classification and componentwise boundary search (section 3.4) until the
// unclassified fraction of a fresh sample set is small enough or the
// reference sets are large enough.  The sampling, classification, ordered
// pick of unclassified samples and the searches run on the device; the host
// keeps the rows (in discovery order), drops exact duplicates and re-packs
// the reference sets between iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <unordered_set>
#include <vector>

#include "rsr_internal.h"

namespace {

rsr_status s1_fail(rsr_ctx* ctx, rsr_status st, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return st;
}

rsr_status s1_hip(rsr_ctx* ctx, hipError_t e, const char* what) {
    return s1_fail(ctx, e == hipErrorOutOfMemory ? RSR_ENOMEM : RSR_EHIP,
                   std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
}

#define S1_HIP(ctx, call)                                 \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return s1_hip(ctx, e_, #call); \
    } while (0)

struct DeviceBuffer {
    void* p = nullptr;
    ~DeviceBuffer() {
        if (p) (void)hipFree(p);
    }
};

struct RefsHandle {
    rsr_refs* r = nullptr;
    ~RefsHandle() {
        if (r) (void)rsr_refs_destroy(r);
    }
};

struct CurrentDevice {
    int prev = -1;
    bool changed = false;
    explicit CurrentDevice(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) changed = hipSetDevice(dev) == hipSuccess;
    }
    ~CurrentDevice() {
        if (changed) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" rsr_status rsr_stage1(rsr_ctx* ctx, const rsr_model* model, const rsr_system* sys,
                                 const rsr_stage1_params* params, const uint8_t* lower0,
                                 int64_t R_L0, const uint8_t* upper0, int64_t R_U0,
                                 uint8_t* lower, int64_t cap_L, uint8_t* upper, int64_t cap_U,
                                 rsr_stage1_result* result) {
    if (!ctx) return RSR_EINVAL;
    if (!model || !sys || !params || !lower || !upper || !result)
        return s1_fail(ctx, RSR_EINVAL, "NULL argument");
    const rsr_stage1_params P = *params;
    if (model->n != sys->n_edges || model->K != sys->K)
        return s1_fail(ctx, RSR_EINVAL, "model and system differ in n or K");
    if (P.N <= 0 || P.N > 0x7FFFFFFFll) return s1_fail(ctx, RSR_EINVAL, "N must be in 1..2^31-1");
    if (P.picks < 1) return s1_fail(ctx, RSR_EINVAL, "picks must be >= 1");
    if (P.max_iters < 1) return s1_fail(ctx, RSR_EINVAL, "max_iters must be >= 1");
    if (!(P.eps_u >= 0.0)) return s1_fail(ctx, RSR_EINVAL, "eps_u must be >= 0");
    if (P.max_rows < 0 || cap_L < P.max_rows || cap_U < P.max_rows)
        return s1_fail(ctx, RSR_EINVAL, "max_rows must be >= 0 and cap_L, cap_U >= max_rows");
    if (R_L0 < 0 || R_U0 < 0 || (R_L0 > 0 && !lower0) || (R_U0 > 0 && !upper0))
        return s1_fail(ctx, RSR_EINVAL, "bad initial rows");
    if (R_L0 > cap_L || R_U0 > cap_U)
        return s1_fail(ctx, RSR_EINVAL, "initial rows exceed cap_L / cap_U");
    const int n = model->n, K = model->K;
    const size_t row = static_cast<size_t>(n);

    std::vector<uint8_t> rows_l(lower0, lower0 + R_L0 * n), rows_u(upper0, upper0 + R_U0 * n);
    std::unordered_set<std::string> seen_l, seen_u;
    for (int64_t r = 0; r < R_L0; ++r)
        seen_l.emplace(reinterpret_cast<const char*>(lower0 + r * n), row);
    for (int64_t r = 0; r < R_U0; ++r)
        seen_u.emplace(reinterpret_cast<const char*>(upper0 + r * n), row);

    CurrentDevice guard(ctx->device);
    const int64_t N = P.N, B = P.picks;
    DeviceBuffer samples, flags, pick, rows, side;
    S1_HIP(ctx, rsr::dev_malloc(&samples.p, sizeof(uint32_t) * rsr::sample_words(n, K) * static_cast<size_t>(N)));
    S1_HIP(ctx, rsr::dev_malloc(&flags.p, static_cast<size_t>(N)));
    S1_HIP(ctx, rsr::dev_malloc(&pick.p, sizeof(int64_t) * static_cast<size_t>(B)));
    S1_HIP(ctx, rsr::dev_malloc(&rows.p, row * static_cast<size_t>(B)));
    S1_HIP(ctx, rsr::dev_malloc(&side.p, static_cast<size_t>(B)));
    std::vector<uint8_t> rows_h(row * static_cast<size_t>(B)), side_h(static_cast<size_t>(B));
    uint64_t* d_total = ctx->ws.counters + 12;
    uint64_t* h_total = ctx->ws.host_counts + 12;

    rsr_stage1_result res{};
    for (int32_t it = 0; it < P.max_iters; ++it) {
        const int64_t R_L = static_cast<int64_t>(rows_l.size() / row);
        const int64_t R_U = static_cast<int64_t>(rows_u.size() / row);
        RefsHandle refs;
        // The loop classifies with the popcount / cascade forms only, so the
        // matrix-core operands are not built.
        rsr_status st = rsr::refs_create(ctx, n, K, rows_l.data(), R_L, rows_u.data(), R_U, false,
                                         &refs.r);
        if (st != RSR_OK) return st;
        st = rsr_sample(ctx, model, P.seed, static_cast<uint32_t>(it), 0, N,
                        static_cast<uint32_t*>(samples.p));
        if (st != RSR_OK) return st;
        st = rsr_classify(ctx, refs.r, static_cast<const uint32_t*>(samples.p), N, RSR_LABEL,
                          RSR_AUTO, static_cast<uint8_t*>(flags.p), nullptr);
        if (st != RSR_OK) return st;
        S1_HIP(ctx, rsr::launch_pick(ctx->stream, static_cast<const uint8_t*>(flags.p), N, B,
                                     static_cast<int64_t*>(pick.p), ctx->ws.count_part, d_total));
        S1_HIP(ctx, hipMemcpyAsync(h_total, d_total, sizeof(uint64_t), hipMemcpyDeviceToHost,
                                   ctx->stream));
        rsr_estimate_t est;
        st = rsr_estimate(ctx, static_cast<const uint8_t*>(flags.p), nullptr, N, &est);  // synchronises
        if (st != RSR_OK) return st;
        res.iterations = it + 1;
        res.p_u = est.p_u;
        if (est.p_u < P.eps_u || R_L + R_U >= P.max_rows || it + 1 == P.max_iters) break;
        const int64_t n_pick = std::min<int64_t>(static_cast<int64_t>(*h_total), B);
        if (n_pick == 0) break;
        st = rsr_boundary_search(ctx, sys, static_cast<const uint32_t*>(samples.p), N,
                                 static_cast<const int64_t*>(pick.p), n_pick,
                                 static_cast<uint8_t*>(rows.p), static_cast<uint8_t*>(side.p));
        if (st != RSR_OK) return st;
        S1_HIP(ctx, hipMemcpyAsync(rows_h.data(), rows.p, row * static_cast<size_t>(n_pick),
                                   hipMemcpyDeviceToHost, ctx->stream));
        S1_HIP(ctx, hipMemcpyAsync(side_h.data(), side.p, static_cast<size_t>(n_pick),
                                   hipMemcpyDeviceToHost, ctx->stream));
        S1_HIP(ctx, hipStreamSynchronize(ctx->stream));
        res.searches += n_pick;
        int64_t total = R_L + R_U;
        for (int64_t j = 0; j < n_pick && total < P.max_rows; ++j) {
            if (side_h[j] > 1) return s1_fail(ctx, RSR_EHIP, "boundary search rejected a pick");
            const uint8_t* r = rows_h.data() + j * row;
            auto& seen = side_h[j] ? seen_u : seen_l;
            if (!seen.emplace(reinterpret_cast<const char*>(r), row).second) {
                res.duplicates += 1;
                continue;
            }
            auto& dst = side_h[j] ? rows_u : rows_l;
            dst.insert(dst.end(), r, r + row);
            total += 1;
        }
    }
    res.R_L = static_cast<int64_t>(rows_l.size() / row);
    res.R_U = static_cast<int64_t>(rows_u.size() / row);
    if (!rows_l.empty()) std::memcpy(lower, rows_l.data(), rows_l.size());
    if (!rows_u.empty()) std::memcpy(upper, rows_u.data(), rows_u.size());
    *result = res;
    return RSR_OK;
}
