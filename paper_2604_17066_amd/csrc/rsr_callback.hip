// System functions given as a host callback (RSR_SYS_HOST_CALLBACK).
//
// The method needs only a coherent system function (section 2.1): Stage 2
// evaluates it on the samples the reference states leave unclassified
// (section 3.5), and the boundary search of section 3.4 evaluates it after
// every single-component step.  For a callback system both run on the host,
// and the device only moves the samples that need it:
//
//   evaluation: k_label (k_eval.hip) writes Y of the classified samples and
//     lists the others; their packed words are gathered into a compact
//     sample-major buffer (k_cb_gather) and copied to pinned host memory, the
//     callback runs on each decoded state vector in index order, and the
//     results go back and are scattered into Y (k_cb_scatter_y).
//   boundary search: the picked samples are gathered the same way, each walk
//     runs on the host, and the rows are copied back and written for the
//     valid picks only (k_cb_rows).
#include <algorithm>
#include <numeric>
#include <string>
#include <vector>

#include "rsr_internal.h"

namespace rsr {
namespace {

constexpr int kBlock = 256;

// out[j][w] = word w of sample idx(j), for j < count; idx(j) = list[j] (i32),
// picks[j] (i64), or j when both are null.  Picks outside 0..N-1 are skipped.
__global__ __launch_bounds__(kBlock) void k_cb_gather(const uint32_t* __restrict__ xs, int64_t N,
                                                      int W, const int32_t* __restrict__ list,
                                                      const int64_t* __restrict__ picks,
                                                      const unsigned long long* __restrict__ d_count,
                                                      int64_t count, uint32_t* __restrict__ out) {
    const int64_t total = d_count ? static_cast<int64_t>(*d_count) : count;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; k < total * W;
         k += stride) {
        const int64_t j = k / W;
        const int w = static_cast<int>(k - j * W);
        const int64_t h = list ? static_cast<int64_t>(list[j]) : (picks ? picks[j] : j);
        if (h < 0 || h >= N) continue;
        out[k] = xs[static_cast<int64_t>(w) * N + h];
    }
}

__global__ __launch_bounds__(kBlock) void k_cb_scatter_y(const int32_t* __restrict__ list,
                                                         const uint8_t* __restrict__ y, int64_t count,
                                                         uint8_t* __restrict__ Y) {
    const int64_t j = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (j < count) Y[list[j]] = y[j];
}

// rows[j][*] = staged[j][*] for every pick with a valid side (< 2).
__global__ __launch_bounds__(kBlock) void k_cb_rows(const uint8_t* __restrict__ staged,
                                                    const uint8_t* __restrict__ side, int64_t n_pick,
                                                    int n, uint8_t* __restrict__ rows) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= n_pick * n) return;
    const int64_t j = k / n;
    if (side[j] < 2) rows[k] = staged[k];
}

unsigned grid_for(int64_t work) {
    int64_t b = (work + kBlock - 1) / kBlock;
    if (b > 4096) b = 4096;
    return static_cast<unsigned>(b < 1 ? 1 : b);
}

// Grows the callback staging buffers to hold `count` samples of W words and
// `bytes` result bytes.
rsr_status ensure_stage(rsr_ctx* ctx, int64_t words, int64_t bytes, int64_t picks) {
    CallbackStage& cb = ctx->ws.cb;
    if (cb.words_cap < words) {
        if (cb.d_words) (void)hipFree(cb.d_words);
        if (cb.h_words) (void)hipHostFree(cb.h_words);
        cb.d_words = nullptr;
        cb.h_words = nullptr;
        cb.words_cap = 0;
        hipError_t e = dev_malloc(&cb.d_words, sizeof(uint32_t) * static_cast<size_t>(words));
        if (e == hipSuccess) e = host_malloc(&cb.h_words, sizeof(uint32_t) * static_cast<size_t>(words));
        if (e != hipSuccess) return hip_error(ctx, e, "callback sample staging");
        cb.words_cap = words;
    }
    if (cb.bytes_cap < bytes) {
        if (cb.d_bytes) (void)hipFree(cb.d_bytes);
        if (cb.h_bytes) (void)hipHostFree(cb.h_bytes);
        cb.d_bytes = nullptr;
        cb.h_bytes = nullptr;
        cb.bytes_cap = 0;
        hipError_t e = dev_malloc(&cb.d_bytes, static_cast<size_t>(bytes));
        if (e == hipSuccess) e = host_malloc(&cb.h_bytes, static_cast<size_t>(bytes));
        if (e != hipSuccess) return hip_error(ctx, e, "callback result staging");
        cb.bytes_cap = bytes;
    }
    if (cb.index_cap < picks) {
        if (cb.h_index) (void)hipHostFree(cb.h_index);
        cb.h_index = nullptr;
        cb.index_cap = 0;
        hipError_t e = host_malloc(&cb.h_index, sizeof(int64_t) * static_cast<size_t>(picks));
        if (e != hipSuccess) return hip_error(ctx, e, "callback pick staging");
        cb.index_cap = picks;
    }
    return RSR_OK;
}

// State vector of a packed sample (thermometer planes of rsr.h).
void decode(const uint32_t* words, int n, int K, uint8_t* x) {
    const int PW = plane_words(n);
    for (int i = 0; i < n; ++i) {
        int v = 0;
        for (int j = 1; j < K; ++j)
            v += static_cast<int>((words[(j - 1) * PW + (i >> 5)] >> (i & 31)) & 1u);
        x[i] = static_cast<uint8_t>(v);
    }
}

// Phi(x) = [phi(x) >= level]; a negative state is an error (returned as -1).
int call_phi(const rsr_system* sys, const uint8_t* x) {
    const int32_t S = sys->phi(x, sys->n_edges, sys->user);
    if (S < 0) return -1;
    return S >= sys->level ? 1 : 0;
}

#define CB_HIP(ctx, call)                                      \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_error(ctx, e_, #call); \
    } while (0)

}  // namespace

rsr_status eval_callback(rsr_ctx* ctx, const rsr_system* sys, const uint32_t* d_samples, int64_t N,
                         const uint8_t* d_flags, int which, uint8_t* d_Y, uint64_t* d_n_evaluated) {
    const int n = sys->n_edges, K = sys->K, W = sample_words(n, K);
    hipStream_t st = ctx->stream;
    int64_t count = N;
    const int32_t* list = nullptr;
    if (which == RSR_UNKNOWN_ONLY) {
        rsr_status s = ensure_list(ctx, N);
        if (s != RSR_OK) return s;
        uint64_t* counter = ctx->ws.counters + 8;
        CB_HIP(ctx, launch_fill_u64(st, counter, 1, 0));
        const SegSrc seg = single_src(d_samples, N, const_cast<uint8_t*>(d_flags), d_Y);
        CB_HIP(ctx, launch_label(st, seg, ctx->ws.list, counter, ctx->cu_count * 16));
        CB_HIP(ctx, hipMemcpyAsync(ctx->ws.host_counts + 8, counter, sizeof(uint64_t),
                                   hipMemcpyDeviceToHost, st));
        CB_HIP(ctx, hipStreamSynchronize(st));
        count = static_cast<int64_t>(ctx->ws.host_counts[8]);
        list = ctx->ws.list;
    }
    if (count > 0) {
        rsr_status s = ensure_stage(ctx, count * W, count, 0);
        if (s != RSR_OK) return s;
        CallbackStage& cb = ctx->ws.cb;
        hipLaunchKernelGGL(k_cb_gather, dim3(grid_for(count * W)), dim3(kBlock), 0, st, d_samples,
                           N, W, list, static_cast<const int64_t*>(nullptr),
                           static_cast<const unsigned long long*>(nullptr), count, cb.d_words);
        CB_HIP(ctx, hipGetLastError());
        CB_HIP(ctx, hipMemcpyAsync(cb.h_words, cb.d_words, sizeof(uint32_t) * count * W,
                                   hipMemcpyDeviceToHost, st));
        std::vector<int32_t> order_idx;
        if (list) {
            order_idx.resize(static_cast<size_t>(count));
            CB_HIP(ctx, hipMemcpyAsync(order_idx.data(), list, sizeof(int32_t) * count,
                                       hipMemcpyDeviceToHost, st));
        }
        CB_HIP(ctx, hipStreamSynchronize(st));
        // The list is filled by atomics, so its order varies; the callback is
        // called in increasing sample index, which makes the call sequence
        // reproducible.
        std::vector<int64_t> order(static_cast<size_t>(count));
        std::iota(order.begin(), order.end(), int64_t{0});
        if (list)
            std::sort(order.begin(), order.end(),
                      [&](int64_t a, int64_t b) { return order_idx[a] < order_idx[b]; });
        std::vector<uint8_t> x(static_cast<size_t>(n));
        for (int64_t j : order) {
            decode(cb.h_words + j * W, n, K, x.data());
            const int y = call_phi(sys, x.data());
            if (y < 0)
                return set_error(ctx, RSR_EINVAL, "system function returned a negative state");
            cb.h_bytes[j] = static_cast<uint8_t>(y);
        }
        if (list) {
            CB_HIP(ctx, hipMemcpyAsync(cb.d_bytes, cb.h_bytes, static_cast<size_t>(count),
                                       hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(k_cb_scatter_y, dim3(grid_for(count)), dim3(kBlock), 0, st, list,
                               cb.d_bytes, count, d_Y);
            CB_HIP(ctx, hipGetLastError());
        } else {
            CB_HIP(ctx, hipMemcpyAsync(d_Y, cb.h_bytes, static_cast<size_t>(count),
                                       hipMemcpyHostToDevice, st));
        }
        // The pinned staging is reused by the next call: wait for the copy.
        CB_HIP(ctx, hipStreamSynchronize(st));
    }
    if (d_n_evaluated) CB_HIP(ctx, launch_fill_u64(st, d_n_evaluated, 1, static_cast<uint64_t>(count)));
    return RSR_OK;
}

rsr_status boundary_callback(rsr_ctx* ctx, const rsr_system* sys, const uint32_t* d_samples,
                             int64_t N, const int64_t* d_pick, int64_t n_pick, uint8_t* d_rows,
                             uint8_t* d_side) {
    const int n = sys->n_edges, K = sys->K, W = sample_words(n, K);
    hipStream_t st = ctx->stream;
    // Bytes: n_pick rows of n states, then n_pick sides.
    rsr_status s = ensure_stage(ctx, n_pick * W, n_pick * (n + 1), n_pick);
    if (s != RSR_OK) return s;
    CallbackStage& cb = ctx->ws.cb;
    hipLaunchKernelGGL(k_cb_gather, dim3(grid_for(n_pick * W)), dim3(kBlock), 0, st, d_samples, N,
                       W, static_cast<const int32_t*>(nullptr), d_pick,
                       static_cast<const unsigned long long*>(nullptr), n_pick, cb.d_words);
    CB_HIP(ctx, hipGetLastError());
    CB_HIP(ctx, hipMemcpyAsync(cb.h_words, cb.d_words, sizeof(uint32_t) * n_pick * W,
                               hipMemcpyDeviceToHost, st));
    CB_HIP(ctx, hipMemcpyAsync(cb.h_index, d_pick, sizeof(int64_t) * n_pick, hipMemcpyDeviceToHost,
                               st));
    CB_HIP(ctx, hipStreamSynchronize(st));
    uint8_t* rows = cb.h_bytes;
    uint8_t* side = cb.h_bytes + n_pick * n;
    for (int64_t j = 0; j < n_pick; ++j) {
        const int64_t h = cb.h_index[j];
        uint8_t* x = rows + j * n;
        if (h < 0 || h >= N) {
            side[j] = 0xFF;
            std::fill(x, x + n, uint8_t{0});
            continue;
        }
        decode(cb.h_words + j * W, n, K, x);
        const int up = call_phi(sys, x);
        if (up < 0) return set_error(ctx, RSR_EINVAL, "system function returned a negative state");
        // Failure side: raise each component in index order while the system
        // stays failed, undoing the step that makes it work; survival side:
        // lower each while it keeps working, undoing the step that fails it.
        for (int i = 0; i < n; ++i) {
            for (;;) {
                if (up ? x[i] == 0 : x[i] == K - 1) break;
                x[i] = static_cast<uint8_t>(up ? x[i] - 1 : x[i] + 1);
                const int y = call_phi(sys, x);
                if (y < 0)
                    return set_error(ctx, RSR_EINVAL, "system function returned a negative state");
                if (y != up) {
                    x[i] = static_cast<uint8_t>(up ? x[i] + 1 : x[i] - 1);
                    break;
                }
            }
        }
        side[j] = static_cast<uint8_t>(up);
    }
    CB_HIP(ctx, hipMemcpyAsync(cb.d_bytes, cb.h_bytes, static_cast<size_t>(n_pick * (n + 1)),
                               hipMemcpyHostToDevice, st));
    CB_HIP(ctx, hipMemcpyAsync(d_side, cb.d_bytes + n_pick * n, static_cast<size_t>(n_pick),
                               hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_cb_rows, dim3(grid_for(n_pick * n)), dim3(kBlock), 0, st, cb.d_bytes,
                       cb.d_bytes + n_pick * n, n_pick, n, d_rows);
    CB_HIP(ctx, hipGetLastError());
    CB_HIP(ctx, hipStreamSynchronize(st));
    return RSR_OK;
}

}  // namespace rsr
