// Batched plan: many (model, reference set, system) jobs in one captured HIP
// graph.
//
// Jobs that share a reference set and a system function form a segment
// (reference states depend on the system only, not on the component
// probabilities, section 5, so every hazard scenario of one network shares
// them).  Each stage of the hot path runs once per segment over the
// concatenation of its jobs' samples, addressed by a global index with a job
// offset table: one sampler launch, one classification cascade, one label and
// one BFS launch, one gradient and one count launch with a job grid dimension.
// Small jobs therefore fill the GPU together and the launch count is
// O(segments), not O(jobs).  Before capture an autotuner times the candidate
// classification configurations of each segment on its own data and keeps the
// fastest.  The whole plan, ending with the copy of every job's counts to
// pinned host memory, is recorded into one HIP graph; rsr_plan_run is one
// graph launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "rsr_internal.h"

namespace {

// kPersist: the persistent LABEL cascade (one round-0 launch and one
// cooperative launch for every later round, over all jobs of the segment).
enum Choice { kCascade = 0, kBitsPerJob = 1, kMfmaPerJob = 2, kMfma4PerJob = 3, kPersist = 4 };

struct Segment {
    const rsr_refs* refs = nullptr;
    const rsr_system* sys = nullptr;
    int n = 0, K = 0, W = 0;
    std::vector<int> jobs;  // plan job indices, in device order
    int first_pos = 0;      // device position of the first job
    int64_t total = 0, max_N = 0;
    bool any_grad = false;
    Choice choice = kCascade;
    rsr::CascadeShape shape;
    float tuned_ms = 0.0f;
};

// One entry of the tuning cache: the configuration chosen for a segment shape.
struct TuneEntry {
    int choice = 0, first = 0, growth = 0, split = 0, tail = 0, chunks = 0;
    double ms = 0.0;
};

// The tuning cache file is one JSON object: keys are segment-shape strings,
// values are objects of numbers {"choice", "first", "growth", "split", "tail",
// "ms"} ("tail": 0 popcount rounds, 1 matrix-core rounds after round 0, 2
// matrix-core rounds from round 0 on) and optionally "chunks" (most chunks of
// a split round, 0 for the built-in caps).  This reader accepts exactly that
// (strings without escapes) and returns false on anything else.
class CacheReader {
  public:
    explicit CacheReader(const std::string& t) : t_(t) {}
    bool parse(std::map<std::string, TuneEntry>& out) {
        ws();
        if (!eat('{')) return false;
        ws();
        if (eat('}')) return tail();
        for (;;) {
            std::string key;
            if (!str(key)) return false;
            ws();
            if (!eat(':')) return false;
            ws();
            TuneEntry e;
            if (!entry(e)) return false;
            out[key] = e;
            ws();
            if (eat(',')) {
                ws();
                continue;
            }
            if (eat('}')) return tail();
            return false;
        }
    }

  private:
    const std::string& t_;
    size_t i_ = 0;
    void ws() {
        while (i_ < t_.size() && std::isspace(static_cast<unsigned char>(t_[i_]))) ++i_;
    }
    bool eat(char c) {
        if (i_ < t_.size() && t_[i_] == c) {
            ++i_;
            return true;
        }
        return false;
    }
    bool tail() {
        ws();
        return i_ == t_.size();
    }
    bool str(std::string& s) {
        if (!eat('"')) return false;
        const size_t b = i_;
        while (i_ < t_.size() && t_[i_] != '"') {
            if (t_[i_] == '\\' || static_cast<unsigned char>(t_[i_]) < 0x20) return false;
            ++i_;
        }
        if (i_ >= t_.size()) return false;
        s = t_.substr(b, i_ - b);
        ++i_;
        return true;
    }
    bool num(double& v) {
        const char* b = t_.c_str() + i_;
        char* e = nullptr;
        v = std::strtod(b, &e);
        if (e == b || !std::isfinite(v)) return false;
        i_ += static_cast<size_t>(e - b);
        return true;
    }
    bool entry(TuneEntry& e) {
        if (!eat('{')) return false;
        int seen = 0;
        ws();
        if (eat('}')) return false;
        for (;;) {
            std::string k;
            double v = 0.0;
            ws();
            if (!str(k)) return false;
            ws();
            if (!eat(':')) return false;
            ws();
            if (!num(v)) return false;
            if (k == "choice") e.choice = static_cast<int>(v), seen |= 1;
            else if (k == "first") e.first = static_cast<int>(v), seen |= 2;
            else if (k == "growth") e.growth = static_cast<int>(v), seen |= 4;
            else if (k == "split") e.split = static_cast<int>(v), seen |= 8;
            else if (k == "tail") e.tail = static_cast<int>(v), seen |= 16;
            else if (k == "ms") e.ms = v, seen |= 32;
            else if (k == "chunks") e.chunks = static_cast<int>(v), seen |= 64;
            else return false;
            ws();
            if (eat(',')) continue;
            if (eat('}')) break;
            return false;
        }
        return (seen & 63) == 63 && e.choice >= kCascade && e.choice <= kPersist &&
               e.chunks >= 0 && e.chunks <= 1024 &&
               (e.choice != kCascade || (e.first >= 1 && e.growth >= 2 && e.split >= 1));
    }
};

}  // namespace

struct rsr_plan {
    rsr_ctx* ctx = nullptr;
    std::vector<rsr_job> jobs;
    std::vector<int> pos;  // plan job index -> device position
    std::vector<Segment> segs;
    rsr::JobDev* d_jobs = nullptr;
    int64_t* d_offsets = nullptr;  // per segment [jobs + 1], concatenated
    std::vector<int64_t> offset_base;
    uint64_t* d_counts = nullptr;     // [jobs][8]
    uint64_t* h_counts = nullptr;     // pinned [jobs][8]
    float* d_G_all = nullptr;         // every job's gradient, gathered (job.g_off)
    float* h_G_all = nullptr;         // pinned copy
    int64_t G_total = 0;
    std::vector<int64_t> host_g_off;  // device position -> offset in the gather buffer
    uint64_t* d_count_part = nullptr;
    uint32_t* d_grad_part = nullptr;
    uint32_t* d_casc_words = nullptr;
    int32_t* d_casc_index = nullptr;
    int64_t casc_cap = 0;
    int casc_w = 0;
    uint64_t* d_casc_counters = nullptr;
    uint32_t* d_casc_state = nullptr;  // persistent cascade state (zeroed per launch)
    int64_t casc_state_words = 0;
    int32_t* d_list = nullptr;
    uint64_t* d_list_counter = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

rsr_status pfail(rsr_ctx* ctx, rsr_status st, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return st;
}

rsr_status phip(rsr_ctx* ctx, hipError_t e, const char* what) {
    return pfail(ctx, e == hipErrorOutOfMemory ? RSR_ENOMEM : RSR_EHIP,
                 std::string(what) + ": " + hipGetErrorName(e));
}

#define PLAN_HIP(ctx, call)                                  \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return phip(ctx, e_, #call);   \
    } while (0)

// The segment's jobs as one sample range; a prefix (n_jobs > 0) takes its
// first n_jobs jobs (device order), `total` samples.
rsr::SegSrc seg_src(const rsr_plan* p, const Segment& s, int si, int n_jobs = 0,
                    int64_t total = 0) {
    rsr::SegSrc src{};
    src.jobs = p->d_jobs + s.first_pos;
    src.offsets = p->d_offsets + p->offset_base[si];
    src.n_jobs = static_cast<int32_t>(n_jobs > 0 ? n_jobs : s.jobs.size());
    src.total = n_jobs > 0 ? total : s.total;
    return src;
}

rsr::CascadeBuffers casc_buffers(const rsr_plan* p) {
    rsr::CascadeBuffers cb;
    cb.words[0] = p->d_casc_words;
    cb.words[1] = p->d_casc_words + static_cast<int64_t>(p->casc_w) * p->casc_cap;
    cb.index[0] = p->d_casc_index;
    cb.index[1] = p->d_casc_index + p->casc_cap;
    cb.match[0] = reinterpret_cast<uint32_t*>(p->d_casc_index + 2 * p->casc_cap);
    cb.match[1] = reinterpret_cast<uint32_t*>(p->d_casc_index + 3 * p->casc_cap);
    cb.stride = p->casc_cap;
    cb.counters = p->d_casc_counters;
    cb.regions = reinterpret_cast<uint32_t*>(p->d_casc_counters + 16);
    return cb;
}

hipError_t enqueue_sample(const rsr_plan* p, int si, hipStream_t st) {
    const Segment& s = p->segs[si];
    return rsr::launch_sample_jobs(st, s.n, s.K, p->d_jobs + s.first_pos,
                                   p->d_offsets + p->offset_base[si],
                                   static_cast<int>(s.jobs.size()), s.total, p->ctx->cu_count * 16);
}

// Classification of the segment, or of its first n_jobs jobs (`total`
// samples) when n_jobs > 0.
hipError_t enqueue_classify(const rsr_plan* p, int si, hipStream_t st, Choice choice,
                            const rsr::CascadeShape& shape, int n_jobs = 0, int64_t total = 0) {
    const Segment& s = p->segs[si];
    const rsr::SegSrc src = seg_src(p, s, si, n_jobs, total);
    if (choice == kPersist) {
        // counters[15] is the barrier time-out flag, cleared once per run at
        // the start of the graph and copied back with the counts.
        const rsr::CascadeBuffers cb = casc_buffers(p);
        hipError_t e = rsr::launch_fill_u64(st, reinterpret_cast<uint64_t*>(p->d_casc_state),
                                            (p->casc_state_words + 1) / 2, 0);
        if (e != hipSuccess) return e;
        return rsr::launch_casc_persist(st, s.refs, src, cb, rsr::mfma_head_shape(),
                                        p->d_casc_state,
                                        reinterpret_cast<unsigned long long*>(p->d_casc_counters + 15),
                                        p->ctx->cu_count);
    }
    if (choice == kCascade) {
        const rsr::CascadeBuffers cb = casc_buffers(p);
        hipError_t e = rsr::launch_fill_u64(st, cb.counters, rsr::CascadeBuffers::kMaxRounds, 0);
        if (e != hipSuccess) return e;
        return rsr::launch_dom_cascade(st, s.refs, src, cb, shape, p->ctx->cu_count * 8);
    }
    for (int k = 0; k < src.n_jobs; ++k) {
        const rsr_job& jb = p->jobs[s.jobs[k]];
        hipError_t e = choice == kMfmaPerJob || choice == kMfma4PerJob
                           ? rsr::launch_dom_mfma(st, s.refs, jb.d_samples, jb.N, RSR_LABEL,
                                                  choice == kMfma4PerJob, p->ctx->cu_count,
                                                  jb.d_flags, nullptr)
                           : rsr::launch_dom_bits(st, s.refs, jb.d_samples, jb.N, RSR_LABEL,
                                                  jb.d_flags, nullptr);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t enqueue_rest(const rsr_plan* p, int si, hipStream_t st) {
    const Segment& s = p->segs[si];
    const rsr::SegSrc src = seg_src(p, s, si);
    const int nj = static_cast<int>(s.jobs.size());
    hipError_t e = rsr::launch_fill_u64(st, p->d_list_counter, 1, 0);
    if (e == hipSuccess)
        e = rsr::launch_label(st, src, p->d_list, p->d_list_counter, p->ctx->cu_count * 16);
    if (e == hipSuccess)
        e = rsr::launch_bfs(st, s.sys, src, p->d_list, p->d_list_counter, RSR_UNKNOWN_ONLY, nullptr,
                            p->ctx->cu_count * 8);
    if (e == hipSuccess && s.any_grad)
        e = rsr::launch_grad(st, s.n, s.K, nullptr, nullptr, nullptr, s.max_N, p->d_grad_part,
                             nullptr, nullptr, p->d_jobs + s.first_pos, nj);
    if (e == hipSuccess && s.any_grad)
        e = rsr::launch_gather_G(st, p->d_jobs + s.first_pos, nj, s.n * s.K, p->d_G_all);
    if (e == hipSuccess)
        e = rsr::launch_counts(st, nullptr, nullptr, s.max_N,
                               p->d_counts + static_cast<int64_t>(s.first_pos) * 8,
                               p->d_count_part, p->d_jobs + s.first_pos, nj);
    return e;
}

// Tuning-cache key of a segment: the device and every property of the
// segment that the timing depends on.
std::string segment_key(const rsr_ctx* ctx, const Segment& s) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s/cu%d/W%d/RL%lld/RU%lld/c%d/f%d/J%zu/T%lld/M%lld",
                  ctx->arch.c_str(), ctx->cu_count, s.W, static_cast<long long>(s.refs->R_L),
                  static_cast<long long>(s.refs->R_U), s.refs->consistent ? 1 : 0,
                  s.refs->KS4 > 0 ? 1 : 0, s.jobs.size(), static_cast<long long>(s.total),
                  static_cast<long long>(s.max_N));
    return buf;
}

bool choice_runs(const Segment& s) {
    switch (s.choice) {
        case kCascade:
            return s.refs->consistent && (!s.shape.mfma_tail || s.refs->KS4 > 0) &&
                   (!s.shape.mfma_head || rsr::casc_head_supported(s.refs));
        case kBitsPerJob: return true;
        case kMfmaPerJob: return s.refs->KS > 0;
        case kMfma4PerJob: return s.refs->KS4 > 0;
        case kPersist: return s.refs->consistent && rsr::casc_persist_supported(s.refs);
    }
    return false;
}

rsr_status write_cache(rsr_ctx* ctx, const std::string& path,
                       const std::map<std::string, TuneEntry>& cache) {
    const std::string tmp = path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return pfail(ctx, RSR_EINVAL, "cannot write tuning cache " + tmp);
    std::fprintf(f, "{\n");
    size_t k = 0;
    for (const auto& kv : cache) {
        const TuneEntry& e = kv.second;
        std::fprintf(f,
                     "  \"%s\": {\"choice\": %d, \"first\": %d, \"growth\": %d, \"split\": %d, "
                     "\"tail\": %d, \"chunks\": %d, \"ms\": %.6g}%s\n",
                     kv.first.c_str(), e.choice, e.first, e.growth, e.split, e.tail, e.chunks, e.ms,
                     ++k < cache.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) {
        std::remove(tmp.c_str());
        return pfail(ctx, RSR_EINVAL, "cannot write tuning cache " + path);
    }
    return RSR_OK;
}

// Samples on which tuning times its candidates: the first jobs of a segment
// up to at least this many (every job when the segment has fewer).  The best
// configuration depends on how the samples are classified, not on how many
// jobs share the launch, and a whole segment can take half a second per
// trial (64 jobs of 1e6 samples on the 1250-edge graph).
constexpr int64_t kTuneSamples = int64_t{1} << 22;

// Times candidate classifications of one segment on its own samples (drawn
// once, the trials on a prefix of kTuneSamples) and keeps the fastest; the
// segment's time is the prefix's scaled by the sample counts.  For a
// consistent reference set the split-round form (popcount or FP4) is chosen
// first on the default cascade shape, then the shape with that form;
// otherwise the per-job forms are compared.
rsr_status tune_segment(rsr_plan* p, int si) {
    Segment& s = p->segs[si];
    rsr_ctx* ctx = p->ctx;
    struct Cand {
        Choice c;
        rsr::CascadeShape shape;
    };
    int n_tune = 0;
    int64_t tune_total = 0;
    while (n_tune < static_cast<int>(s.jobs.size()) && tune_total < kTuneSamples)
        tune_total += p->jobs[s.jobs[n_tune++]].N;
    const float scale = static_cast<float>(static_cast<double>(s.total) / static_cast<double>(tune_total));
    PLAN_HIP(ctx, enqueue_sample(p, si, p->cap));
    hipEvent_t a, b;
    PLAN_HIP(ctx, hipEventCreate(&a));
    PLAN_HIP(ctx, hipEventCreate(&b));
    float best = 1e30f;
    auto trial = [&](const std::vector<Cand>& cands) -> rsr_status {
        for (const Cand& c : cands) {
            PLAN_HIP(ctx, enqueue_classify(p, si, p->cap, c.c, c.shape, n_tune, tune_total));  // warm-up
            PLAN_HIP(ctx, hipEventRecord(a, p->cap));
            for (int rep = 0; rep < 2; ++rep)
                PLAN_HIP(ctx, enqueue_classify(p, si, p->cap, c.c, c.shape, n_tune, tune_total));
            PLAN_HIP(ctx, hipEventRecord(b, p->cap));
            PLAN_HIP(ctx, hipEventSynchronize(b));
            float ms = 0.0f;
            PLAN_HIP(ctx, hipEventElapsedTime(&ms, a, b));
            if (ms < best) {
                best = ms;
                s.choice = c.c;
                s.shape = c.shape;
            }
        }
        return RSR_OK;
    };
    rsr_status st = RSR_OK;
    if (s.refs->consistent) {
        std::vector<Cand> forms = {{kCascade, rsr::CascadeShape{}}};
        if (s.refs->KS4 > 0) {
            forms.push_back({kCascade, rsr::mfma_tail_shape()});
            forms.push_back({kCascade, rsr::mfma_wide_shape()});
        }
        if (s.refs->KS4 > 0 && rsr::casc_head_supported(s.refs))
            forms.push_back({kCascade, rsr::mfma_head_shape()});
        if (rsr::casc_persist_supported(s.refs)) forms.push_back({kPersist, rsr::mfma_head_shape()});
        st = trial(forms);
        // The persistent cascade keeps its own round sizes.
        if (st != RSR_OK || s.choice == kPersist) {
            s.tuned_ms = best / 2.0f * scale;
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            return st;
        }
        const bool tail = s.shape.mfma_tail, head = s.shape.mfma_head;
        std::vector<Cand> shapes;
        // The matrix-core round 0 is one 32-row tile per side.
        const std::vector<int> firsts = head ? std::vector<int>{32} : std::vector<int>{8, 16, 32, 64};
        const int growths[] = {4, 8};
        const int splits[] = {64, 256, 512};
        for (int f : firsts)
            for (int g : growths)
                for (int sp : splits)
                    shapes.push_back({kCascade, rsr::CascadeShape{f, g, sp, tail, head}});
        if (st == RSR_OK) st = trial(shapes);
        // Then the chosen shape with fewer and with more chunks per split
        // round: the best cap depends on the rows and the survivors (measured
        // alone, 32 is the faster on 1e5 rows of 1250 bits and 64 on 4.7e4
        // rows of 900; inside a plan most segments take 8 to 32).
        if (st == RSR_OK) {
            std::vector<Cand> caps;
            for (int mc : {8, 16, 32, 128}) {
                rsr::CascadeShape c = s.shape;
                c.max_chunks = mc;
                caps.push_back({kCascade, c});
            }
            st = trial(caps);
        }
    } else {
        std::vector<Cand> forms = {{kBitsPerJob, rsr::CascadeShape{}}};
        if (s.refs->KS > 0) forms.push_back({kMfmaPerJob, rsr::CascadeShape{}});
        if (s.refs->KS4 > 0) forms.push_back({kMfma4PerJob, rsr::CascadeShape{}});
        st = trial(forms);
    }
    s.tuned_ms = best / 2.0f * scale;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return st;
}

void free_plan(rsr_plan* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap) (void)hipStreamDestroy(p->cap);
    void* dev[] = {p->d_jobs, p->d_offsets, p->d_counts, p->d_count_part, p->d_grad_part,
                   p->d_casc_words, p->d_casc_index, p->d_casc_counters, p->d_casc_state,
                   p->d_list, p->d_list_counter};
    for (void* d : dev)
        if (d) (void)hipFree(d);
    if (p->h_counts) (void)hipHostFree(p->h_counts);
    if (p->h_G_all) (void)hipHostFree(p->h_G_all);
    if (p->d_G_all) (void)hipFree(p->d_G_all);
    delete p;
}

}  // namespace

extern "C" {

rsr_status rsr_plan_create(rsr_ctx* ctx, const rsr_job* jobs, int32_t n_jobs,
                           const char* tune_cache, rsr_plan** out) {
    if (!ctx || !out) return RSR_EINVAL;
    *out = nullptr;
    if (!jobs || n_jobs <= 0) return pfail(ctx, RSR_EINVAL, "no jobs");
    for (int32_t j = 0; j < n_jobs; ++j) {
        const rsr_job& jb = jobs[j];
        if (!jb.model || !jb.refs || !jb.sys || !jb.d_samples || !jb.d_flags || !jb.d_Y)
            return pfail(ctx, RSR_EINVAL, "job " + std::to_string(j) + ": NULL handle or buffer");
        if (jb.N <= 0 || jb.N > 0x7FFFFFFFll)
            return pfail(ctx, RSR_EINVAL, "job " + std::to_string(j) + ": N out of range");
        if (jb.model->n != jb.refs->n || jb.model->K != jb.refs->K ||
            jb.sys->n_edges != jb.refs->n || jb.sys->K != jb.refs->K)
            return pfail(ctx, RSR_EINVAL, "job " + std::to_string(j) + ": n/K mismatch");
        if (jb.model->ctx->device != ctx->device || jb.refs->ctx->device != ctx->device)
            return pfail(ctx, RSR_EINVAL, "job " + std::to_string(j) + ": handle on another device");
        if (jb.sys->kind == RSR_SYS_HOST_CALLBACK)
            return pfail(ctx, RSR_EUNSUPPORTED,
                         "job " + std::to_string(j) + ": host-callback systems cannot run in a plan");
    }
    // The tuning cache is read (and checked) before any device work.
    const bool tune = tune_cache != nullptr;
    const std::string cache_path = tune_cache ? tune_cache : "";
    std::map<std::string, TuneEntry> cache;
    if (!cache_path.empty()) {
        if (FILE* f = std::fopen(cache_path.c_str(), "rb")) {
            std::string text;
            char buf[4096];
            size_t got;
            while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
            std::fclose(f);
            if (!CacheReader(text).parse(cache))
                return pfail(ctx, RSR_EINVAL, "tuning cache " + cache_path + " is not a valid cache file");
        }
    }
    rsr_plan* p = new (std::nothrow) rsr_plan();
    if (!p) return pfail(ctx, RSR_ENOMEM, "host allocation");
    p->ctx = ctx;
    p->jobs.assign(jobs, jobs + n_jobs);
    // Segments: jobs sharing (refs, system), in order of first appearance.
    for (int32_t j = 0; j < n_jobs; ++j) {
        const rsr_job& jb = jobs[j];
        auto it = std::find_if(p->segs.begin(), p->segs.end(), [&](const Segment& s) {
            return s.refs == jb.refs && s.sys == jb.sys;
        });
        if (it == p->segs.end()) {
            Segment s;
            s.refs = jb.refs;
            s.sys = jb.sys;
            s.n = jb.refs->n;
            s.K = jb.refs->K;
            s.W = jb.refs->W;
            s.choice = jb.refs->consistent ? kCascade : kBitsPerJob;
            // Untuned, a cascade takes the shape of rsr_classify's automatic
            // form: matrix-core rounds when the reference handle has FP4
            // operands, growing faster from kWideRows rows per side on.
            const int64_t rows = std::max(jb.refs->R_L, jb.refs->R_U);
            if (jb.refs->KS4 > 0)
                s.shape = rows >= rsr::kWideRows ? rsr::mfma_wide_shape() : rsr::mfma_tail_shape();
            p->segs.push_back(s);
            it = p->segs.end() - 1;
        }
        it->jobs.push_back(j);
        it->total += jb.N;
        it->max_N = std::max(it->max_N, static_cast<int64_t>(jb.N));
        it->any_grad = it->any_grad || jb.d_G != nullptr;
    }
    // Largest work first.
    std::stable_sort(p->segs.begin(), p->segs.end(), [](const Segment& a, const Segment& b) {
        return a.total * (a.W + a.refs->R_L + a.refs->R_U) >
               b.total * (b.W + b.refs->R_L + b.refs->R_U);
    });
    p->pos.assign(n_jobs, 0);
    std::vector<rsr::JobDev> host_jobs;
    std::vector<int64_t> host_offsets;
    int64_t max_total = 0, max_words = 0, max_grad = 0;
    int max_jobs = 0;
    for (Segment& s : p->segs) {
        if (s.total > 0x7FFFFFFFll) {
            free_plan(p);
            return pfail(ctx, RSR_EUNSUPPORTED, "a segment holds more than 2^31-1 samples");
        }
        s.first_pos = static_cast<int>(host_jobs.size());
        p->offset_base.push_back(static_cast<int64_t>(host_offsets.size()));
        int64_t off = 0;
        for (int j : s.jobs) {
            const rsr_job& jb = jobs[j];
            p->pos[j] = static_cast<int>(host_jobs.size());
            rsr::JobDev d{};
            d.thresh = jb.model->d_thresh;
            d.half = jb.model->d_half;
            d.p = jb.model->d_p;
            d.samples = jb.d_samples;
            d.flags = jb.d_flags;
            d.Y = jb.d_Y;
            d.G = jb.d_G;
            d.N = jb.N;
            d.seed = jb.seed;
            d.stream_id = jb.stream_id;
            d.n = s.n;
            d.K = s.K;
            d.g_off = p->G_total;
            p->host_g_off.push_back(p->G_total);
            p->G_total += static_cast<int64_t>(s.n) * s.K;
            host_jobs.push_back(d);
            host_offsets.push_back(off);
            off += jb.N;
        }
        host_offsets.push_back(off);
        max_total = std::max(max_total, s.total);
        max_words = std::max(max_words, static_cast<int64_t>(s.W));
        max_jobs = std::max(max_jobs, static_cast<int>(s.jobs.size()));
        const int64_t bx = rsr::grad_blocks(s.max_N);
        max_grad = std::max(max_grad, static_cast<int64_t>(s.jobs.size()) *
                                          (static_cast<int64_t>(s.W) * bx * 32 + bx));
    }
    // The persistent cascade's compact buffers hold per-block regions with
    // some slack beyond the segment's samples; its state holds one ticket per
    // group of them.
    int64_t cap = max_total, state_words = 0;
    for (const Segment& s : p->segs) {
        if (!s.refs->consistent || !rsr::casc_persist_supported(s.refs)) continue;
        const int64_t sc = rsr::casc_persist_stride(s.refs, s.total, ctx->cu_count);
        cap = std::max(cap, sc);
    }
    for (const Segment& s : p->segs) {
        if (!s.refs->consistent || !rsr::casc_persist_supported(s.refs)) continue;
        state_words = std::max(state_words, rsr::casc_persist_state_words(cap, s.refs->KS));
    }
    p->casc_cap = cap;
    p->casc_w = static_cast<int>(max_words);
    p->casc_state_words = state_words;
    hipError_t e = hipSuccess;
    auto dmalloc = [&](void** ptr, size_t bytes) {
        if (e == hipSuccess) e = rsr::dev_malloc(ptr, bytes > 0 ? bytes : 8);
    };
    dmalloc(reinterpret_cast<void**>(&p->d_jobs), sizeof(rsr::JobDev) * host_jobs.size());
    dmalloc(reinterpret_cast<void**>(&p->d_offsets), sizeof(int64_t) * host_offsets.size());
    dmalloc(reinterpret_cast<void**>(&p->d_counts), sizeof(uint64_t) * 8 * n_jobs);
    dmalloc(reinterpret_cast<void**>(&p->d_count_part),
            sizeof(uint64_t) * 8 * rsr::kMaxReduceBlocks * max_jobs);
    dmalloc(reinterpret_cast<void**>(&p->d_grad_part), sizeof(uint32_t) * max_grad);
    dmalloc(reinterpret_cast<void**>(&p->d_casc_words),
            sizeof(uint32_t) * 2 * static_cast<size_t>(max_words) * cap);
    dmalloc(reinterpret_cast<void**>(&p->d_casc_index), sizeof(int32_t) * 4 * cap);
    if (state_words > 0)
        dmalloc(reinterpret_cast<void**>(&p->d_casc_state),
                sizeof(uint32_t) * static_cast<size_t>((state_words + 1) / 2 * 2));
    dmalloc(reinterpret_cast<void**>(&p->d_casc_counters),
            sizeof(uint64_t) * rsr::CascadeBuffers::kCounterU64);
    dmalloc(reinterpret_cast<void**>(&p->d_list), sizeof(int32_t) * max_total);
    dmalloc(reinterpret_cast<void**>(&p->d_list_counter), sizeof(uint64_t) * 2);
    dmalloc(reinterpret_cast<void**>(&p->d_G_all), sizeof(float) * p->G_total);
    if (e == hipSuccess)
        e = rsr::host_malloc(&p->h_counts, sizeof(uint64_t) * (8 * n_jobs + 1));
    if (e == hipSuccess)
        e = rsr::host_malloc(&p->h_G_all, sizeof(float) * (p->G_total + 1));
    if (e == hipSuccess)
        e = hipMemcpy(p->d_jobs, host_jobs.data(), sizeof(rsr::JobDev) * host_jobs.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->d_offsets, host_offsets.data(), sizeof(int64_t) * host_offsets.size(),
                      hipMemcpyHostToDevice);
    // The persistent cascade's time-out flag (counters[15]) must read 0 in
    // the tuner's trials too.
    if (e == hipSuccess) e = hipMemset(p->d_casc_counters, 0, sizeof(uint64_t) * 16);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        free_plan(p);
        return phip(ctx, e, "rsr_plan_create allocation");
    }
    // Work enqueued on the context stream before this call must be finished
    // before the tuner touches the jobs' buffers.
    e = ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_plan(p);
        return phip(ctx, e, "rsr_plan_create sync");
    }
    if (tune) {
        bool added = false;
        for (size_t si = 0; si < p->segs.size(); ++si) {
            Segment& sg = p->segs[si];
            const std::string key = segment_key(ctx, sg);
            auto it = cache.find(key);
            if (it != cache.end()) {
                const TuneEntry& te = it->second;
                sg.choice = static_cast<Choice>(te.choice);
                sg.shape = rsr::CascadeShape{te.first, te.growth, te.split, te.tail != 0, te.tail == 2,
                                             te.chunks};
                sg.tuned_ms = static_cast<float>(te.ms);
                // A stored choice the handle cannot run (no matrix-core
                // operands, or a cascade on inconsistent rows) is retimed.
                if (choice_runs(sg)) continue;
            }
            rsr_status st = tune_segment(p, static_cast<int>(si));
            if (st != RSR_OK) {
                free_plan(p);
                return st;
            }
            TuneEntry te;
            te.choice = sg.choice;
            te.first = sg.shape.first;
            te.growth = sg.shape.growth;
            te.split = sg.shape.split_rows;
            te.chunks = sg.shape.max_chunks;
            te.tail = sg.shape.mfma_head ? 2 : (sg.shape.mfma_tail ? 1 : 0);
            te.ms = sg.tuned_ms;
            cache[key] = te;
            added = true;
        }
        if (added && !cache_path.empty()) {
            rsr_status st = write_cache(ctx, cache_path, cache);
            if (st != RSR_OK) {
                free_plan(p);
                return st;
            }
        }
    }
    // Record the whole plan.
    e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = rsr::launch_fill_u64(p->cap, p->d_casc_counters + 15, 1, 0);
    for (size_t si = 0; si < p->segs.size() && e == hipSuccess; ++si) {
        const Segment& s = p->segs[si];
        e = enqueue_sample(p, static_cast<int>(si), p->cap);
        if (e == hipSuccess) e = enqueue_classify(p, static_cast<int>(si), p->cap, s.choice, s.shape);
        if (e == hipSuccess) e = enqueue_rest(p, static_cast<int>(si), p->cap);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->h_counts, p->d_counts, sizeof(uint64_t) * 8 * n_jobs,
                           hipMemcpyDeviceToHost, p->cap);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->h_counts + 8 * static_cast<size_t>(n_jobs), p->d_casc_counters + 15,
                           sizeof(uint64_t), hipMemcpyDeviceToHost, p->cap);
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->h_G_all, p->d_G_all, sizeof(float) * p->G_total,
                           hipMemcpyDeviceToHost, p->cap);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(p->cap, &graph);
    if (e == hipSuccess) e = e2;
    p->graph = graph;
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        free_plan(p);
        return phip(ctx, e, "rsr_plan_create capture");
    }
    *out = p;
    return RSR_OK;
}

rsr_status rsr_plan_run(rsr_plan* p) {
    if (!p) return RSR_EINVAL;
    PLAN_HIP(p->ctx, hipGraphLaunch(p->exec, p->ctx->stream));
    return RSR_OK;
}

rsr_status rsr_plan_results(rsr_plan* p, rsr_estimate_t* est, float* G_host) {
    if (!p) return RSR_EINVAL;
    if (!est) return pfail(p->ctx, RSR_EINVAL, "NULL estimate array");
    rsr_ctx* ctx = p->ctx;
    PLAN_HIP(ctx, ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize());
    if (p->h_counts[8 * p->jobs.size()] != 0)
        return pfail(ctx, RSR_EHIP, "a persistent classification timed out at a grid barrier");
    size_t g_off = 0;
    for (size_t j = 0; j < p->jobs.size(); ++j) {
        const uint64_t* c = p->h_counts + static_cast<size_t>(p->pos[j]) * 8;
        const rsr_job& jb = p->jobs[j];
        rsr_estimate_t& o = est[j];
        o.n_L = c[0];
        o.n_U = c[1];
        o.n_u = c[2];
        o.n_both = c[3];
        o.n_u_up = c[4];
        o.N = static_cast<uint64_t>(jb.N);
        const double Nd = static_cast<double>(jb.N);
        o.p_L = static_cast<double>(o.n_L) / Nd;
        o.p_U = static_cast<double>(o.n_U) / Nd;
        o.p_u = static_cast<double>(o.n_u) / Nd;
        const double P = static_cast<double>(o.n_U + o.n_u_up) / Nd;
        o.P = P;
        o.se = std::sqrt(P * (1.0 - P) / Nd);
        o.cov = P > 0.0 ? std::sqrt((1.0 - P) / (Nd * P)) : HUGE_VAL;
        const size_t gsz = static_cast<size_t>(jb.model->n) * jb.model->K;
        if (G_host && jb.d_G)
            std::memcpy(G_host + g_off, p->h_G_all + p->host_g_off[p->pos[j]], sizeof(float) * gsz);
        g_off += gsz;
    }
    return RSR_OK;
}

rsr_status rsr_plan_destroy(rsr_plan* p) {
    if (!p) return RSR_EINVAL;
    rsr_ctx* ctx = p->ctx;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    free_plan(p);
    return RSR_OK;
}

}  // extern "C"
