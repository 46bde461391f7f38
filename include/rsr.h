/*
 * rsr.h - C ABI of the MI355X (gfx950) library for the Stage-2 hot path of the
 * Reference-state System Reliability (RSR) method, Byun, Ryu & Song,
 * arXiv 2604.17066.
 *
 * The hot path, for one target system level:
 *   rsr_sample        draw Monte Carlo component-state samples (section 3.1)
 *   rsr_classify      classify them against lower / upper reference states
 *                     (section 3.3, Algorithm 1, eq. violation_matrix)
 *   rsr_eval_unknown  evaluate the system function on unclassified samples
 *                     (section 3.5, Stage 2)
 *   rsr_estimate      reduce labels to probability estimates (section 3.3.1)
 *   rsr_grad          score-function partials dP/dp[i][s]
 * and, for Stage 1, rsr_boundary_search (new reference states from
 * unclassified samples, section 3.4) and the loop around it, rsr_stage1,
 * plus handles for the problem data (component-state probabilities,
 * reference states, system function) and a batched plan that runs many
 * (model, system) jobs in one captured HIP graph.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named d_* are device pointers owned by the caller; every other
 *   pointer is host memory owned by the caller and only read during the call
 *   (handles copy what they need).
 * - All device work is enqueued on the HIP stream given to rsr_ctx_create, in
 *   call order.  Only rsr_estimate, rsr_plan_results and the *_create calls
 *   synchronise with the host.
 * - Every call returns an rsr_status.  Nothing throws or aborts across the
 *   ABI.  On failure the context keeps a message (rsr_last_error).  Inputs are
 *   validated before any launch; asynchronous device faults surface as
 *   RSR_EHIP at the next synchronising call.
 * - A context is not thread-safe; use one per host thread.
 * - Handles (models, reference sets, systems, plans) belong to the context
 *   that created them and must be destroyed before it.
 *
 * State encoding (the layout of d_samples)
 * ----------------------------------------
 * n components with K ordered states 0..K-1 (the paper's N and M, section
 * 2.1).  A state vector x is stored as K-1 thermometer planes t_j = [x >= j],
 * j = 1..K-1, plane-major, each plane padded to whole 32-bit words:
 *   PW = ceil(n / 32) words per plane, W = (K-1) * PW words per sample,
 *   bit (i mod 32) of word (j-1)*PW + i/32  =  [x_i >= j],  pad bits are 0.
 * Samples are stored word-major: word w of sample h is d_samples[w * N + h].
 * Componentwise x <= r holds iff t(x) AND NOT t(r) is all zero, and x >= r
 * iff t(r) AND NOT t(x) is all zero, which is the zero test of the paper's
 * violation matrix (section 3.3.2) on a K-1 bit code per component instead
 * of the paper's K-bit one-hot / down-set / up-set code.
 */
#ifndef RSR_H
#define RSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RSR_OK = 0,
    RSR_EINVAL = 1,       /* an argument failed validation; nothing was launched */
    RSR_ENOMEM = 2,       /* a device or pinned-host allocation failed */
    RSR_EHIP = 3,         /* a HIP runtime call failed (message has the HIP error) */
    RSR_EUNSUPPORTED = 4  /* valid request outside the library's limits */
} rsr_status;

enum { RSR_LABEL = 0, RSR_COUNT = 1 };                  /* rsr_classify mode */
enum { RSR_AUTO = 0, RSR_POPCOUNT = 1, RSR_MFMA = 2, RSR_MFMA_FP4 = 3, RSR_PERSIST = 4 };  /* rsr_classify form */
enum { RSR_UNKNOWN_ONLY = 0, RSR_ALL = 1 };             /* rsr_eval_unknown which */
enum { RSR_SYS_ST_CONNECTIVITY = 1, RSR_SYS_GLOBAL_CONNECTIVITY = 2, RSR_SYS_MAX_FLOW = 3,
       RSR_SYS_HOST_CALLBACK = 4 };  /* rsr_system_desc kind */

/* Limits of the library. */
#define RSR_MAX_K 16
#define RSR_MAX_BITS 4096   /* n * (K-1) */
#define RSR_MAX_NODES 4096

typedef struct rsr_ctx rsr_ctx;
typedef struct rsr_model rsr_model;
typedef struct rsr_refs rsr_refs;
typedef struct rsr_system rsr_system;
typedef struct rsr_plan rsr_plan;

/* Estimates (section 3.3.1).  Counts: n_L = #{lower-classified}, n_U =
 * #{upper-classified and not lower}, n_u = #{unclassified}, n_both = #{samples
 * with both flags} (0 for valid reference sets), n_u_up = #{unclassified with
 * Y = 1}, N = samples.  p_L, p_U, p_u = the three counts over N;
 * P = (n_U + n_u_up) / N estimates P(S >= level); se = sqrt(P (1-P) / N);
 * cov = sqrt((1-P) / (N P)), +inf at P = 0.  Every division is in fp64 in
 * exactly this form, so results are reproducible bit for bit. */
typedef struct {
    uint64_t n_L, n_U, n_u, n_both, n_u_up, N;
    double p_L, p_U, p_u, P, se, cov;
} rsr_estimate_t;

/* System function description (section 2.1).  Graph systems: components are
 * the undirected edges (edge_u[e], edge_v[e]) of a graph with n_nodes nodes;
 * n_edges = n.
 *   RSR_SYS_ST_CONNECTIVITY: Phi = 1 when sink is reachable from source over
 *     edges whose state is at least `level` (1 <= level <= K-1), else 0:
 *     single-OD connectivity for K = 2 (section 4.1), and for K > 2 the
 *     level-`level` bottleneck system, one target state of section 3.5's
 *     multi-state workflow (the paper fixes no multi-state s-t function;
 *     this one is coherent in every component).
 *   RSR_SYS_GLOBAL_CONNECTIVITY: edges work when their state is at least 1;
 *     the system state is 0 when some node is cut off from the rest, 1 when
 *     the working edges connect every node but some single edge failure
 *     would disconnect them, 2 when every pair of nodes keeps two
 *     edge-disjoint paths (no bridge); Phi = 1 when that state is at least
 *     `level` (1 or 2) (sections 4.2 and 4.5).  source and sink are unused.
 *   RSR_SYS_MAX_FLOW: edge e carries up to x_e units of flow in either
 *     direction; the system state is the maximum flow from source to sink,
 *     and Phi = 1 when it is at least `level` (the demand d >= 1).  Its
 *     reference states are the d-minimal path and cut vectors (section 2.2).
 * Any other coherent system function (section 2.1 only asks that Phi be
 * non-decreasing in every component state):
 *   RSR_SYS_HOST_CALLBACK: phi(x, n, user) is called on the host with a state
 *     vector x (n bytes, states 0..K-1, valid only during the call) and
 *     returns the system state S >= 0; Phi = 1 when S >= `level` (>= 1).
 *     n_edges = n; the graph fields are unused and may be 0 / NULL.  phi is
 *     called from the thread that calls the library, one state at a time,
 *     and must not call the library.  A negative return aborts the call that
 *     made it with RSR_EINVAL. */
typedef struct {
    int32_t kind;       /* one of the RSR_SYS_* kinds */
    int32_t n_nodes;    /* graph systems: 2..RSR_MAX_NODES */
    int32_t n_edges;    /* = n, the number of components */
    int32_t K;          /* states per component */
    const int32_t* edge_u;  /* host [n_edges], node ids in [0, n_nodes) */
    const int32_t* edge_v;  /* host [n_edges] */
    int32_t source, sink;   /* distinct node ids (s-t connectivity and max flow) */
    int32_t level;
    int32_t (*phi)(const uint8_t* x, int32_t n, void* user);  /* RSR_SYS_HOST_CALLBACK */
    void* user;             /* passed to phi unchanged */
} rsr_system_desc;

/* ---- context ------------------------------------------------------------ */

/* Creates a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  EHIP if the device is absent. */
rsr_status rsr_ctx_create(int device, void* hip_stream, rsr_ctx** out);
rsr_status rsr_ctx_destroy(rsr_ctx* ctx);
/* Message of the last failed call on ctx ("" if none).  Valid until the next
 * call on ctx. */
const char* rsr_last_error(const rsr_ctx* ctx);
const char* rsr_status_str(rsr_status s);

/* Words per sample, W = (K-1) * ceil(n/32); 0 for invalid n or K. */
size_t rsr_words(int32_t n, int32_t K);

/* Host helper, no device: inverse-CDF thresholds of a model (section 3.1).
 * p is host [n][K] with rows of probabilities; C is host [n][K-1] with
 * C[i][s-1] = min(floor(2^32 * (p[i][0] + ... + p[i][s-1])), 2^32), the sum
 * formed left to right in fp64.  A sample's component i is in state
 * #{s : u >= C[i][s-1]} for its 32-bit uniform word u.  EINVAL on a
 * non-finite entry, an entry outside [0,1] or a row sum off 1 by > 1e-9. */
rsr_status rsr_thresholds(int32_t n, int32_t K, const double* p, uint64_t* C);

/* ---- problem data handles ---------------------------------------------- */

/* Model: n independent components with state probabilities p (host [n][K],
 * row i = P(X_i = 0..K-1); section 2.1).  Validates p as rsr_thresholds does,
 * then copies thresholds and probabilities to the device (synchronous). */
rsr_status rsr_model_create(rsr_ctx* ctx, int32_t n, int32_t K, const double* p,
                            rsr_model** out);
rsr_status rsr_model_destroy(rsr_model* model);
/* Replaces the probabilities of a model (same n and K) without allocating:
 * validates p as rsr_model_create does, then uploads the new thresholds and
 * probabilities through the model's pinned staging buffer on the context
 * stream.  Asynchronous: work enqueued on the stream before the call sees
 * the old values, work enqueued after it the new ones.  If the previous
 * upload has not yet left the staging buffer, the call first waits for it.
 * EINVAL as for rsr_model_create (the model is then unchanged). */
rsr_status rsr_model_update(rsr_model* model, const double* p);

/* Reference states for one target level (section 2.2, sets L(m') and U(m')):
 * lower = host [R_L][n] uint8 states, each certifying S < level for every
 * x <= row; upper = host [R_U][n], each certifying S >= level for every
 * x >= row.  Rows need not be antichains: duplicates and dominated rows are
 * legal.  R_L = 0 or R_U = 0 is legal (nothing matches on that side).
 * EINVAL on a state >= K.  The handle holds packed device copies and can be
 * reused with any model of the same n and K (section 5). */
rsr_status rsr_refs_create(rsr_ctx* ctx, int32_t n, int32_t K, const uint8_t* lower,
                           int64_t R_L, const uint8_t* upper, int64_t R_U, rsr_refs** out);
rsr_status rsr_refs_destroy(rsr_refs* refs);
/* *out = 1 when no upper row lies below a lower row (checked on the device
 * at creation).  Then no sample can be dominated on both sides (valid
 * reference sets always pass; section 2.2), and rsr_classify in RSR_LABEL mode
 * stops at a sample's first match on either side.  Rows are kept in order of
 * increasing size (fewest constrained components first); no result depends on
 * the order. */
rsr_status rsr_refs_consistent(const rsr_refs* refs, int32_t* out);

/* System function handle: copies the graph to the device.  EINVAL on a node
 * id out of range; for s-t connectivity on source == sink or level outside
 * 1..K-1; for global connectivity on level outside 1..2; for max flow on
 * source == sink or level outside 1..255.  EUNSUPPORTED when the per-sample
 * search state of global connectivity or max flow exceeds 64 KB of LDS per
 * four samples (about 2800 nodes at 4096 edges). */
rsr_status rsr_system_create(rsr_ctx* ctx, const rsr_system_desc* desc, rsr_system** out);
rsr_status rsr_system_destroy(rsr_system* sys);

/* ---- hot path ------------------------------------------------------------ */

/* Draws samples first_sample .. first_sample+N-1 of the model into
 * d_samples (device [W][N] u32, layout above).  The 32-bit uniform word u of
 * component i of sample h is built from Philox4x32-10 (Salmon et al., SC'11)
 * blocks with key (low32(seed), high32(seed)): its high 16 bits are the half
 * at position j = i mod 8 (half j mod 2 of word j div 2, low half first) of
 * the block with counter (i div 8, low32(h), high32(h), stream_id), its low 16
 * bits the half at the same position of the block with counter
 * ((i div 8) | 2^31, low32(h), high32(h), stream_id).  The state is
 * #{s : u >= C[i][s]} with the thresholds of rsr_thresholds.  Any sample range
 * can therefore be drawn independently and reproduced on any device or host.
 * EINVAL: N <= 0, NULL pointer. */
rsr_status rsr_sample(rsr_ctx* ctx, const rsr_model* model, uint64_t seed, uint32_t stream_id,
                      uint64_t first_sample, int64_t N, uint32_t* d_samples);

/* Dominance classification (section 3.3, Algorithm 1).  For each sample h:
 *   RSR_LABEL: bit0 of d_flags[h] = some lower row r has x_h <= r;
 *              bit1 = some upper row r has x_h >= r, tested only when bit0 is
 *              clear (Algorithm 1 gives the lower set precedence), else 0.
 *   RSR_COUNT: both bits exact; if d_match is not NULL, d_match[2h] and
 *              d_match[2h+1] receive the number of matching lower and upper
 *              rows (u32, device [N][2]).
 * form selects the kernel: RSR_POPCOUNT (bit-packed AND-NOT on the vector
 * ALU), RSR_MFMA (int8 matrix-core contraction of eq. violation_matrix, COUNT
 * and LABEL modes alike), RSR_MFMA_FP4 (the same contraction with FP4 E2M1
 * operands 0 / +-1 and fp32 accumulation, exact because every partial sum
 * is a small integer), RSR_AUTO (the cascade for LABEL mode on consistent
 * rows, else the FP4 form up to 1280 bits, else the popcount form),
 * RSR_PERSIST (the cascade with its rounds after round 0 in one persistent,
 * cooperative launch; its grid barriers wait with a time limit, and a
 * barrier that timed out is reported as RSR_EHIP by the next rsr_estimate).
 * The automatic cascade runs one launch per round, each round after round 0
 * 6 times the rows of the one before, 8 times from 16384 rows per side on.
 * Every form returns identical outputs.  EINVAL: refs built for another n/K,
 * N <= 0, NULL d_flags.  EUNSUPPORTED: a matrix-core form (RSR_PERSIST
 * included) with n*(K-1) > 1280; RSR_PERSIST in COUNT mode, on inconsistent
 * rows or with N > 2^31-1. */
rsr_status rsr_classify(rsr_ctx* ctx, const rsr_refs* refs, const uint32_t* d_samples,
                        int64_t N, int32_t mode, int32_t form, uint8_t* d_flags,
                        uint32_t* d_match);

/* Stage-2 evaluation of the system function (section 3.5).  d_Y (device [N]
 * u8) receives, for RSR_UNKNOWN_ONLY: 0 for a lower-flagged sample (bit0),
 * 1 for an upper-flagged one (bit1 without bit0), Phi(x_h) for the others;
 * for RSR_ALL: Phi(x_h) for every sample (plain Monte Carlo; d_flags may then
 * be NULL).  Phi is evaluated by a batched breadth-first search on the device.
 * d_n_evaluated (device u64, may be NULL) receives the number of Phi
 * evaluations.  EINVAL: system built for another n/K, N <= 0. */
rsr_status rsr_eval_unknown(rsr_ctx* ctx, const rsr_system* sys, const uint32_t* d_samples,
                            int64_t N, const uint8_t* d_flags, int32_t which, uint8_t* d_Y,
                            uint64_t* d_n_evaluated);

/* Reduces flags (and Y, if not NULL) to counts on the device, copies them to
 * the host and fills *out as rsr_estimate_t says.  It returns when the counts
 * have reached the host: every earlier operation of the context's stream has
 * then ended, and the counting kernel has read all of flags and Y (with
 * 16-byte aligned flags and Y that kernel's last block publishes the counts
 * and the host returns at once; its exit may still be in flight, ordered
 * before any later work of the stream).
 * With d_Y == NULL, n_u_up = 0 and P, se, cov are NaN (bounds only).
 * EHIP: a device error, or a persistent cascade since the previous call
 * whose grid barrier timed out (the flag is cleared with the report). */
rsr_status rsr_estimate(rsr_ctx* ctx, const uint8_t* d_flags, const uint8_t* d_Y, int64_t N,
                        rsr_estimate_t* out);

/* Score-function partials of P = E[Y] with respect to the state
 * probabilities (independent components make P multilinear in them):
 *   c[i][s] = #{h : Y_h = 1 and x_{h,i} = s}          (exact, u64)
 *   G[i][s] = c[i][s] / (N * p[i][s])  in fp32, 0 where p[i][s] = 0,
 * computed as (float)c / ((float)N * (float)p).  For K = 2 with p[i][1] the
 * survival probability, dP/dp_i = G[i][1] - G[i][0] (Birnbaum importance).
 * d_G is device [n][K] f32; d_counts is device [n][K] u64 or NULL.
 * d_samples must hold the samples of `model` that produced d_Y. */
rsr_status rsr_grad(rsr_ctx* ctx, const rsr_model* model, const uint32_t* d_samples,
                    const uint8_t* d_Y, int64_t N, float* d_G, uint64_t* d_counts);

/* Binary Birnbaum importance (K = 2 with p[i][1] the survival probability of
 * component i and p[i][0] = 1 - p[i][1]): the derivative of P along that
 * constraint, I_i = dP/dp[i][1] - dP/dp[i][0] = c[i][1] / (N p[i][1]) -
 * c[i][0] / (N p[i][0]), with the counts c of rsr_grad, each quotient formed
 * in fp64 from the model's fp64 probabilities (0 where p = 0) and the
 * difference rounded once to fp32.  d_I is device [n] f32.  EINVAL: K != 2,
 * NULL argument, N <= 0. */
rsr_status rsr_importance(rsr_ctx* ctx, const rsr_model* model, const uint32_t* d_samples,
                          const uint8_t* d_Y, int64_t N, float* d_I);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * rsr_eval_unknown without any allocation.  Same arguments, outputs and
 * errors as rsr_eval_unknown, except that the list of unclassified samples
 * and its counter live in a fixed scratch array of the library, one per
 * device, of 16 MiB + 64 bytes, held until the process ends; so N is limited
 * to 2^22 samples (EINVAL beyond), and host-callback systems, which stage
 * samples in allocated host and device memory, are EUNSUPPORTED.  The
 * counter is cleared by a kernel at the start of every call.  Every call on
 * one device shares that device's scratch: calls that overlap on one device
 * (on different streams or from different host threads) race, so the
 * caller must order them. */
rsr_status rsr_eval_unknown_noalloc(rsr_ctx* ctx, const rsr_system* sys,
                                    const uint32_t* d_samples, int64_t N,
                                    const uint8_t* d_flags, int32_t which, uint8_t* d_Y,
                                    uint64_t* d_n_evaluated);

/* ---- Stage 1: new reference states -------------------------------------- */

/* Componentwise boundary search (section 3.4, fig. x1x2_find_ref) from the
 * samples d_pick[0..n_pick-1] (device i64 indices into the N samples of
 * d_samples, drawn for a model with the system's n and K).  For each start
 * x the components are visited in index order; each is moved one state at a
 * time towards K-1 when Phi(x) says S < level (a failure sample), or towards
 * 0 when S >= level (a survival sample), and the step that changes the side
 * is undone, which ends that component's walk.  The result is a maximal
 * failure state (a new lower reference state) or a minimal survival state
 * (a new upper one):
 *   d_rows  device [n_pick][n] u8: the boundary state of pick j in row j
 *   d_side  device [n_pick] u8:   0 lower, 1 upper, 0xFF if d_pick[j] is not
 *                                 in 0..N-1 (row j is then left untouched).
 * For s-t connectivity at a level the side depends only on which edges reach
 * the level, so a failure result holds every edge at K-1 or level-1 and a
 * survival result at level or 0.  Rows from different picks may coincide.
 * EINVAL: NULL argument, N out of 1..2^31-1, n_pick < 0.  n_pick = 0 is a
 * no-op. */
rsr_status rsr_boundary_search(rsr_ctx* ctx, const rsr_system* sys, const uint32_t* d_samples,
                               int64_t N, const int64_t* d_pick, int64_t n_pick,
                               uint8_t* d_rows, uint8_t* d_side);

/* Stage 1 of the workflow (section 3.5, Stage 1 of fig. rsr_alg): alternate
 * sample classification and boundary search until the unclassified fraction
 * of a fresh sample set falls below eps_u or the reference sets reach
 * max_rows rows.  Iteration it (0, 1, ...):
 *   1. draw N samples with key `seed` and stream_id = it (rsr_sample);
 *   2. classify them against the current rows in LABEL mode;
 *   3. p_u = (unclassified samples) / N; stop if p_u < eps_u, if the rows
 *      number max_rows or more, or if it + 1 = max_iters;
 *   4. search from the first `picks` unclassified samples in index order
 *      (the paper picks one at random per iteration; samples are i.i.d., so
 *      the lowest-index ones are a uniformly random subset, and picks > 1
 *      finds that many rows per sample set);
 *   5. append each new row to its side in pick order, dropping rows already
 *      present and stopping at max_rows rows in total.
 * A row found from an unclassified sample is never dominated by an existing
 * row of a valid reference set (the sample would have been classified), so
 * exact duplicates are the only redundancy to remove.  Rows are host
 * [R][n] u8, in discovery order after the initial rows (lower0 / upper0,
 * which may be NULL with R = 0).  lower / upper must hold cap_L / cap_U rows;
 * both must be at least max_rows.  Synchronous. */
typedef struct {
    int64_t N;          /* samples per iteration, 1..2^31-1 */
    int64_t picks;      /* unclassified samples searched per iteration, >= 1 */
    double eps_u;       /* target unclassified fraction */
    int64_t max_rows;   /* cap on R_L + R_U */
    int32_t max_iters;  /* cap on iterations, >= 1 */
    uint64_t seed;
} rsr_stage1_params;

typedef struct {
    int32_t iterations;  /* sample sets drawn and classified */
    double p_u;          /* unclassified fraction of the last sample set */
    int64_t R_L, R_U;    /* rows returned */
    int64_t searches;    /* boundary searches run */
    int64_t duplicates;  /* search results dropped as already present */
} rsr_stage1_result;

rsr_status rsr_stage1(rsr_ctx* ctx, const rsr_model* model, const rsr_system* sys,
                      const rsr_stage1_params* params, const uint8_t* lower0, int64_t R_L0,
                      const uint8_t* upper0, int64_t R_U0, uint8_t* lower, int64_t cap_L,
                      uint8_t* upper, int64_t cap_U, rsr_stage1_result* result);

/* ---- batched plan -------------------------------------------------------- */

/* One job = the full hot path (sample, classify in LABEL mode, evaluate the
 * unclassified samples, count, gradient) for one model against one
 * reference set and system.  Buffers are caller-owned device memory:
 * d_samples [W][N] u32, d_flags [N] u8, d_Y [N] u8, d_G [n][K] f32 (NULL:
 * no gradient). */
typedef struct {
    const rsr_model* model;
    const rsr_refs* refs;
    const rsr_system* sys;
    uint64_t seed;
    uint32_t stream_id;
    int64_t N;
    uint32_t* d_samples;
    uint8_t* d_flags;
    uint8_t* d_Y;
    float* d_G;
} rsr_job;

/* Builds a plan for n_jobs jobs: chooses a kernel configuration per job shape,
 * orders the work, and records every launch of every job into one HIP graph.
 * The configuration of a segment (the jobs sharing a reference set and a
 * system) is chosen by timing candidates on its own samples (its first jobs,
 * at least 2^22 samples, or all of them when it has fewer), with results
 * kept in a tuning cache:
 *   tune_cache NULL:  no timing; every segment takes the default
 *                     configuration (the automatic classification form);
 *   tune_cache "":    every segment is timed, nothing is stored;
 *   a file path:      a JSON object whose keys name a device and a segment
 *                     shape (device name, CU count, packed words W, R_L, R_U,
 *                     consistency, matrix-core operands, jobs and samples per
 *                     job) and whose values are the chosen configuration:
 *                     {"choice": 0 cascade, 1 popcount per job, 2 int8
 *                     per job, 3 FP4 per job, 4 persistent cascade;
 *                     "first", "growth", "split": the cascade's round
 *                     rows; "tail": 0 popcount rounds, 1 FP4 rounds after
 *                     round 0, 2 FP4 rounds from round 0 on; "chunks"
 *                     (optional on reading): most chunks of a split round,
 *                     0 for the library's own caps; "ms": the
 *                     segment's classification time, timed on those
 *                     samples and scaled to all of them}.
 *                     Segments whose key is present take the stored choice
 *                     without timing; the others are timed, and the file is
 *                     rewritten (via a temporary file and a rename) with the
 *                     new entries added.  A missing file counts as empty.
 * The plan keeps the job array's pointers, so the handles and buffers must
 * outlive it.  Synchronous.  EINVAL: bad job (NULL handle, n/K mismatch),
 * a tuning cache that is not such a JSON object.  EUNSUPPORTED: a job whose
 * system is RSR_SYS_HOST_CALLBACK (host work cannot run inside the graph). */
rsr_status rsr_plan_create(rsr_ctx* ctx, const rsr_job* jobs, int32_t n_jobs,
                           const char* tune_cache, rsr_plan** out);
/* Launches the plan's graph on the context stream (asynchronous). */
rsr_status rsr_plan_run(rsr_plan* plan);
/* Synchronises and copies the per-job estimates (host [n_jobs]) and, if
 * G_host is not NULL, every job's gradient concatenated in job order (host,
 * sum of n*K floats).  EHIP: a device error, or a persistent cascade of the
 * run whose blocks did not all reach a grid barrier within its time limit
 * (its flags are then not to be trusted). */
rsr_status rsr_plan_results(rsr_plan* plan, rsr_estimate_t* est, float* G_host);
rsr_status rsr_plan_destroy(rsr_plan* plan);

/* ---- testing ---------------------------------------------------------------- */

/* Failure injection for tests of the error paths: after `after` more
 * successful device or pinned-host allocations made by the library (on any
 * context), the next one fails as if the device were out of memory (the call
 * that made it returns RSR_ENOMEM and releases what it had allocated); later
 * allocations succeed again.  A negative `after` disarms it.  Not
 * thread-safe with respect to concurrent library calls. */
rsr_status rsr_debug_fail_alloc(int64_t after);

/* For tests of the persistent cascade's time-out path: its grid barriers
 * then wait at most `ticks` ticks of the 100 MHz real-time counter (0: a
 * block that has to wait at all gives up at once, sets the error flag and
 * leaves, so every launch still ends); a negative value restores the
 * default of 10 s.  Applies to launches made after the call, on every
 * context, and to plans recorded after it (a plan keeps the limit it was
 * recorded with).  Not thread-safe with respect to concurrent library
 * calls. */
rsr_status rsr_debug_barrier_timeout(int64_t ticks);

#ifdef __cplusplus
}
#endif
#endif /* RSR_H */
