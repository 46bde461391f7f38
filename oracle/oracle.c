/*
 * Plain CPU oracle for the Stage-2 hot path of the Reference-state System
 * Reliability (RSR) method (Byun, Ryu & Song, arXiv 2604.17066).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU path: component states are plain uint8 values, every
 * test is the textbook definition written as loops, and the random generator
 * is an independent implementation of Philox4x32-10 written from its
 * published description (Salmon, Moraes, Dror & Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11, section 3.2).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (see build.py).
 * -ffp-contract=off keeps the few floating-point expressions in the order in
 * which they are written, so that the estimator values are reproducible.
 *
 * Notation.  n components, each with K ordered states 0..K-1 (the paper's N and
 * M, section 2.1).  A component-state vector x is a row of n uint8 values.
 * The partial order x <= y is componentwise (section 2.2).  A lower reference
 * state r certifies S <= m' for every x <= r; an upper reference state r
 * certifies S >= m'+1 for every x >= r (section 2.2, sets L(m') and U(m')).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Threads                                                                    */
/* ------------------------------------------------------------------------- */

void or_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

int or_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (SC'11, section 3.2)                                         */
/* ------------------------------------------------------------------------- */
/* One round maps the counter (c0,c1,c2,c3) with round key (k0,k1) to
 *   (hi(B*c2) ^ c1 ^ k0, lo(B*c2), hi(A*c0) ^ c3 ^ k1, lo(A*c0))
 * with the two multipliers A and B given in the paper.  The key is bumped by
 * the two Weyl constants before every round after the first. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    const uint32_t mulA = 0xD2511F53u, mulB = 0xCD9E8D57u;
    const uint32_t weyl0 = 0x9E3779B9u, weyl1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += weyl0;
            k1 += weyl1;
        }
        uint64_t prodA = (uint64_t)mulA * (uint64_t)c0;
        uint64_t prodB = (uint64_t)mulB * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(prodB >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)prodB;
        uint32_t n2 = (uint32_t)(prodA >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)prodA;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------- */
/* Sampling of independent component states                                  */
/* ------------------------------------------------------------------------- */
/* The paper assumes P(X) can be sampled (section 3.1) and, in its examples,
 * independent components.  Component i takes state s with probability
 * p[i][s].  Inverse-CDF with integer thresholds: with a 32-bit uniform word u,
 *   x_i = #{ s in 1..K-1 : u >= C[i][s] },  C[i][s] = floor(2^32 * sum_{s'<s} p[i][s'])
 * clamped to [0, 2^32].  The cumulative sum is formed left to right in fp64. */
int or_thresholds(int n, int K, const double* p, uint64_t* C) {
    if (n <= 0 || K < 2) return 1;
    for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int s = 1; s < K; ++s) {
            acc = acc + p[(size_t)i * K + (s - 1)];
            double scaled = floor(acc * 4294967296.0);
            uint64_t c;
            if (!(scaled > 0.0)) c = 0;
            else if (scaled >= 4294967296.0) c = 4294967296ull;
            else c = (uint64_t)scaled;
            C[(size_t)i * (K - 1) + (s - 1)] = c;
        }
    }
    return 0;
}

/* 16-bit half at position j (0..7) of a Philox block: half (j mod 2) of word
 * (j div 2), half 0 being the low 16 bits. */
static uint32_t block_half(const uint32_t out[4], int j) {
    return (out[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
}

/* The 32-bit uniform word of component i of sample h.  Its high 16 bits are
 * the half at position (i mod 8) of the Philox4x32-10 block with counter
 * (i div 8, low32(h), high32(h), stream_id); its low 16 bits are the half at
 * the same position of the block whose first counter word also has bit 31
 * set.  Key (low32(seed), high32(seed)) for both. */
static uint32_t draw_word(uint64_t seed, uint32_t stream_id, uint64_t h, int i) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t hi_ctr[4] = {(uint32_t)(i >> 3), (uint32_t)h, (uint32_t)(h >> 32), stream_id};
    uint32_t lo_ctr[4] = {(uint32_t)(i >> 3) | 0x80000000u, (uint32_t)h, (uint32_t)(h >> 32),
                          stream_id};
    uint32_t hi[4], lo[4];
    or_philox4x32_10(hi_ctr, key, hi);
    or_philox4x32_10(lo_ctr, key, lo);
    const int j = i & 7;
    return (block_half(hi, j) << 16) | block_half(lo, j);
}

static void sample_one(int n, int K, const uint64_t* C, uint64_t seed, uint32_t stream_id,
                       uint64_t h, uint8_t* x) {
    for (int i = 0; i < n; ++i) {
        uint64_t u = draw_word(seed, stream_id, h, i);
        int state = 0;
        for (int s = 1; s < K; ++s)
            if (u >= C[(size_t)i * (K - 1) + (s - 1)]) state += 1;
        x[i] = (uint8_t)state;
    }
}

/* States of samples first..first+N-1, row-major [N][n]. */
void or_sample(int n, int K, const uint64_t* C, uint64_t seed, uint32_t stream_id,
               uint64_t first, int64_t N, uint8_t* x) {
#pragma omp parallel for schedule(static)
    for (int64_t h = 0; h < N; ++h)
        sample_one(n, K, C, seed, stream_id, first + (uint64_t)h, x + (size_t)h * n);
}

/* States of the samples whose global indices are listed in idx[0..m-1]. */
void or_sample_at(int n, int K, const uint64_t* C, uint64_t seed, uint32_t stream_id,
                  const uint64_t* idx, int64_t m, uint8_t* x) {
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; ++j)
        sample_one(n, K, C, seed, stream_id, idx[j], x + (size_t)j * n);
}

/* ------------------------------------------------------------------------- */
/* Reference-state classification (section 3.3.1, Algorithm 1)               */
/* ------------------------------------------------------------------------- */
/* A sample x is dominated by a lower reference state r when x <= r
 * componentwise, and by an upper reference state r when x >= r.  Algorithm 1
 * gives the lower set precedence.  mode 0 (label): bit0 = some lower state
 * dominates x; bit1 = some upper state dominates x, examined only when bit0 is
 * clear (otherwise 0).  mode 1 (count): mL, mU = number of dominating lower
 * and upper states, and both flag bits are exact. */
static int leq_row(const uint8_t* x, const uint8_t* r, int n) {
    for (int i = 0; i < n; ++i)
        if (x[i] > r[i]) return 0;
    return 1;
}

static int geq_row(const uint8_t* x, const uint8_t* r, int n) {
    for (int i = 0; i < n; ++i)
        if (x[i] < r[i]) return 0;
    return 1;
}

void or_classify(int n, const uint8_t* lower, int64_t RL, const uint8_t* upper, int64_t RU,
                 const uint8_t* x, int64_t N, int mode, uint8_t* flags, uint32_t* mL,
                 uint32_t* mU) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t h = 0; h < N; ++h) {
        const uint8_t* xh = x + (size_t)h * n;
        uint32_t cl = 0, cu = 0;
        for (int64_t r = 0; r < RL; ++r) {
            if (leq_row(xh, lower + (size_t)r * n, n)) {
                cl += 1;
                if (mode == 0) break;
            }
        }
        if (mode == 1 || cl == 0) {
            for (int64_t r = 0; r < RU; ++r) {
                if (geq_row(xh, upper + (size_t)r * n, n)) {
                    cu += 1;
                    if (mode == 0) break;
                }
            }
        }
        flags[h] = (uint8_t)((cl > 0 ? 1 : 0) | (cu > 0 ? 2 : 0));
        if (mL) mL[h] = cl;
        if (mU) mU[h] = cu;
    }
}

/* The paper's own encoding (section 3.2) and violation count
 * (section 3.3.2, eq. violation_matrix) for one sample and one reference
 * state, both of n components with M states:
 *   sample   H[i][m] = 1 iff m == x_i                    (one-hot)
 *   lower    R[i][m] = 1 iff m <= r_i                    (down-set)
 *   upper    R[i][m] = 1 iff m >= r_i                    (up-set)
 *   V = sum_{i,m} H[i][m] * (1 - R[i][m]).
 * side 0 = lower, 1 = upper.  enc receives H (n*M entries) when non-NULL,
 * renc receives R. */
int64_t or_paper_violation(int n, int M, const uint8_t* x, const uint8_t* r, int side,
                           uint8_t* enc, uint8_t* renc) {
    int64_t v = 0;
    for (int i = 0; i < n; ++i) {
        for (int m = 0; m < M; ++m) {
            int hv = (m == (int)x[i]) ? 1 : 0;
            int rv = side == 0 ? (m <= (int)r[i] ? 1 : 0) : (m >= (int)r[i] ? 1 : 0);
            if (enc) enc[i * M + m] = (uint8_t)hv;
            if (renc) renc[i * M + m] = (uint8_t)rv;
            v += (int64_t)hv * (int64_t)(1 - rv);
        }
    }
    return v;
}

/* ------------------------------------------------------------------------- */
/* System function: s-t connectivity at a level                               */
/* ------------------------------------------------------------------------- */
/* Components are the undirected edges of a graph; an edge is usable when its
 * state is at least `level`.  Phi = 1 when t is reachable from s over usable
 * edges (the single-OD connectivity of section 4.1; for K > 2 the level gives
 * the coherent bottleneck system S >= level, one target state of the
 * multi-state workflow of section 3.5, a reading: the paper fixes no
 * multi-state s-t function).  Plain queue BFS over an edge
 * list; adjacency is rebuilt on every call. */
int or_phi_st(int n_nodes, int n_edges, const int32_t* eu, const int32_t* ev, int s, int t,
              int level, const uint8_t* x) {
    if (s == t) return 1;
    uint8_t* seen = (uint8_t*)calloc((size_t)n_nodes, 1);
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_nodes);
    int head = 0, tail = 0, found = 0;
    seen[s] = 1;
    queue[tail++] = s;
    while (head < tail && !found) {
        int u = queue[head++];
        for (int e = 0; e < n_edges; ++e) {
            if ((int)x[e] < level) continue;
            int w;
            if (eu[e] == u) w = ev[e];
            else if (ev[e] == u) w = eu[e];
            else continue;
            if (!seen[w]) {
                seen[w] = 1;
                if (w == t) { found = 1; break; }
                queue[tail++] = w;
            }
        }
    }
    free(seen);
    free(queue);
    return found;
}

/* ------------------------------------------------------------------------- */
/* System function: global connectivity (section 4.2) and its levels (4.5)     */
/* ------------------------------------------------------------------------- */
/* Number of nodes reachable from node 0 over the edges with x_e >= 1, edge
 * `skip` left out (skip = -1: none).  Plain queue BFS. */
static int reach_count(int n_nodes, int n_edges, const int32_t* eu, const int32_t* ev,
                       const uint8_t* x, int skip) {
    uint8_t* seen = (uint8_t*)calloc((size_t)n_nodes, 1);
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_nodes);
    int head = 0, tail = 0;
    seen[0] = 1;
    queue[tail++] = 0;
    while (head < tail) {
        int u = queue[head++];
        for (int e = 0; e < n_edges; ++e) {
            if (e == skip || x[e] < 1) continue;
            int w;
            if (eu[e] == u) w = ev[e];
            else if (ev[e] == u) w = eu[e];
            else continue;
            if (!seen[w]) {
                seen[w] = 1;
                queue[tail++] = w;
            }
        }
    }
    free(seen);
    free(queue);
    return tail;
}

/* System state of global connectivity over the working edges (x_e >= 1):
 * 0 when some node is cut off from the rest, 1 when the graph is connected
 * but some single edge failure would disconnect it, 2 when it stays
 * connected after the failure of any one working edge (by Menger's theorem,
 * two edge-disjoint paths between every pair of nodes).  Written as the
 * definition: one BFS, then one BFS per working edge left out. */
int or_state_global(int n_nodes, int n_edges, const int32_t* eu, const int32_t* ev,
                    const uint8_t* x) {
    if (reach_count(n_nodes, n_edges, eu, ev, x, -1) < n_nodes) return 0;
    for (int e = 0; e < n_edges; ++e) {
        if (x[e] < 1) continue;
        if (reach_count(n_nodes, n_edges, eu, ev, x, e) < n_nodes) return 1;
    }
    return 2;
}

/* Phi for the target S >= level: 1 when or_state_global reaches level. */
int or_phi_global(int n_nodes, int n_edges, const int32_t* eu, const int32_t* ev, int level,
                  const uint8_t* x) {
    return or_state_global(n_nodes, n_edges, eu, ev, x) >= level;
}

/* Stage 2 evaluation (section 3.5) for global connectivity: as or_eval. */
int64_t or_eval_global(int n_nodes, int n_edges, const int32_t* eu, const int32_t* ev, int level,
                       const uint8_t* x, const uint8_t* flags, int64_t N, int which,
                       uint8_t* Y) {
    int64_t evaluated = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : evaluated)
    for (int64_t h = 0; h < N; ++h) {
        const uint8_t* xh = x + (size_t)h * n_edges;
        if (which == 0 && (flags[h] & 1)) {
            Y[h] = 0;
        } else if (which == 0 && (flags[h] & 2)) {
            Y[h] = 1;
        } else {
            Y[h] = (uint8_t)or_phi_global(n_nodes, n_edges, eu, ev, level, xh);
            evaluated += 1;
        }
    }
    return evaluated;
}

/* ------------------------------------------------------------------------- */
/* System function: single-OD maximum flow (section 2.2, d-MPs and d-MCs)      */
/* ------------------------------------------------------------------------- */
/* Maximum s-t flow when undirected edge e carries up to x[e] units in either
 * direction (the component state is the capacity).  Edmonds-Karp: repeat a
 * breadth-first search for a shortest path with spare capacity and push its
 * bottleneck along it, until no such path is left.  flow[e] > 0 is flow from
 * eu[e] to ev[e]. */
int or_maxflow_st(int n_nodes, int n_edges, const int32_t* eu, const int32_t* ev, int s, int t,
                  const uint8_t* x) {
    if (s == t) return 1 << 30;
    int* flow = (int*)calloc((size_t)n_edges, sizeof(int));
    int* via = (int*)malloc(sizeof(int) * (size_t)n_nodes);
    int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_nodes);
    int total = 0;
    for (;;) {
        for (int v = 0; v < n_nodes; ++v) via[v] = -1;
        via[s] = n_edges;  /* marks s as reached */
        int head = 0, tail = 0;
        queue[tail++] = s;
        while (head < tail && via[t] < 0) {
            int u = queue[head++];
            for (int e = 0; e < n_edges; ++e) {
                int w, spare;
                if (eu[e] == u) { w = ev[e]; spare = x[e] - flow[e]; }
                else if (ev[e] == u) { w = eu[e]; spare = x[e] + flow[e]; }
                else continue;
                if (spare > 0 && via[w] < 0) {
                    via[w] = e;
                    queue[tail++] = w;
                }
            }
        }
        if (via[t] < 0) break;
        /* bottleneck along the path, then push it */
        int push = 1 << 30;
        for (int w = t; w != s;) {
            int e = via[w];
            int from = (ev[e] == w) ? eu[e] : ev[e];
            int spare = (from == eu[e]) ? x[e] - flow[e] : x[e] + flow[e];
            if (spare < push) push = spare;
            w = from;
        }
        for (int w = t; w != s;) {
            int e = via[w];
            int from = (ev[e] == w) ? eu[e] : ev[e];
            if (from == eu[e]) flow[e] += push; else flow[e] -= push;
            w = from;
        }
        total += push;
    }
    free(flow);
    free(via);
    free(queue);
    return total;
}

/* Stage 2 evaluation of the system function (section 3.5): Y = 0 for a
 * lower-classified sample, 1 for an upper-classified one, Phi(x) for the
 * unclassified ones.  which = 1 evaluates Phi on every sample (plain Monte
 * Carlo).  Returns the number of Phi evaluations. */
int64_t or_eval(int n_nodes, int n_edges, const int32_t* eu, const int32_t* ev, int s, int t,
                int level, const uint8_t* x, const uint8_t* flags, int64_t N, int which,
                uint8_t* Y) {
    int64_t evaluated = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : evaluated)
    for (int64_t h = 0; h < N; ++h) {
        const uint8_t* xh = x + (size_t)h * n_edges;
        if (which == 0 && (flags[h] & 1)) {
            Y[h] = 0;
        } else if (which == 0 && (flags[h] & 2)) {
            Y[h] = 1;
        } else {
            Y[h] = (uint8_t)or_phi_st(n_nodes, n_edges, eu, ev, s, t, level, xh);
            evaluated += 1;
        }
    }
    return evaluated;
}

/* ------------------------------------------------------------------------- */
/* Componentwise boundary search (section 3.4, fig. x1x2_find_ref)            */
/* ------------------------------------------------------------------------- */
/* above(x) = 1 when the system state at x reaches the target (S >= level). */
typedef int (*or_above_fn)(const uint8_t* x, const void* user);

/* One search, in place on x.  When x is below the target (a failure sample),
 * the components are visited in index order; each is raised one state at a
 * time while it is below K-1, and a raise that reaches the target is undone,
 * which ends the visit of that component.  When x reaches the target (a
 * survival sample) the search is the mirror image: lowering towards 0, and a
 * lowering that leaves the target is undone.  The result is a maximal failure
 * state (returns 0, a lower reference state) or a minimal survival state
 * (returns 1, an upper reference state).  *evals counts calls of above(),
 * including the first one on the sample itself. */
static int boundary_search(int n, int K, uint8_t* x, or_above_fn above, const void* user,
                           int64_t* evals) {
    int start = above(x, user);
    int64_t calls = 1;
    for (int i = 0; i < n; ++i) {
        if (!start) {
            while (x[i] < K - 1) {
                x[i] += 1;
                calls += 1;
                if (above(x, user)) {
                    x[i] -= 1;
                    break;
                }
            }
        } else {
            while (x[i] > 0) {
                x[i] -= 1;
                calls += 1;
                if (!above(x, user)) {
                    x[i] += 1;
                    break;
                }
            }
        }
    }
    if (evals) *evals += calls;
    return start;
}

struct table_user {
    int n, K, level;
    const uint8_t* table;
};

static int above_table(const uint8_t* x, const void* user) {
    const struct table_user* u = (const struct table_user*)user;
    uint64_t idx = 0;
    for (int i = u->n - 1; i >= 0; --i) idx = idx * (uint64_t)u->K + x[i];
    return u->table[idx] >= u->level;
}

/* Boundary search with the system state given as a table over all K^n states
 * (digit i of the index in base K is x_i, least significant first).  x: [Ns][n]
 * start states; out: [Ns][n] boundary states; side: [Ns] 0 lower / 1 upper.
 * Returns the total number of system-function evaluations. */
int64_t or_boundary_table(int n, int K, const uint8_t* table, int level, const uint8_t* x,
                          int64_t Ns, uint8_t* out, uint8_t* side) {
    struct table_user u = {n, K, level, table};
    int64_t evals = 0;
    for (int64_t h = 0; h < Ns; ++h) {
        memcpy(out + (size_t)h * n, x + (size_t)h * n, (size_t)n);
        side[h] = (uint8_t)boundary_search(n, K, out + (size_t)h * n, above_table, &u, &evals);
    }
    return evals;
}

struct st_user {
    int n_nodes, n_edges, s, t, level;
    const int32_t *eu, *ev;
};

static int above_st(const uint8_t* x, const void* user) {
    const struct st_user* u = (const struct st_user*)user;
    return or_phi_st(u->n_nodes, u->n_edges, u->eu, u->ev, u->s, u->t, u->level, x);
}

/* Boundary search for s-t connectivity at `level` (components = edges). */
int64_t or_boundary_st(int n_nodes, int n_edges, const int32_t* eu, const int32_t* ev, int s,
                       int t, int level, int K, const uint8_t* x, int64_t Ns, uint8_t* out,
                       uint8_t* side) {
    struct st_user u = {n_nodes, n_edges, s, t, level, eu, ev};
    int64_t evals = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : evals)
    for (int64_t h = 0; h < Ns; ++h) {
        int64_t e = 0;
        memcpy(out + (size_t)h * n_edges, x + (size_t)h * n_edges, (size_t)n_edges);
        side[h] = (uint8_t)boundary_search(n_edges, K, out + (size_t)h * n_edges, above_st, &u, &e);
        evals += e;
    }
    return evals;
}

struct global_user {
    int n_nodes, n_edges, level;
    const int32_t *eu, *ev;
};

static int above_global(const uint8_t* x, const void* user) {
    const struct global_user* u = (const struct global_user*)user;
    return or_phi_global(u->n_nodes, u->n_edges, u->eu, u->ev, u->level, x);
}

struct flow_user {
    int n_nodes, n_edges, s, t, demand;
    const int32_t *eu, *ev;
};

static int above_flow(const uint8_t* x, const void* user) {
    const struct flow_user* u = (const struct flow_user*)user;
    return or_maxflow_st(u->n_nodes, u->n_edges, u->eu, u->ev, u->s, u->t, x) >= u->demand;
}

/* Boundary search for the target max flow >= demand: the results are
 * d-minimal path vectors (upper) and d-minimal cut vectors (lower). */
int64_t or_boundary_flow(int n_nodes, int n_edges, const int32_t* eu, const int32_t* ev, int s,
                         int t, int demand, int K, const uint8_t* x, int64_t Ns, uint8_t* out,
                         uint8_t* side) {
    struct flow_user u = {n_nodes, n_edges, s, t, demand, eu, ev};
    int64_t evals = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : evals)
    for (int64_t h = 0; h < Ns; ++h) {
        int64_t e = 0;
        memcpy(out + (size_t)h * n_edges, x + (size_t)h * n_edges, (size_t)n_edges);
        side[h] = (uint8_t)boundary_search(n_edges, K, out + (size_t)h * n_edges, above_flow, &u, &e);
        evals += e;
    }
    return evals;
}

/* Stage 2 evaluation for the max-flow target: as or_eval. */
int64_t or_eval_flow(int n_nodes, int n_edges, const int32_t* eu, const int32_t* ev, int s, int t,
                     int demand, const uint8_t* x, const uint8_t* flags, int64_t N, int which,
                     uint8_t* Y) {
    int64_t evaluated = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : evaluated)
    for (int64_t h = 0; h < N; ++h) {
        const uint8_t* xh = x + (size_t)h * n_edges;
        if (which == 0 && (flags[h] & 1)) {
            Y[h] = 0;
        } else if (which == 0 && (flags[h] & 2)) {
            Y[h] = 1;
        } else {
            Y[h] = (uint8_t)(or_maxflow_st(n_nodes, n_edges, eu, ev, s, t, xh) >= demand);
            evaluated += 1;
        }
    }
    return evaluated;
}

/* Boundary search for global connectivity at `level` (components = edges). */
int64_t or_boundary_global(int n_nodes, int n_edges, const int32_t* eu, const int32_t* ev,
                           int level, int K, const uint8_t* x, int64_t Ns, uint8_t* out,
                           uint8_t* side) {
    struct global_user u = {n_nodes, n_edges, level, eu, ev};
    int64_t evals = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : evals)
    for (int64_t h = 0; h < Ns; ++h) {
        int64_t e = 0;
        memcpy(out + (size_t)h * n_edges, x + (size_t)h * n_edges, (size_t)n_edges);
        side[h] = (uint8_t)boundary_search(n_edges, K, out + (size_t)h * n_edges, above_global,
                                           &u, &e);
        evals += e;
    }
    return evals;
}

/* ------------------------------------------------------------------------- */
/* Estimators (section 3.3.1)                                                 */
/* ------------------------------------------------------------------------- */
/* counts: [0] n_L = #{lower}, [1] n_U = #{upper and not lower},
 * [2] n_u = #{neither}, [3] n_both, [4] n_u_up = #{neither and Y = 1},
 * [5] N.  Y may be NULL (then n_u_up = 0). */
void or_counts(const uint8_t* flags, const uint8_t* Y, int64_t N, uint64_t counts[6]) {
    uint64_t nL = 0, nU = 0, nu = 0, nb = 0, nuu = 0;
    for (int64_t h = 0; h < N; ++h) {
        int lo = flags[h] & 1, up = (flags[h] >> 1) & 1;
        if (lo) nL += 1;
        else if (up) nU += 1;
        else {
            nu += 1;
            if (Y && Y[h]) nuu += 1;
        }
        if (lo && up) nb += 1;
    }
    counts[0] = nL; counts[1] = nU; counts[2] = nu; counts[3] = nb; counts[4] = nuu;
    counts[5] = (uint64_t)N;
}

/* est: [0] p_L = n_L/N, [1] p_U = n_U/N, [2] p_u = n_u/N,
 * [3] P = (n_U + n_u_up)/N  (estimate of P(S >= m'+1)),
 * [4] standard error sqrt(P(1-P)/N),
 * [5] coefficient of variation sqrt((1-P)/(N P)) (section 3.3.1), +inf at P = 0.
 * has_Y = 0 leaves P, se and cov as NaN (bounds only). */
void or_estimate(const uint64_t counts[6], int has_Y, double est[6]) {
    double Nd = (double)counts[5];
    est[0] = (double)counts[0] / Nd;
    est[1] = (double)counts[1] / Nd;
    est[2] = (double)counts[2] / Nd;
    if (!has_Y) {
        est[3] = NAN; est[4] = NAN; est[5] = NAN;
        return;
    }
    double P = (double)(counts[1] + counts[4]) / Nd;
    est[3] = P;
    est[4] = sqrt(P * (1.0 - P) / Nd);
    est[5] = P > 0.0 ? sqrt((1.0 - P) / (Nd * P)) : INFINITY;
}

/* ------------------------------------------------------------------------- */
/* Score-function gradient                                                    */
/* ------------------------------------------------------------------------- */
/* With independent components, P = E[Y] is multilinear in the state
 * probabilities, and its partial derivative with respect to p[i][s] (the
 * other entries held fixed) is E[Y * 1{x_i = s}] / p[i][s].  The estimator
 * counts c[i][s] = #{h : Y_h = 1 and x_{h,i} = s} and returns
 * G[i][s] = c[i][s] / (N p[i][s]) in fp64, and 0 where p[i][s] = 0. */
void or_grad(int n, int K, const double* p, const uint8_t* x, const uint8_t* Y, int64_t N,
             uint64_t* counts, double* G) {
    memset(counts, 0, sizeof(uint64_t) * (size_t)n * K);
    for (int64_t h = 0; h < N; ++h) {
        if (!Y[h]) continue;
        const uint8_t* xh = x + (size_t)h * n;
        for (int i = 0; i < n; ++i) counts[(size_t)i * K + xh[i]] += 1;
    }
    for (int i = 0; i < n; ++i)
        for (int s = 0; s < K; ++s) {
            double pv = p[(size_t)i * K + s];
            G[(size_t)i * K + s] =
                pv > 0.0 ? (double)counts[(size_t)i * K + s] / ((double)N * pv) : 0.0;
        }
}

/* ------------------------------------------------------------------------- */
/* Brute force over all K^n states (section 2.1, exhaustive enumeration)      */
/* ------------------------------------------------------------------------- */
/* State index: x_i is digit i (least significant first) of the index in base K. */
static void index_to_state(uint64_t idx, int n, int K, uint8_t* x) {
    for (int i = 0; i < n; ++i) {
        x[i] = (uint8_t)(idx % (uint64_t)K);
        idx /= (uint64_t)K;
    }
}

static uint64_t state_count(int n, int K) {
    uint64_t total = 1;
    for (int i = 0; i < n; ++i) total *= (uint64_t)K;
    return total;
}

/* Phi over every state for s-t connectivity at `level`. */
void bf_phi_table_st(int n_nodes, int n_edges, const int32_t* eu, const int32_t* ev, int s,
                     int t, int level, int K, uint8_t* table) {
    uint64_t total = state_count(n_edges, K);
#pragma omp parallel
    {
        uint8_t* x = (uint8_t*)malloc((size_t)n_edges);
#pragma omp for schedule(static)
        for (int64_t idx = 0; idx < (int64_t)total; ++idx) {
            index_to_state((uint64_t)idx, n_edges, K, x);
            table[idx] = (uint8_t)or_phi_st(n_nodes, n_edges, eu, ev, s, t, level, x);
        }
        free(x);
    }
}

/* System state of global connectivity over every state (0, 1 or 2; compare
 * with a level for Phi). */
void bf_state_table_global(int n_nodes, int n_edges, const int32_t* eu, const int32_t* ev, int K,
                           uint8_t* table) {
    uint64_t total = state_count(n_edges, K);
#pragma omp parallel
    {
        uint8_t* x = (uint8_t*)malloc((size_t)n_edges);
#pragma omp for schedule(static)
        for (int64_t idx = 0; idx < (int64_t)total; ++idx) {
            index_to_state((uint64_t)idx, n_edges, K, x);
            table[idx] = (uint8_t)or_state_global(n_nodes, n_edges, eu, ev, x);
        }
        free(x);
    }
}

/* Max flow of every one of the K^n states, capped at 255. */
void bf_maxflow_table(int n_nodes, int n_edges, const int32_t* eu, const int32_t* ev, int s,
                      int t, int K, uint8_t* table) {
    uint64_t total = state_count(n_edges, K);
#pragma omp parallel
    {
        uint8_t* x = (uint8_t*)malloc((size_t)n_edges);
#pragma omp for schedule(static)
        for (int64_t idx = 0; idx < (int64_t)total; ++idx) {
            index_to_state((uint64_t)idx, n_edges, K, x);
            int f = or_maxflow_st(n_nodes, n_edges, eu, ev, s, t, x);
            table[idx] = (uint8_t)(f > 255 ? 255 : f);
        }
        free(x);
    }
}

/* Exact P = sum_x Phi(x) prod_i p[i][x_i] and exact partials
 * Gx[i][s] = sum_{x : x_i = s} Phi(x) prod_{j != i} p[j][x_j].
 * Gx may be NULL. */
double bf_exact(int n, int K, const double* p, const uint8_t* table, double* Gx) {
    uint64_t total = state_count(n, K);
    double P = 0.0;
    if (Gx) memset(Gx, 0, sizeof(double) * (size_t)n * K);
    uint8_t* x = (uint8_t*)malloc((size_t)n);
    for (uint64_t idx = 0; idx < total; ++idx) {
        if (!table[idx]) continue;
        index_to_state(idx, n, K, x);
        double prob = 1.0;
        for (int i = 0; i < n; ++i) prob *= p[(size_t)i * K + x[i]];
        P += prob;
        if (Gx) {
            for (int i = 0; i < n; ++i) {
                double rest = 1.0;
                for (int j = 0; j < n; ++j)
                    if (j != i) rest *= p[(size_t)j * K + x[j]];
                Gx[(size_t)i * K + x[i]] += rest;
            }
        }
    }
    free(x);
    return P;
}

/* Reference states of a coherent Phi given as a table, for the target
 * S >= level (section 2.2): upper = minimal states with Phi >= level, lower =
 * maximal states with Phi < level.  By monotonicity a state is minimal
 * (maximal) when every single-step decrement (increment) leaves the set.
 * Writes at most cap rows to each of lower/upper ([cap][n]) and returns the
 * counts.  A count above cap means the buffers were too small. */
void bf_reference_sets(int n, int K, const uint8_t* table, int level, uint8_t* lower,
                       int64_t* n_lower, uint8_t* upper, int64_t* n_upper, int64_t cap) {
    uint64_t total = state_count(n, K);
    uint8_t* x = (uint8_t*)malloc((size_t)n);
    int64_t nl = 0, nu = 0;
    uint64_t stride[64];
    stride[0] = 1;
    for (int i = 1; i < n && i < 64; ++i) stride[i] = stride[i - 1] * (uint64_t)K;
    for (uint64_t idx = 0; idx < total; ++idx) {
        index_to_state(idx, n, K, x);
        int above = table[idx] >= level;
        int extreme = 1;
        for (int i = 0; i < n && extreme; ++i) {
            if (above && x[i] > 0) {
                if (table[idx - stride[i]] >= level) extreme = 0;
            } else if (!above && x[i] < K - 1) {
                if (table[idx + stride[i]] < level) extreme = 0;
            }
        }
        if (!extreme) continue;
        if (above) {
            if (nu < cap) memcpy(upper + (size_t)nu * n, x, (size_t)n);
            nu += 1;
        } else {
            if (nl < cap) memcpy(lower + (size_t)nl * n, x, (size_t)n);
            nl += 1;
        }
    }
    free(x);
    *n_lower = nl;
    *n_upper = nu;
}

/* Probability of one full state under independent components:
 * prod_i p[i][x_i] (section 2.2 worked example). */
double or_state_prob(int n, int K, const double* p, const uint8_t* x) {
    double prob = 1.0;
    for (int i = 0; i < n; ++i) prob *= p[(size_t)i * K + x[i]];
    return prob;
}
