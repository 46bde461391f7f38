"""The five workloads of the hot path, as seeded synthetic inputs.

Each builder returns a plain dict: the model as an [n][K] fp64 matrix of
component-state probabilities, the Philox key (`seed`) and stream id, the
sample count N, the reference-state rows (uint8, [R][n]) and, for network
workloads, the graph with its source and sink.  Sizes can be scaled down for
tests; the defaults are the full workload sizes.

  tiny     12-node / 20-edge graph, every minimal path and cut, N = 1e5
  graph2   119-node / 295-edge graph (the size of the paper's Graph 2),
           1e4 upper + 1e4 lower rows, N = 1e6
  scaling  n = 295, 1e5 + 1e5 Bernoulli rows, N = 1e6 (kernel only)
  multi    graph2 with three-state edges, bottleneck levels 1 and 2, N = 1e6
  batched  8 graphs of 50..500 nodes x 64 hazard scenarios
"""
import functools

import numpy as np

from . import graphs as G
from . import refs as RF


def binary_model(p_survive):
    p = np.asarray(p_survive, dtype=np.float64)
    return np.ascontiguousarray(np.stack([1.0 - p, p], axis=1))


@functools.lru_cache(maxsize=None)
def _tiny_graph():
    g = G.rgg(12, 20, seed=1)
    s, t = G.st_farthest_pair(g)
    return G.with_terminals(g, s, t)


def tiny(N=100_000):
    """12 nodes, 20 undirected edges, source/sink = Euclidean farthest pair;
    edge survival p ~ U[0.80, 0.99]; complete reference sets."""
    g = _tiny_graph()
    n = g["edge_u"].size
    rng = np.random.default_rng(11)
    p_surv = rng.uniform(0.80, 0.99, n)
    paths = RF.all_min_paths(g)
    cuts = RF.all_min_cuts(g)
    return {
        "name": "tiny", "graph": g, "n": n, "K": 2, "level": 1,
        "p": binary_model(p_surv), "seed": 1, "stream": 0, "N": int(N),
        "upper": RF.paths_to_upper(paths, n), "lower": RF.cuts_to_lower(cuts, n),
    }


@functools.lru_cache(maxsize=None)
def _graph1():
    g = G.rgg(59, 262, seed=1)
    s, t = G.st_degree_rule(g)
    return G.with_terminals(g, s, t)


def global1(N=1_000_000):
    """Global connectivity of a 59-node / 262-edge random geometric graph (the
    size of the paper's Graph 1) with edge failure p ~ U[0.01, 0.20]; the
    reference states are grown by the Stage-1 loop, so none are given."""
    g = _graph1()
    n = g["edge_u"].size
    rng = np.random.default_rng(21)
    return {"name": "global1", "graph": g, "n": n, "K": 2,
            "p": binary_model(1.0 - rng.uniform(0.01, 0.20, n)), "seed": 21, "stream": 0,
            "N": int(N)}


def global2(N=1_000_000):
    """Global connectivity of graph2 (119 nodes / 295 edges) with its edge
    probabilities; reference states grown by the Stage-1 loop."""
    c = graph2(N=N, R_U=10, R_L=10)
    return {"name": "global2", "graph": c["graph"], "n": c["n"], "K": 2, "p": c["p"],
            "seed": 22, "stream": 0, "N": int(N)}


@functools.lru_cache(maxsize=None)
def _graph2():
    g = G.rgg(119, 295, seed=2)
    s, t = G.st_degree_rule(g)
    return G.with_terminals(g, s, t)


@functools.lru_cache(maxsize=None)
def _graph2_refs(R_U, R_L):
    g = _graph2()
    n = g["edge_u"].size
    rng = np.random.default_rng(21)
    p_fail = rng.uniform(0.01, 0.20, n)
    paths = RF.sample_paths(g, 1.0 - p_fail, R_U, seed=22)
    cuts = RF.sample_cuts(g, R_L, seed=23)
    return p_fail, RF.paths_to_upper(paths, n), RF.cuts_to_lower(cuts, n)


def graph2(N=1_000_000, R_U=10_000, R_L=10_000):
    """119 nodes / 295 edges, origin = highest degree, destination = most hops
    away; edge failure probability ~ U[0.01, 0.20]."""
    g = _graph2()
    n = g["edge_u"].size
    p_fail, upper, lower = _graph2_refs(int(R_U), int(R_L))
    return {
        "name": "graph2", "graph": g, "n": n, "K": 2, "level": 1,
        "p": binary_model(1.0 - p_fail), "seed": 2, "stream": 0, "N": int(N),
        "upper": upper, "lower": lower,
    }


def scaling(N=1_000_000, R_U=100_000, R_L=100_000, n=295):
    """Kernel-only scaling: Bernoulli(0.05) upper rows, Bernoulli(0.9) lower
    rows, p ~ U[0.7, 0.99].  The rows are not the reference sets of any
    particular system, so a sample may match on both sides."""
    rng = np.random.default_rng(31)
    p_surv = rng.uniform(0.7, 0.99, n)
    return {
        "name": "scaling", "graph": None, "n": n, "K": 2, "level": 1,
        "p": binary_model(p_surv), "seed": 3, "stream": 0, "N": int(N),
        "upper": RF.bernoulli_rows(int(R_U), n, 0.05, seed=32),
        "lower": RF.bernoulli_rows(int(R_L), n, 0.9, seed=33),
    }


@functools.lru_cache(maxsize=None)
def _multi_refs(R_per_level):
    g = _graph2()
    n = g["edge_u"].size
    rng = np.random.default_rng(41)
    p = rng.dirichlet([8.0, 2.0, 1.0], size=n)[:, ::-1].copy()
    levels = {}
    half = R_per_level // 2
    for k in (1, 2):
        p_ge = p[:, k:].sum(axis=1)
        paths = RF.sample_paths(g, p_ge, half, seed=42 + k)
        cuts = RF.sample_cuts(g, R_per_level - half, seed=44 + k)
        levels[k] = (RF.cuts_to_lower(cuts, n, K=3, level=k),
                     RF.paths_to_upper(paths, n, K=3, level=k))
    return p, levels


def multi(N=1_000_000, R_per_level=50_000):
    """graph2 with edge states {0,1,2}; (p0, p1, p2) = reversed Dirichlet(8,2,1)
    so that most mass sits on the best state; system level S = the largest k
    such that t is reachable from s over edges with state >= k."""
    g = _graph2()
    n = g["edge_u"].size
    p, levels = _multi_refs(int(R_per_level))
    return {
        "name": "multi", "graph": g, "n": n, "K": 3, "p": np.ascontiguousarray(p),
        "seed": 4, "stream": 0, "N": int(N),
        "levels": {k: {"lower": lo, "upper": up} for k, (lo, up) in levels.items()},
    }


BATCH_NODES = (50, 69, 96, 134, 186, 259, 360, 500)
BATCH_EDGES = (120, 172, 240, 335, 465, 647, 900, 1250)
BATCH_REFS = (1_000, 2_100, 4_500, 9_700, 21_000, 44_000, 94_000, 200_000)


@functools.lru_cache(maxsize=None)
def _batch_graph(g_idx):
    g = G.rgg(BATCH_NODES[g_idx], BATCH_EDGES[g_idx], seed=5 + g_idx, spanning=True)
    s, t = G.st_degree_rule(g)
    return G.with_terminals(g, s, t)


def hazard_scenarios(graph, n_scen, seed, beta=1.5, n_fourier=16):
    """Edge failure probabilities of n_scen hazard scenarios.

    Each scenario has an epicentre ~ U[0,1]^2 and an intensity field
    f(z) = exp(-3 |z - epicentre|) + 0.3 * (mean of n_fourier random Fourier
    features); p_fail,e = sigmoid(alpha + beta f(midpoint_e)), with alpha set by
    bisection so that the mean p_fail equals a target ~ U[0.02, 0.15], then
    clipped to [1e-4, 0.5].  Returns [n_scen][E] survival probabilities."""
    rng = np.random.default_rng(seed)
    mid = G.edge_midpoints(graph)
    out = np.zeros((n_scen, mid.shape[0]))
    for sc in range(n_scen):
        epi = rng.random(2)
        freq = rng.normal(0.0, 4.0, (n_fourier, 2))
        phase = rng.uniform(0, 2 * np.pi, n_fourier)
        target = rng.uniform(0.02, 0.15)
        dist = np.hypot(mid[:, 0] - epi[0], mid[:, 1] - epi[1])
        f = np.exp(-3.0 * dist) + 0.3 * np.cos(mid @ freq.T + phase).mean(axis=1)
        lo, hi = -20.0, 20.0
        for _ in range(100):
            a = 0.5 * (lo + hi)
            m = (1.0 / (1.0 + np.exp(-(a + beta * f)))).mean()
            lo, hi = (a, hi) if m < target else (lo, a)
        pf = np.clip(1.0 / (1.0 + np.exp(-(0.5 * (lo + hi) + beta * f))), 1e-4, 0.5)
        out[sc] = 1.0 - pf
    return out


@functools.lru_cache(maxsize=None)
def _batch_refs(g_idx, R):
    g = _batch_graph(g_idx)
    n = g["edge_u"].size
    base = hazard_scenarios(g, 8, seed=500 + g_idx).mean(axis=0)
    half = R // 2
    paths = RF.sample_paths(g, base, half, seed=510 + g_idx)
    cuts = RF.sample_cuts(g, R - half, seed=520 + g_idx)
    return RF.cuts_to_lower(cuts, n), RF.paths_to_upper(paths, n)


def batched(n_scen=64, N=1_000_000, graphs=range(8), ref_scale=1.0):
    """8 graphs of uneven size, each with its own reference sets (shared by
    every scenario, since reference states depend only on the system
    function), times n_scen hazard scenarios: one job per (graph, scenario)."""
    jobs = []
    systems = []
    for g_idx in graphs:
        g = _batch_graph(g_idx)
        n = g["edge_u"].size
        R = max(2, int(round(BATCH_REFS[g_idx] * ref_scale)))
        lower, upper = _batch_refs(g_idx, R)
        systems.append({"graph": g, "n": n, "K": 2, "level": 1, "lower": lower,
                        "upper": upper, "g_idx": g_idx})
        p_all = hazard_scenarios(g, n_scen, seed=600 + g_idx)
        for sc in range(n_scen):
            jobs.append({"system": len(systems) - 1, "p": binary_model(p_all[sc]),
                         "seed": 1000 + 64 * g_idx + sc, "stream": 0, "N": int(N)})
    return {"name": "batched", "systems": systems, "jobs": jobs}
