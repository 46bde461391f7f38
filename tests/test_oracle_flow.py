"""Pins of the oracle's single-OD maximum flow with multi-state edge
capacities (section 2.2: reference states as d-minimal paths and cuts): the
max-flow min-cut theorem against brute force over every s-t node cut,
series and parallel closed forms, and boundary searches that land on
brute-force boundary states."""
import itertools

import numpy as np

import oracle
import workloads as WL
from test_oracle_pins import _bridge, _graph


def _min_cut(graph, x):
    """Minimum over node sets T (s in T, t not) of the capacity leaving T."""
    n = graph["n_nodes"]
    s, t = graph["source"], graph["sink"]
    others = [v for v in range(n) if v not in (s, t)]
    eu, ev = graph["edge_u"], graph["edge_v"]
    best = None
    for mask in range(1 << len(others)):
        side = np.zeros(n, dtype=bool)
        side[s] = True
        for k, v in enumerate(others):
            side[v] = bool(mask >> k & 1)
        cap = int(np.asarray(x, dtype=np.int64)[side[eu] != side[ev]].sum())
        best = cap if best is None else min(best, cap)
    return best


def test_max_flow_equals_min_cut():
    rng = np.random.default_rng(71)
    b = _bridge()
    for x in itertools.product(range(4), repeat=5):
        assert oracle.maxflow_st(b, np.array(x, np.uint8)) == _min_cut(b, x)
    c = WL.configs.tiny(N=10)
    g = c["graph"]
    for _ in range(60):
        x = rng.integers(0, 5, size=c["n"]).astype(np.uint8)
        assert oracle.maxflow_st(g, x) == _min_cut(g, x)
    grid = WL.graphs.grid(3, 3)
    for _ in range(60):
        x = rng.integers(0, 4, size=grid["edge_u"].size).astype(np.uint8)
        assert oracle.maxflow_st(grid, x) == _min_cut(grid, x)


def test_series_parallel_closed_forms():
    rng = np.random.default_rng(72)
    n = 6
    series = _graph(n + 1, [(i, i + 1) for i in range(n)], 0, n)
    par = _graph(2, [(0, 1)] * n, 0, 1)
    for _ in range(50):
        x = rng.integers(0, 7, size=n).astype(np.uint8)
        assert oracle.maxflow_st(series, x) == int(x.min())
        assert oracle.maxflow_st(par, x) == int(x.sum())


def test_boundary_flow_lands_on_d_minimal_vectors():
    """Bridge network, capacities 0..3: from every one of the 4^5 states, the
    search for max flow >= d (d = 1..4) ends in a brute-force d-minimal path
    vector (upper) or d-minimal cut vector (lower) on its start's side, and
    the table and max-flow routes agree."""
    b = _bridge()
    K = 4
    table = oracle.maxflow_table(b, K)
    idx = np.arange(K ** 5)
    states = np.stack([(idx // K ** i) % K for i in range(5)], axis=1).astype(np.uint8)
    for d in (1, 2, 3, 4):
        lo, up = oracle.reference_sets(table, 5, K, level=d)
        lo_set, up_set = set(map(bytes, lo)), set(map(bytes, up))
        out, side, _ = oracle.boundary_flow(b, states, K, d)
        out_t, side_t, _ = oracle.boundary_table(table, 5, K, states, level=d)
        np.testing.assert_array_equal(out, out_t)
        np.testing.assert_array_equal(side, side_t)
        assert np.array_equal(side, (table >= d).astype(np.uint8))
        for h in range(states.shape[0]):
            assert bytes(out[h]) in (up_set if side[h] else lo_set)
        Y, nev = oracle.eval_unknown_flow(b, states, None, which=1, demand=d)
        np.testing.assert_array_equal(Y, (table >= d).astype(np.uint8))
