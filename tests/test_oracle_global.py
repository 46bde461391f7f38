"""Pins of the oracle's global-connectivity system function (section 4.2)
and its three levels (section 4.5): closed forms on cycles, trees and
parallel edges; an independent all-pairs edge-disjoint-path count (unit
capacity max flow, Menger) on small graphs; the matrix-tree theorem for the
number of minimal survival states; and boundary searches that land on
brute-force boundary states."""
import itertools

import numpy as np

import oracle
import workloads as WL
from test_oracle_pins import _bridge, _graph


def _max_edge_disjoint(n_nodes, edges, x, s, t, cap=2):
    """Edge-disjoint s-t paths over working edges by augmenting paths on a
    unit-capacity undirected network, stopped at `cap`."""
    flow = {}
    adj = [[] for _ in range(n_nodes)]
    for e, (u, v) in enumerate(edges):
        if x[e] >= 1:
            adj[u].append((v, e, 0))
            adj[v].append((u, e, 1))
    used = [0] * len(edges)  # +1: u->v, -1: v->u
    paths = 0
    while paths < cap:
        prev = {s: None}
        stack = [s]
        while stack and t not in prev:
            a = stack.pop()
            for b, e, rev in adj[a]:
                d = -1 if rev else 1          # direction a->b on edge e
                if b in prev or used[e] == d:  # already carries flow this way
                    continue
                prev[b] = (a, e, d)
                stack.append(b)
        if t not in prev:
            break
        b = t
        while prev[b] is not None:
            a, e, d = prev[b]
            used[e] = 0 if used[e] == -d else d
            b = a
        paths += 1
    return paths


def _menger_state(n_nodes, edges, x):
    low = 2
    for s, t in itertools.combinations(range(n_nodes), 2):
        low = min(low, _max_edge_disjoint(n_nodes, edges, x, s, t))
        if low == 0:
            break
    return low


def test_state_against_all_pairs_edge_disjoint_paths():
    k4 = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    for x in itertools.product([0, 1], repeat=6):
        g = _graph(4, k4, 0, 3)
        assert oracle.state_global(g, np.array(x, np.uint8)) == _menger_state(4, k4, x)
    b = _bridge()
    edges = list(zip(b["edge_u"].tolist(), b["edge_v"].tolist()))
    for x in itertools.product([0, 1], repeat=5):
        assert oracle.state_global(b, np.array(x, np.uint8)) == _menger_state(4, edges, x)
    c = WL.configs.tiny(N=10)
    g = c["graph"]
    edges = list(zip(g["edge_u"].tolist(), g["edge_v"].tolist()))
    rng = np.random.default_rng(41)
    for _ in range(150):
        x = (rng.random(len(edges)) < rng.uniform(0.7, 1.0)).astype(np.uint8)
        assert oracle.state_global(g, x) == _menger_state(g["n_nodes"], edges, x)


def test_closed_forms_cycle_tree_parallel():
    """Cycle: S = 2 with no failure, 1 with one, 0 with more.  Path (a tree):
    S = 1 when every edge works, else 0.  n parallel edges: S = min(#working,
    2).  P(S >= 1) and P(S >= 2) by enumeration match the closed forms."""
    n = 7
    rng = np.random.default_rng(42)
    p = rng.uniform(0.6, 0.97, n)
    cycle = _graph(n, [(i, (i + 1) % n) for i in range(n)], 0, 1)
    path = _graph(n + 1, [(i, i + 1) for i in range(n)], 0, n)
    par = _graph(2, [(0, 1)] * n, 0, 1)
    all_work = np.prod(p)
    one_fails = sum((1 - p[i]) * np.prod(np.delete(p, i)) for i in range(n))
    none_work = np.prod(1 - p)
    for g, want1, want2 in [(cycle, all_work + one_fails, all_work),
                            (path, all_work, 0.0),
                            (par, 1 - none_work, 1 - none_work - sum(
                                p[i] * np.prod(1 - np.delete(p, i)) for i in range(n)))]:
        table = oracle.state_table_global(g)
        P1, _ = oracle.exact(oracle.state_probs_binary(p), (table >= 1).astype(np.uint8),
                             want_grad=False)
        P2, _ = oracle.exact(oracle.state_probs_binary(p), (table >= 2).astype(np.uint8),
                             want_grad=False)
        assert abs(P1 - want1) < 1e-14 and abs(P2 - want2) < 1e-14


def test_minimal_survival_states_are_spanning_trees():
    """Level 1: the minimal working edge sets that connect every node are the
    spanning trees, counted by the matrix-tree theorem (any cofactor of the
    graph Laplacian)."""
    c = WL.configs.tiny(N=10)
    g = c["graph"]
    n = c["n"]
    table = oracle.state_table_global(g)
    lo, up = oracle.reference_sets(table, n, 2, level=1)
    L = np.zeros((g["n_nodes"], g["n_nodes"]))
    for u, v in zip(g["edge_u"], g["edge_v"]):
        L[u, u] += 1
        L[v, v] += 1
        L[u, v] -= 1
        L[v, u] -= 1
    trees = round(np.linalg.det(L[1:, 1:]))
    assert len(up) == trees
    assert np.all(up.sum(axis=1) == g["n_nodes"] - 1)


def test_boundary_search_global_lands_on_boundary_states():
    c = WL.configs.tiny(N=10)
    g, n = c["graph"], c["n"]
    table = oracle.state_table_global(g)
    rng = np.random.default_rng(43)
    x = (rng.random((150, n)) < rng.uniform(0.6, 1.0, (150, 1))).astype(np.uint8)
    for level in (1, 2):
        lo, up = oracle.reference_sets(table, n, 2, level=level)
        lo_set, up_set = set(map(bytes, lo)), set(map(bytes, up))
        out, side, _ = oracle.boundary_global(g, x, level=level)
        out_t, side_t, _ = oracle.boundary_table(table, n, 2, x, level=level)
        np.testing.assert_array_equal(out, out_t)
        np.testing.assert_array_equal(side, side_t)
        for h in range(x.shape[0]):
            assert side[h] == (oracle.state_global(g, x[h]) >= level)
            assert bytes(out[h]) in (up_set if side[h] else lo_set)


def test_eval_unknown_global_with_complete_refs():
    """Stage-2 evaluation with half of the reference sets of each level: the
    flagged samples take their flag's value, the rest are evaluated, and
    every Y equals the system state test (invariant I1 for this system)."""
    # 3 x 4 grid: 12 nodes, 17 edges, two-edge-connected when intact.
    edges = [(r * 4 + c, r * 4 + c + 1) for r in range(3) for c in range(3)]
    edges += [(r * 4 + c, (r + 1) * 4 + c) for r in range(2) for c in range(4)]
    g = _graph(12, edges, 0, 11)
    n = len(edges)
    table = oracle.state_table_global(g)
    assert set(np.unique(table).tolist()) == {0, 1, 2}
    p = WL.configs.binary_model(np.random.default_rng(44).uniform(0.85, 0.99, n))
    x = oracle.sample(p, 7, 0, 0, 4000)
    idx = (x.astype(np.uint64) << np.arange(n, dtype=np.uint64)).sum(axis=1)
    for level in (1, 2):
        lo, up = oracle.reference_sets(table, n, 2, level=level)
        flags, _, _ = oracle.classify(lo[: len(lo) // 2], up[: len(up) // 2], x, mode=0)
        Y, nev = oracle.eval_unknown_global(g, x, flags, level=level)
        np.testing.assert_array_equal(Y, (table[idx] >= level).astype(np.uint8))
        assert nev == int(((flags & 3) == 0).sum())
        assert 0 < nev < x.shape[0]
