"""Hypothesis strategies for random coherent systems: s-t connectivity of a
random multigraph (parallel edges allowed, no self-loops) at a level of a
K-state model, small enough for its system function to be tabulated over all
K^n states.  Input generation only: no arithmetic of the method."""
import numpy as np
from hypothesis import strategies as st


def graph_dict(n_nodes, edges, s, t):
    e = np.array(edges, dtype=np.int32).reshape(-1, 2)
    return {"n_nodes": int(n_nodes), "edge_u": e[:, 0].copy(), "edge_v": e[:, 1].copy(),
            "source": int(s), "sink": int(t)}


@st.composite
def st_systems(draw, max_states=1 << 14, min_edges=1):
    """(graph, K, level, p, seed): K in {2, 3}, 3..7 nodes, min_edges..n_max
    edges with K^n <= max_states, source and sink distinct, level in 1..K-1, state
    probabilities of each component in [0.05, 1) normalised to sum 1, and a
    seed for everything else a test draws."""
    K = draw(st.sampled_from((2, 3)))
    n_max = int(np.floor(np.log(max_states) / np.log(K) + 1e-9))
    n_nodes = draw(st.integers(3, 7))
    n_edges = draw(st.integers(min(min_edges, n_max), n_max))
    pair = st.tuples(st.integers(0, n_nodes - 1), st.integers(0, n_nodes - 1)).filter(
        lambda e: e[0] != e[1])
    edges = draw(st.lists(pair, min_size=n_edges, max_size=n_edges))
    s = draw(st.integers(0, n_nodes - 1))
    t = draw(st.integers(0, n_nodes - 2))
    t = t + 1 if t >= s else t
    level = draw(st.integers(1, K - 1))
    seed = draw(st.integers(0, 2**31 - 1))
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.05, 1.0, (n_edges, K))
    p /= p.sum(axis=1, keepdims=True)
    return graph_dict(n_nodes, edges, s, t), K, level, np.ascontiguousarray(p), seed


def all_states(n, K):
    """Every state of n components with K states, row idx = sum x_i K^i."""
    idx = np.arange(K ** n, dtype=np.int64)
    return np.stack([(idx // K ** i) % K for i in range(n)], axis=1).astype(np.uint8)
