"""Reference-state rows for s-t connectivity built from the graph structure.

For a binary s-t connectivity system the paper notes (section 2.2) that the
upper reference states are the link (path) sets and the lower reference
states are the cut sets.  Minimal path sets are exactly the edge sets of
simple s-t paths, and minimal cut sets are exactly the edge sets delta(T)
between a connected node set T (holding t, not s) and its connected
complement.  This module builds such sets from the graph alone - enumerating
all of them on tiny graphs, and sampling probable ones on larger graphs - and
turns them into uint8 state rows:

  upper row for level k:  state k on the path's edges, 0 elsewhere
  lower row for level k:  state k-1 on the cut's edges, K-1 elsewhere

which are the minimal states with S >= k and the maximal states with S < k of
the bottleneck system "t reachable from s over edges with state >= k".
"""
import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import dijkstra


def _adjacency(graph):
    n = graph["n_nodes"]
    adj = [[] for _ in range(n)]
    for e, (u, v) in enumerate(zip(graph["edge_u"].tolist(), graph["edge_v"].tolist())):
        adj[u].append((v, e))
        adj[v].append((u, e))
    return adj


def all_min_paths(graph, s=None, t=None):
    """All simple s-t paths, as sorted tuples of edge ids (depth-first order)."""
    s = graph["source"] if s is None else s
    t = graph["sink"] if t is None else t
    adj = _adjacency(graph)
    out = []
    on_path = [False] * graph["n_nodes"]
    edges = []

    def walk(u):
        if u == t:
            out.append(tuple(sorted(edges)))
            return
        on_path[u] = True
        for v, e in adj[u]:
            if not on_path[v]:
                edges.append(e)
                walk(v)
                edges.pop()
        on_path[u] = False

    walk(s)
    return sorted(set(out))


def _reach(adj, start, blocked):
    seen = {start}
    stack = [start]
    while stack:
        u = stack.pop()
        for v, _ in adj[u]:
            if v not in seen and not blocked[v]:
                seen.add(v)
                stack.append(v)
    return seen


def all_min_cuts(graph, s=None, t=None):
    """All minimal s-t cut sets, as sorted tuples of edge ids.

    Enumerates every node set T with t in T, s not in T, both T and its
    complement connected; the cut is the set of edges crossing (T, V\\T)."""
    s = graph["source"] if s is None else s
    t = graph["sink"] if t is None else t
    n = graph["n_nodes"]
    adj = _adjacency(graph)
    others = [v for v in range(n) if v not in (s, t)]
    eu, ev = graph["edge_u"], graph["edge_v"]
    out = set()
    for mask in range(1 << len(others)):
        in_t = np.zeros(n, dtype=bool)
        in_t[t] = True
        for k, v in enumerate(others):
            if mask >> k & 1:
                in_t[v] = True
        if len(_reach(adj, t, ~in_t)) != int(in_t.sum()):
            continue
        if len(_reach(adj, s, in_t)) != n - int(in_t.sum()):
            continue
        cut = np.nonzero(in_t[eu] != in_t[ev])[0]
        out.add(tuple(int(e) for e in cut))
    return sorted(out)


def sample_paths(graph, p_edge, count, seed, s=None, t=None, max_calls=None):
    """Distinct probable s-t paths: shortest paths under the weights
    -log(p_e) times independent Exp(1) noise (PCG64, `seed`)."""
    s = graph["source"] if s is None else s
    t = graph["sink"] if t is None else t
    n = graph["n_nodes"]
    eu, ev = graph["edge_u"], graph["edge_v"]
    E = eu.size
    rng = np.random.default_rng(seed)
    base = -np.log(np.clip(np.asarray(p_edge, dtype=np.float64), 1e-12, 1.0)) + 1e-3
    eid = {}
    for e in range(E):
        eid[(int(eu[e]), int(ev[e]))] = e
        eid[(int(ev[e]), int(eu[e]))] = e
    rows = np.concatenate([eu, ev])
    cols = np.concatenate([ev, eu])
    found = []
    seen = set()
    max_calls = max_calls or 20 * count + 100
    calls = 0
    while len(found) < count and calls < max_calls:
        calls += 1
        w = base * rng.exponential(1.0, E) + 1e-9
        mat = csr_matrix((np.concatenate([w, w]), (rows, cols)), shape=(n, n))
        _, pred = dijkstra(mat, directed=True, indices=s, return_predecessors=True)
        if pred[t] < 0:
            continue
        path = []
        v = t
        while v != s:
            u = int(pred[v])
            path.append(eid[(u, v)])
            v = u
        key = tuple(sorted(path))
        if key not in seen:
            seen.add(key)
            found.append(key)
    return found


def sample_cuts(graph, count, seed, s=None, t=None, mean_size=4.0, max_attempts=None):
    """Distinct minimal s-t cuts from random connected growth.

    A node set T is grown from t (or, alternately, from s) by a geometric
    number of random neighbour additions; the side holding the other terminal
    is then taken as the component of the rest that contains it, which makes
    both sides connected and so the crossing edges a minimal cut."""
    s = graph["source"] if s is None else s
    t = graph["sink"] if t is None else t
    n = graph["n_nodes"]
    adj = _adjacency(graph)
    eu, ev = graph["edge_u"], graph["edge_v"]
    rng = np.random.default_rng(seed)
    found = []
    seen = set()
    max_attempts = max_attempts or 30 * count + 100
    attempts = 0
    while len(found) < count and attempts < max_attempts:
        attempts += 1
        grow_from, other = (t, s) if attempts % 2 else (s, t)
        size = int(rng.geometric(1.0 / mean_size))
        grown = np.zeros(n, dtype=bool)
        grown[grow_from] = True
        members = [grow_from]
        for _ in range(size - 1):
            cand = [v for u in members for v, _ in adj[u] if not grown[v] and v != other]
            if not cand:
                break
            v = cand[int(rng.integers(len(cand)))]
            grown[v] = True
            members.append(v)
        other_side = _reach(adj, other, grown)
        side = np.ones(n, dtype=bool)
        side[list(other_side)] = False
        cut = np.nonzero(side[eu] != side[ev])[0]
        key = tuple(int(e) for e in cut)
        if key and key not in seen:
            seen.add(key)
            found.append(key)
    return found


def paths_to_upper(paths, n, K=2, level=1):
    rows = np.zeros((len(paths), n), dtype=np.uint8)
    for r, path in enumerate(paths):
        rows[r, list(path)] = level
    return rows


def cuts_to_lower(cuts, n, K=2, level=1):
    rows = np.full((len(cuts), n), K - 1, dtype=np.uint8)
    for r, cut in enumerate(cuts):
        rows[r, list(cut)] = level - 1
    return rows


def bernoulli_rows(R, n, rho, seed):
    """R rows of n independent Bernoulli(rho) 0/1 states."""
    rng = np.random.default_rng(seed)
    return (rng.random((R, n)) < rho).astype(np.uint8)
