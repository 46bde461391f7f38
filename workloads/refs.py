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


def _csr_parts(graph):
    eu, ev = graph["edge_u"], graph["edge_v"]
    return np.concatenate([eu, ev]), np.concatenate([ev, eu])


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


def sample_paths(graph, p_edge, count, seed, s=None, t=None, vias_per_draw=64, max_draws=None):
    """Distinct probable s-t paths.  Each draw perturbs the weights -log(p_e)
    by independent Exp(1) factors (PCG64, `seed`), builds the shortest-path
    trees of s and t, and joins them through random via nodes; loop erasure
    makes every joined walk a simple path, i.e. a minimal path set."""
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
    rows, cols = _csr_parts(graph)
    found, seen = [], set()
    max_draws = max_draws or (20 * count) // vias_per_draw + 100
    draws = 0
    while len(found) < count and draws < max_draws:
        draws += 1
        w = base * rng.exponential(1.0, E) + 1e-9
        mat = csr_matrix((np.concatenate([w, w]), (rows, cols)), shape=(n, n))
        _, pred = dijkstra(mat, directed=True, indices=[s, t], return_predecessors=True)
        ps, pt = pred[0], pred[1]
        for v in rng.permutation(n)[:vias_per_draw]:
            v = int(v)
            if v != s and ps[v] < 0:
                continue
            # s -> v along the tree of s, then v -> t along the tree of t
            a = [v]
            while a[-1] != s:
                a.append(int(ps[a[-1]]))
            a.reverse()
            b = v
            seq = list(a)
            while b != t:
                b = int(pt[b])
                seq.append(b)
            # loop erasure
            pos, walk = {}, []
            for node in seq:
                if node in pos:
                    k = pos[node]
                    for dropped in walk[k + 1:]:
                        del pos[dropped]
                    walk = walk[:k + 1]
                else:
                    pos[node] = len(walk)
                    walk.append(node)
            key = tuple(sorted(eid[(walk[i], walk[i + 1])] for i in range(len(walk) - 1)))
            if key not in seen:
                seen.add(key)
                found.append(key)
                if len(found) >= count:
                    break
    return found


def sample_cuts(graph, count, seed, s=None, t=None, max_draws=None):
    """Distinct minimal s-t cuts.  Each draw grows a ball around one terminal
    (alternately the sink and the source) in the order of a shortest-path
    tree under Exp(1) edge weights (PCG64, `seed`).  For every ball B not
    holding the other terminal, that terminal's component in V minus B is one
    side and its complement the other; both are connected, so the crossing
    edges form a minimal cut.  Components are tracked with a union-find that
    adds nodes farthest first."""
    s = graph["source"] if s is None else s
    t = graph["sink"] if t is None else t
    n = graph["n_nodes"]
    eu, ev = graph["edge_u"], graph["edge_v"]
    E = eu.size
    adj = [[] for _ in range(n)]
    for a, b in zip(eu.tolist(), ev.tolist()):
        adj[a].append(b)
        adj[b].append(a)
    rng = np.random.default_rng(seed)
    rows, cols = _csr_parts(graph)
    found, seen = [], set()
    max_draws = max_draws or 40 * count // max(1, n // 4) + 200
    draws = 0
    while len(found) < count and draws < max_draws:
        draws += 1
        center, other = (t, s) if draws % 2 else (s, t)
        w = rng.exponential(1.0, E) + 1e-9
        mat = csr_matrix((np.concatenate([w, w]), (rows, cols)), shape=(n, n))
        dist = dijkstra(mat, directed=True, indices=center)
        order = np.argsort(dist, kind="stable").tolist()
        kmax = order.index(other)  # the ball may hold order[:k] for k <= kmax
        # union-find over the complement, adding nodes farthest-first
        parent = list(range(n))
        members = {}

        def find(x):
            while parent[x] != x:
                parent[x] = parent[parent[x]]
                x = parent[x]
            return x

        active = np.zeros(n, dtype=bool)
        in_side = np.zeros(n, dtype=bool)
        last_size = -1
        for k in range(n - 1, 0, -1):
            node = order[k]
            active[node] = True
            members[node] = [node]
            for nb in adj[node]:
                if active[nb]:
                    ra, rb = find(node), find(nb)
                    if ra != rb:
                        if len(members[ra]) < len(members[rb]):
                            ra, rb = rb, ra
                        parent[rb] = ra
                        members[ra].extend(members.pop(rb))
            if k > kmax:
                continue
            side = members[find(other)]
            if len(side) == last_size:  # the side only grows: same size, same set
                continue
            last_size = len(side)
            in_side[:] = False
            in_side[side] = True
            key = tuple(np.nonzero(in_side[eu] != in_side[ev])[0].tolist())
            if key and key not in seen:
                seen.add(key)
                found.append(key)
                if len(found) >= count:
                    break
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
