"""Random geometric graphs in the unit square (the paper's test networks,
section 2.4 "Limitations of decomposition-based approaches", exist only as
figures, so seeded graphs of the same node and edge counts stand in)."""
import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components, shortest_path


def _connected(n_nodes, eu, ev):
    adj = csr_matrix((np.ones(eu.size), (eu, ev)), shape=(n_nodes, n_nodes))
    ncomp, _ = connected_components(adj, directed=False)
    return ncomp == 1


def rgg(n_nodes: int, n_edges: int, seed: int, max_tries: int = 1000, spanning: bool = False):
    """Connected random geometric graph with exactly n_edges edges.

    Nodes are uniform in the unit square (PCG64 seeded with `seed`); the edges
    are the n_edges closest node pairs, ties broken by (distance, i, j).  A
    disconnected draw is redrawn with seed+1, seed+2, ...  With spanning=True
    (for sizes where the closest pairs are rarely connected) the edges are
    instead the Euclidean minimum spanning tree plus the closest remaining
    pairs.  Edge e joins edge_u[e] < edge_v[e]; edges are listed in order of
    increasing length."""
    for k in range(max_tries):
        rng = np.random.default_rng(seed + k)
        pos = rng.random((n_nodes, 2))
        iu, ju = np.triu_indices(n_nodes, k=1)
        d = np.hypot(pos[iu, 0] - pos[ju, 0], pos[iu, 1] - pos[ju, 1])
        ranked = np.lexsort((ju, iu, d))
        if spanning:
            # Kruskal over the ranked pairs, then fill with the shortest others.
            parent = np.arange(n_nodes)

            def find(x):
                while parent[x] != x:
                    parent[x] = parent[parent[x]]
                    x = parent[x]
                return x

            tree = []
            for r in ranked:
                a, b = find(iu[r]), find(ju[r])
                if a != b:
                    parent[a] = b
                    tree.append(r)
                    if len(tree) == n_nodes - 1:
                        break
            in_tree = np.zeros(ranked.size, dtype=bool)
            in_tree[tree] = True
            rest = ranked[~in_tree[ranked]][: n_edges - len(tree)]
            chosen = np.concatenate([np.array(tree, dtype=ranked.dtype), rest])
            order = chosen[np.lexsort((ju[chosen], iu[chosen], d[chosen]))]
        else:
            order = ranked[:n_edges]
        eu = iu[order].astype(np.int32)
        ev = ju[order].astype(np.int32)
        if _connected(n_nodes, eu, ev):
            return {"n_nodes": int(n_nodes), "edge_u": eu, "edge_v": ev, "pos": pos,
                    "seed_used": int(seed + k)}
    raise RuntimeError("no connected graph found")


def st_farthest_pair(graph):
    """Source and sink = the Euclidean farthest node pair (lower id first)."""
    pos = graph["pos"]
    n = pos.shape[0]
    iu, ju = np.triu_indices(n, k=1)
    d = np.hypot(pos[iu, 0] - pos[ju, 0], pos[iu, 1] - pos[ju, 1])
    k = int(np.argmax(d))
    return int(iu[k]), int(ju[k])


def st_degree_rule(graph):
    """Origin = the node of highest degree (lowest id on ties); destination =
    the node with the most BFS hops from it (ties: larger Euclidean distance,
    then lowest id).  This is the rule the paper states for its two graphs."""
    n = graph["n_nodes"]
    eu, ev = graph["edge_u"], graph["edge_v"]
    deg = np.bincount(np.concatenate([eu, ev]), minlength=n)
    s = int(np.argmax(deg))
    adj = csr_matrix((np.ones(eu.size), (eu, ev)), shape=(n, n))
    hops = shortest_path(adj, directed=False, unweighted=True, indices=s)
    pos = graph["pos"]
    dist = np.hypot(pos[:, 0] - pos[s, 0], pos[:, 1] - pos[s, 1])
    best = max(range(n), key=lambda v: (hops[v], dist[v], -v))
    return s, int(best)


def with_terminals(graph, s, t):
    g = dict(graph)
    g["source"] = int(s)
    g["sink"] = int(t)
    return g


def edge_midpoints(graph):
    pos = graph["pos"]
    return 0.5 * (pos[graph["edge_u"]] + pos[graph["edge_v"]])


def grid(rows: int, cols: int):
    """rows x cols grid graph (node r*cols + c), edges row-major then
    column-major; two-edge-connected for rows, cols >= 2."""
    eu, ev = [], []
    for r in range(rows):
        for c in range(cols - 1):
            eu.append(r * cols + c)
            ev.append(r * cols + c + 1)
    for r in range(rows - 1):
        for c in range(cols):
            eu.append(r * cols + c)
            ev.append((r + 1) * cols + c)
    return {"n_nodes": rows * cols, "edge_u": np.array(eu, dtype=np.int32),
            "edge_v": np.array(ev, dtype=np.int32), "source": 0, "sink": rows * cols - 1}
