"""ctypes binding of the plain-C oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the oracle is a slow, obviously correct CPU
implementation of what the RSR Stage-2 hot path computes (arXiv 2604.17066,
sections 2.2, 3.2, 3.3 and 3.5), and of the componentwise boundary search of
Stage 1 (section 3.4).  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it.  It shares no code with the
product package, and it never imports it.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RSR_ORACLE_LIB lets the mutation test load a deliberately broken build.
_LIB_PATH = os.environ.get("RSR_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "or_set_threads": (None, [ctypes.c_int]),
        "or_get_threads": (ctypes.c_int, []),
        "or_philox4x32_10": (None, [_u32p, _u32p, _u32p]),
        "or_thresholds": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _f64p, _u64p]),
        "or_sample": (None, [ctypes.c_int, ctypes.c_int, _u64p, ctypes.c_uint64, ctypes.c_uint32,
                             ctypes.c_uint64, ctypes.c_int64, _u8p]),
        "or_sample_at": (None, [ctypes.c_int, ctypes.c_int, _u64p, ctypes.c_uint64,
                                ctypes.c_uint32, _u64p, ctypes.c_int64, _u8p]),
        "or_classify": (None, [ctypes.c_int, _u8p, ctypes.c_int64, _u8p, ctypes.c_int64, _u8p,
                               ctypes.c_int64, ctypes.c_int, _u8p, _u32p, _u32p]),
        "or_paper_violation": (ctypes.c_int64, [ctypes.c_int, ctypes.c_int, _u8p, _u8p,
                                                ctypes.c_int, _u8p, _u8p]),
        "or_phi_st": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i32p, _i32p, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, _u8p]),
        "or_eval": (ctypes.c_int64, [ctypes.c_int, ctypes.c_int, _i32p, _i32p, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, _u8p, _u8p, ctypes.c_int64,
                                     ctypes.c_int, _u8p]),
        "or_counts": (None, [_u8p, _u8p, ctypes.c_int64, _u64p]),
        "or_estimate": (None, [_u64p, ctypes.c_int, _f64p]),
        "or_grad": (None, [ctypes.c_int, ctypes.c_int, _f64p, _u8p, _u8p, ctypes.c_int64, _u64p,
                           _f64p]),
        "bf_phi_table_st": (None, [ctypes.c_int, ctypes.c_int, _i32p, _i32p, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_int, _u8p]),
        "bf_exact": (ctypes.c_double, [ctypes.c_int, ctypes.c_int, _f64p, _u8p, _f64p]),
        "bf_reference_sets": (None, [ctypes.c_int, ctypes.c_int, _u8p, ctypes.c_int, _u8p, _i64p,
                                     _u8p, _i64p, ctypes.c_int64]),
        "or_state_prob": (ctypes.c_double, [ctypes.c_int, ctypes.c_int, _f64p, _u8p]),
        "or_state_global": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i32p, _i32p, _u8p]),
        "or_phi_global": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i32p, _i32p, ctypes.c_int,
                                         _u8p]),
        "or_eval_global": (ctypes.c_int64, [ctypes.c_int, ctypes.c_int, _i32p, _i32p, ctypes.c_int,
                                            _u8p, _u8p, ctypes.c_int64, ctypes.c_int, _u8p]),
        "or_boundary_global": (ctypes.c_int64, [ctypes.c_int, ctypes.c_int, _i32p, _i32p,
                                                ctypes.c_int, ctypes.c_int, _u8p, ctypes.c_int64,
                                                _u8p, _u8p]),
        "bf_state_table_global": (None, [ctypes.c_int, ctypes.c_int, _i32p, _i32p, ctypes.c_int,
                                         _u8p]),
        "or_maxflow_st": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i32p, _i32p, ctypes.c_int,
                                         ctypes.c_int, _u8p]),
        "or_eval_flow": (ctypes.c_int64, [ctypes.c_int, ctypes.c_int, _i32p, _i32p, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, _u8p, _u8p, ctypes.c_int64,
                                          ctypes.c_int, _u8p]),
        "or_boundary_flow": (ctypes.c_int64, [ctypes.c_int, ctypes.c_int, _i32p, _i32p,
                                              ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_int, _u8p, ctypes.c_int64, _u8p, _u8p]),
        "bf_maxflow_table": (None, [ctypes.c_int, ctypes.c_int, _i32p, _i32p, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, _u8p]),
        "or_boundary_table": (ctypes.c_int64, [ctypes.c_int, ctypes.c_int, _u8p, ctypes.c_int,
                                               _u8p, ctypes.c_int64, _u8p, _u8p]),
        "or_boundary_st": (ctypes.c_int64, [ctypes.c_int, ctypes.c_int, _i32p, _i32p,
                                            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            _u8p, ctypes.c_int64, _u8p, _u8p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def set_threads(t: int) -> None:
    _load().or_set_threads(int(t))


def get_threads() -> int:
    return int(_load().or_get_threads())


def philox4x32_10(ctr, key):
    """One Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().or_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32),
                             _ptr(out, ctypes.c_uint32))
    return out


def state_probs_binary(p_survive):
    """[n] survival probabilities -> [n][2] state probabilities (1 - p, p)."""
    p = _c(p_survive, np.float64)
    return np.ascontiguousarray(np.stack([1.0 - p, p], axis=1))


def thresholds(p):
    """[n][K] state probabilities -> [n][K-1] uint64 inverse-CDF thresholds."""
    p = _c(p, np.float64)
    n, K = p.shape
    C = np.zeros((n, K - 1), dtype=np.uint64)
    rc = _load().or_thresholds(n, K, _ptr(p, ctypes.c_double), _ptr(C, ctypes.c_uint64))
    if rc != 0:
        raise ValueError("bad model shape")
    return C


def sample(p, seed, stream_id, first, N):
    """States [N][n] uint8 of samples first..first+N-1."""
    p = _c(p, np.float64)
    n, K = p.shape
    C = thresholds(p)
    x = np.zeros((N, n), dtype=np.uint8)
    _load().or_sample(n, K, _ptr(C, ctypes.c_uint64), int(seed), int(stream_id), int(first),
                      int(N), _ptr(x, ctypes.c_uint8))
    return x


def sample_at(p, seed, stream_id, indices):
    """States [m][n] uint8 of the samples with the given global indices."""
    p = _c(p, np.float64)
    n, K = p.shape
    C = thresholds(p)
    idx = _c(indices, np.uint64)
    x = np.zeros((idx.size, n), dtype=np.uint8)
    _load().or_sample_at(n, K, _ptr(C, ctypes.c_uint64), int(seed), int(stream_id),
                         _ptr(idx, ctypes.c_uint64), int(idx.size), _ptr(x, ctypes.c_uint8))
    return x


def classify(lower, upper, x, mode=0):
    """Algorithm 1 on uint8 states.  Returns (flags, mL, mU); mL/mU exact in mode 1."""
    x = _c(x, np.uint8)
    N, n = x.shape
    lower = _c(lower, np.uint8).reshape(-1, n)
    upper = _c(upper, np.uint8).reshape(-1, n)
    flags = np.zeros(N, dtype=np.uint8)
    mL = np.zeros(N, dtype=np.uint32)
    mU = np.zeros(N, dtype=np.uint32)
    _load().or_classify(n, _ptr(lower, ctypes.c_uint8), lower.shape[0],
                        _ptr(upper, ctypes.c_uint8), upper.shape[0], _ptr(x, ctypes.c_uint8),
                        N, int(mode), _ptr(flags, ctypes.c_uint8), _ptr(mL, ctypes.c_uint32),
                        _ptr(mU, ctypes.c_uint32))
    return flags, mL, mU


def paper_violation(x, r, M, side):
    """The paper's one-hot / down-set / up-set encoding and violation count.

    Returns (V, H, R) with H and R as [n][M] 0/1 matrices.  side 0 = lower, 1 = upper."""
    x = _c(x, np.uint8)
    r = _c(r, np.uint8)
    n = x.size
    H = np.zeros((n, M), dtype=np.uint8)
    R = np.zeros((n, M), dtype=np.uint8)
    v = _load().or_paper_violation(n, M, _ptr(x, ctypes.c_uint8), _ptr(r, ctypes.c_uint8),
                                   int(side), _ptr(H, ctypes.c_uint8), _ptr(R, ctypes.c_uint8))
    return int(v), H, R


def _graph_args(graph):
    eu = _c(graph["edge_u"], np.int32)
    ev = _c(graph["edge_v"], np.int32)
    return eu, ev


def phi_st(graph, x, level=1):
    eu, ev = _graph_args(graph)
    x = _c(x, np.uint8)
    return int(_load().or_phi_st(int(graph["n_nodes"]), eu.size, _ptr(eu, ctypes.c_int32),
                                 _ptr(ev, ctypes.c_int32), int(graph["source"]),
                                 int(graph["sink"]), int(level), _ptr(x, ctypes.c_uint8)))


def eval_unknown(graph, x, flags, which=0, level=1):
    """Y per sample: lower -> 0, upper -> 1, else Phi(x).  which=1: Phi on every sample."""
    eu, ev = _graph_args(graph)
    x = _c(x, np.uint8)
    N = x.shape[0]
    flags = _c(flags, np.uint8) if flags is not None else np.zeros(N, dtype=np.uint8)
    Y = np.zeros(N, dtype=np.uint8)
    nev = _load().or_eval(int(graph["n_nodes"]), eu.size, _ptr(eu, ctypes.c_int32),
                          _ptr(ev, ctypes.c_int32), int(graph["source"]), int(graph["sink"]),
                          int(level), _ptr(x, ctypes.c_uint8), _ptr(flags, ctypes.c_uint8), N,
                          int(which), _ptr(Y, ctypes.c_uint8))
    return Y, int(nev)


def counts(flags, Y=None):
    flags = _c(flags, np.uint8)
    Yc = _c(Y, np.uint8) if Y is not None else None
    out = np.zeros(6, dtype=np.uint64)
    _load().or_counts(_ptr(flags, ctypes.c_uint8), _ptr(Yc, ctypes.c_uint8), flags.size,
                      _ptr(out, ctypes.c_uint64))
    return out


COUNT_NAMES = ("n_L", "n_U", "n_u", "n_both", "n_u_up", "N")
EST_NAMES = ("p_L", "p_U", "p_u", "P", "se", "cov")


def estimate(cnt, has_Y=True):
    cnt = _c(cnt, np.uint64)
    est = np.zeros(6, dtype=np.float64)
    _load().or_estimate(_ptr(cnt, ctypes.c_uint64), 1 if has_Y else 0,
                        _ptr(est, ctypes.c_double))
    return est


def grad(p, x, Y):
    """Score-function counts c[n][K] and G[n][K] = c / (N p) in fp64."""
    p = _c(p, np.float64)
    n, K = p.shape
    x = _c(x, np.uint8)
    Y = _c(Y, np.uint8)
    N = x.shape[0]
    c = np.zeros((n, K), dtype=np.uint64)
    G = np.zeros((n, K), dtype=np.float64)
    _load().or_grad(n, K, _ptr(p, ctypes.c_double), _ptr(x, ctypes.c_uint8),
                    _ptr(Y, ctypes.c_uint8), N, _ptr(c, ctypes.c_uint64),
                    _ptr(G, ctypes.c_double))
    return c, G


def phi_table_st(graph, K=2, level=1):
    eu, ev = _graph_args(graph)
    n = eu.size
    total = K ** n
    table = np.zeros(total, dtype=np.uint8)
    _load().bf_phi_table_st(int(graph["n_nodes"]), n, _ptr(eu, ctypes.c_int32),
                            _ptr(ev, ctypes.c_int32), int(graph["source"]), int(graph["sink"]),
                            int(level), int(K), _ptr(table, ctypes.c_uint8))
    return table


def exact(p, table, want_grad=True):
    """Exact P and partials by enumeration of all K^n states."""
    p = _c(p, np.float64)
    n, K = p.shape
    table = _c(table, np.uint8)
    G = np.zeros((n, K), dtype=np.float64) if want_grad else None
    P = _load().bf_exact(n, K, _ptr(p, ctypes.c_double), _ptr(table, ctypes.c_uint8),
                         _ptr(G, ctypes.c_double))
    return float(P), G


def reference_sets(table, n, K, level=1, cap=1 << 16):
    """(lower, upper) complete reference sets of a tabulated coherent Phi."""
    table = _c(table, np.uint8)
    lower = np.zeros((cap, n), dtype=np.uint8)
    upper = np.zeros((cap, n), dtype=np.uint8)
    nl = ctypes.c_int64(0)
    nu = ctypes.c_int64(0)
    _load().bf_reference_sets(n, K, _ptr(table, ctypes.c_uint8), int(level),
                              _ptr(lower, ctypes.c_uint8), ctypes.byref(nl),
                              _ptr(upper, ctypes.c_uint8), ctypes.byref(nu), cap)
    if nl.value > cap or nu.value > cap:
        raise ValueError("reference-set buffers too small")
    return lower[: nl.value].copy(), upper[: nu.value].copy()


def state_global(graph, x):
    """Global-connectivity system state of one state vector: 0 disconnected,
    1 connected with a bridge, 2 two-edge-connected (edges work when x_e >= 1)."""
    eu, ev = _graph_args(graph)
    x = _c(x, np.uint8)
    return int(_load().or_state_global(int(graph["n_nodes"]), eu.size, _ptr(eu, ctypes.c_int32),
                                       _ptr(ev, ctypes.c_int32), _ptr(x, ctypes.c_uint8)))


def eval_unknown_global(graph, x, flags, which=0, level=1):
    """As eval_unknown, for global connectivity at `level` (1 or 2)."""
    eu, ev = _graph_args(graph)
    x = _c(x, np.uint8)
    N = x.shape[0]
    flags = _c(flags, np.uint8) if flags is not None else np.zeros(N, dtype=np.uint8)
    Y = np.zeros(N, dtype=np.uint8)
    nev = _load().or_eval_global(int(graph["n_nodes"]), eu.size, _ptr(eu, ctypes.c_int32),
                                 _ptr(ev, ctypes.c_int32), int(level), _ptr(x, ctypes.c_uint8),
                                 _ptr(flags, ctypes.c_uint8), N, int(which),
                                 _ptr(Y, ctypes.c_uint8))
    return Y, int(nev)


def state_table_global(graph, K=2):
    """Global-connectivity system state (0, 1, 2) of every one of the K^n states."""
    eu, ev = _graph_args(graph)
    n = eu.size
    table = np.zeros(K ** n, dtype=np.uint8)
    _load().bf_state_table_global(int(graph["n_nodes"]), n, _ptr(eu, ctypes.c_int32),
                                  _ptr(ev, ctypes.c_int32), int(K), _ptr(table, ctypes.c_uint8))
    return table


def boundary_global(graph, x, K=2, level=1):
    """Componentwise boundary search for global connectivity at `level`."""
    eu, ev = _graph_args(graph)
    x = _c(np.atleast_2d(x), np.uint8)
    out = np.zeros_like(x)
    side = np.zeros(x.shape[0], dtype=np.uint8)
    nev = _load().or_boundary_global(int(graph["n_nodes"]), eu.size, _ptr(eu, ctypes.c_int32),
                                     _ptr(ev, ctypes.c_int32), int(level), int(K),
                                     _ptr(x, ctypes.c_uint8), x.shape[0],
                                     _ptr(out, ctypes.c_uint8), _ptr(side, ctypes.c_uint8))
    return out, side, int(nev)


def maxflow_st(graph, x):
    """Maximum s-t flow with edge capacities x (Edmonds-Karp)."""
    eu, ev = _graph_args(graph)
    x = _c(x, np.uint8)
    return int(_load().or_maxflow_st(int(graph["n_nodes"]), eu.size, _ptr(eu, ctypes.c_int32),
                                     _ptr(ev, ctypes.c_int32), int(graph["source"]),
                                     int(graph["sink"]), _ptr(x, ctypes.c_uint8)))


def eval_unknown_flow(graph, x, flags, which=0, demand=1):
    """As eval_unknown, for the target max flow >= demand."""
    eu, ev = _graph_args(graph)
    x = _c(x, np.uint8)
    N = x.shape[0]
    flags = _c(flags, np.uint8) if flags is not None else np.zeros(N, dtype=np.uint8)
    Y = np.zeros(N, dtype=np.uint8)
    nev = _load().or_eval_flow(int(graph["n_nodes"]), eu.size, _ptr(eu, ctypes.c_int32),
                               _ptr(ev, ctypes.c_int32), int(graph["source"]), int(graph["sink"]),
                               int(demand), _ptr(x, ctypes.c_uint8), _ptr(flags, ctypes.c_uint8),
                               N, int(which), _ptr(Y, ctypes.c_uint8))
    return Y, int(nev)


def maxflow_table(graph, K):
    """Max flow (capped at 255) of every one of the K^n states."""
    eu, ev = _graph_args(graph)
    n = eu.size
    table = np.zeros(K ** n, dtype=np.uint8)
    _load().bf_maxflow_table(int(graph["n_nodes"]), n, _ptr(eu, ctypes.c_int32),
                             _ptr(ev, ctypes.c_int32), int(graph["source"]), int(graph["sink"]),
                             int(K), _ptr(table, ctypes.c_uint8))
    return table


def boundary_flow(graph, x, K, demand):
    """Componentwise boundary search for the target max flow >= demand."""
    eu, ev = _graph_args(graph)
    x = _c(np.atleast_2d(x), np.uint8)
    out = np.zeros_like(x)
    side = np.zeros(x.shape[0], dtype=np.uint8)
    nev = _load().or_boundary_flow(int(graph["n_nodes"]), eu.size, _ptr(eu, ctypes.c_int32),
                                   _ptr(ev, ctypes.c_int32), int(graph["source"]),
                                   int(graph["sink"]), int(demand), int(K),
                                   _ptr(x, ctypes.c_uint8), x.shape[0],
                                   _ptr(out, ctypes.c_uint8), _ptr(side, ctypes.c_uint8))
    return out, side, int(nev)


def boundary_table(table, n, K, x, level=1):
    """Componentwise boundary search (section 3.4) with the system state given
    as a table over all K^n states.  Returns (states [Ns][n], side [Ns] with
    0 = lower / 1 = upper reference state, number of system evaluations)."""
    table = _c(table, np.uint8)
    x = _c(np.atleast_2d(x), np.uint8)
    out = np.zeros_like(x)
    side = np.zeros(x.shape[0], dtype=np.uint8)
    ev = _load().or_boundary_table(n, K, _ptr(table, ctypes.c_uint8), int(level),
                                   _ptr(x, ctypes.c_uint8), x.shape[0],
                                   _ptr(out, ctypes.c_uint8), _ptr(side, ctypes.c_uint8))
    return out, side, int(ev)


def boundary_st(graph, x, K=2, level=1):
    """Componentwise boundary search for s-t connectivity at `level`."""
    eu, ev = _graph_args(graph)
    x = _c(np.atleast_2d(x), np.uint8)
    out = np.zeros_like(x)
    side = np.zeros(x.shape[0], dtype=np.uint8)
    nev = _load().or_boundary_st(int(graph["n_nodes"]), eu.size, _ptr(eu, ctypes.c_int32),
                                 _ptr(ev, ctypes.c_int32), int(graph["source"]),
                                 int(graph["sink"]), int(level), int(K), _ptr(x, ctypes.c_uint8),
                                 x.shape[0], _ptr(out, ctypes.c_uint8),
                                 _ptr(side, ctypes.c_uint8))
    return out, side, int(nev)


def stage1(graph, p, N, picks, eps_u, max_rows, max_iters, seed, K=2, level=1, lower0=None,
           upper0=None, kind="st"):
    """The Stage-1 loop (section 3.5, fig. rsr_alg), written with the plain
    functions above.  Iteration it draws N samples (key seed, stream it),
    classifies them against the current rows (Algorithm 1), and stops when the
    unclassified fraction p_u is below eps_u, the rows number max_rows, or it
    is the last iteration; otherwise it searches from the first `picks`
    unclassified samples in index order (section 3.4) and appends each result
    not already present, in pick order, up to max_rows rows in total.
    kind = "global" uses global connectivity instead of s-t connectivity, and
    kind = "flow" the target max flow >= level.
    Returns (lower rows, upper rows, dict of iterations, p_u, searches,
    duplicates)."""
    n = np.asarray(p).shape[0]
    rows = [list(map(bytes, np.zeros((0, n), np.uint8) if lower0 is None else np.asarray(lower0, np.uint8))),
            list(map(bytes, np.zeros((0, n), np.uint8) if upper0 is None else np.asarray(upper0, np.uint8)))]
    seen = [set(rows[0]), set(rows[1])]
    info = {"iterations": 0, "p_u": 1.0, "searches": 0, "duplicates": 0}
    for it in range(max_iters):
        x = sample(p, seed, it, 0, N)
        as_arr = [np.frombuffer(b"".join(r), np.uint8).reshape(-1, n) for r in rows]
        flags, _, _ = classify(as_arr[0], as_arr[1], x, mode=0)
        unknown = np.nonzero((flags & 3) == 0)[0]
        info["iterations"] = it + 1
        info["p_u"] = unknown.size / N
        total = len(rows[0]) + len(rows[1])
        if info["p_u"] < eps_u or total >= max_rows or it + 1 == max_iters:
            break
        chosen = unknown[:picks]
        if chosen.size == 0:
            break
        if kind == "flow":
            out, side, _ = boundary_flow(graph, x[chosen], K, level)
        else:
            search = boundary_global if kind == "global" else boundary_st
            out, side, _ = search(graph, x[chosen], K=K, level=level)
        info["searches"] += chosen.size
        for r, sd in zip(out, side):
            if total >= max_rows:
                break
            key = bytes(r)
            if key in seen[sd]:
                info["duplicates"] += 1
                continue
            seen[sd].add(key)
            rows[sd].append(key)
            total += 1
    lo, up = (np.frombuffer(b"".join(r), np.uint8).reshape(-1, n).copy() for r in rows)
    return lo, up, info


def state_prob(p, x):
    p = _c(p, np.float64)
    n, K = p.shape
    x = _c(x, np.uint8)
    return float(_load().or_state_prob(n, K, _ptr(p, ctypes.c_double), _ptr(x, ctypes.c_uint8)))


def pmf_from_cdf(cdf):
    """System-state PMF from P(S <= m') for m' = 0..M_S-2 (section 3.5):
    P(S = 0) = P(S <= 0), P(S = m') = P(S <= m') - P(S <= m'-1),
    P(S = M_S-1) = 1 - P(S <= M_S-2)."""
    cdf = [float(c) for c in cdf]
    out = [cdf[0]]
    for k in range(1, len(cdf)):
        out.append(cdf[k] - cdf[k - 1])
    out.append(1.0 - cdf[-1])
    return out
