"""Property tests of the oracle on random coherent systems (s-t connectivity
of random multigraphs, K = 2 or 3 states, every level), tabulated over all
K^n states so that each property is checked against brute force:

* the system function is coherent: nondecreasing in every component, 0 at
  the all-failed state, and 1 at the all-working state exactly when the
  terminals are joined in the multigraph (section 2.1);
* complete reference sets (section 2.2) classify every state, on the side
  the table gives, and their rows are the extreme states of their side;
* with any subsets of the reference rows, LABEL flags (Algorithm 1) are never
  wrong, Stage 2 evaluates exactly the unclassified samples, and the RSR
  estimate equals crude Monte Carlo on the same samples (section 3.1);
* the boundary search (section 3.4) from any state ends on a reference row of
  that state's side, above a failed start and below a working one;
* the score-function counts (section 3.5) add up per component to the
  number of working samples, and sum_s p_is G_is = P-hat for every i."""
import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from strategies import all_states, st_systems

SETTINGS = settings(max_examples=150, deadline=None, derandomize=True, database=None,
                    suppress_health_check=[HealthCheck.too_slow, HealthCheck.filter_too_much])


def _table(graph, K, level):
    return oracle.phi_table_st(graph, K=K, level=level)


def _index(x, K):
    return (x.astype(np.int64) * (K ** np.arange(x.shape[1], dtype=np.int64))).sum(axis=1)


def _joined(graph):
    """Terminals joined when every edge works (union-find, not BFS)."""
    parent = list(range(graph["n_nodes"]))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for u, v in zip(graph["edge_u"], graph["edge_v"]):
        parent[find(int(u))] = find(int(v))
    return find(graph["source"]) == find(graph["sink"])


@SETTINGS
@given(st_systems())
def test_system_function_is_coherent(sysd):
    graph, K, level, _, _ = sysd
    n = graph["edge_u"].size
    table = _table(graph, K, level)
    x = all_states(n, K)
    idx = _index(x, K)
    assert table[0] == 0
    assert table[-1] == int(_joined(graph))
    for i in range(n):
        up = x[:, i] < K - 1
        assert np.all(table[idx[up] + K ** i] >= table[idx[up]]), i


@SETTINGS
@given(st_systems())
def test_complete_reference_sets_classify_every_state(sysd):
    graph, K, level, _, _ = sysd
    n = graph["edge_u"].size
    table = _table(graph, K, level)
    lo, up = oracle.reference_sets(table, n, K, level=1)
    x = all_states(n, K)
    flags, mL, mU = oracle.classify(lo, up, x, mode=1)
    np.testing.assert_array_equal(flags == 1, table == 0)
    np.testing.assert_array_equal(flags == 2, table == 1)
    assert np.all((mL > 0) == (table == 0)) and np.all((mU > 0) == (table == 1))
    # Rows are the extreme states of their side: one step up from a lower
    # row, or down from an upper row, crosses to the other side.
    for rows, val, step in ((lo, 0, 1), (up, 1, -1)):
        assert len({bytes(r) for r in rows}) == len(rows)
        ri = _index(rows, K)
        assert np.all(table[ri] == val)
        for i in range(n):
            can = (rows[:, i] < K - 1) if step == 1 else (rows[:, i] > 0)
            assert np.all(table[ri[can] + step * K ** i] == 1 - val), (val, i)


@SETTINGS
@given(st_systems(), st.floats(0.0, 1.0), st.floats(0.0, 1.0), st.integers(1, 3000))
def test_partial_reference_sets_give_crude_monte_carlo(sysd, keep_l, keep_u, N):
    graph, K, level, p, seed = sysd
    n = graph["edge_u"].size
    table = _table(graph, K, level)
    lo, up = oracle.reference_sets(table, n, K, level=1)
    rng = np.random.default_rng(seed + 1)
    lo = np.ascontiguousarray(lo[rng.random(len(lo)) < keep_l])
    up = np.ascontiguousarray(up[rng.random(len(up)) < keep_u])
    x = oracle.sample(p, seed, 3, 0, N)
    phi = table[_index(x, K)]
    fl, _, _ = oracle.classify(lo, up, x, mode=0)
    assert np.all(phi[fl == 1] == 0) and np.all(phi[fl == 2] == 1)
    Y, nev = oracle.eval_unknown(graph, x, fl, which=0, level=level)
    unknown = fl == 0
    assert nev == int(unknown.sum())
    np.testing.assert_array_equal(Y[unknown], phi[unknown])
    cnt = oracle.counts(fl, Y)
    assert int(cnt[0] + cnt[1] + cnt[2]) == N
    est = oracle.estimate(cnt)
    want = int(phi.sum()) / N
    assert abs(est[3] - want) <= 1e-15 * max(1.0, want)
    # Score-function counts over every sample's Phi.
    c, G = oracle.grad(p, x, phi)
    assert np.all(c.sum(axis=1) == int(phi.sum()))
    np.testing.assert_allclose((p * G).sum(axis=1), want, rtol=1e-12, atol=1e-15)


@SETTINGS
@given(st_systems(), st.integers(1, 40))
def test_boundary_search_ends_on_a_reference_row(sysd, n_starts):
    graph, K, level, _, seed = sysd
    n = graph["edge_u"].size
    table = _table(graph, K, level)
    lo, up = oracle.reference_sets(table, n, K, level=1)
    lo_set, up_set = {bytes(r) for r in lo}, {bytes(r) for r in up}
    x = np.random.default_rng(seed + 2).integers(0, K, (n_starts, n)).astype(np.uint8)
    out, side, _ = oracle.boundary_st(graph, x, K=K, level=level)
    phi = table[_index(x, K)]
    np.testing.assert_array_equal(side, phi)
    for h in range(n_starts):
        if phi[h]:
            assert bytes(out[h]) in up_set and np.all(out[h] <= x[h])
        else:
            assert bytes(out[h]) in lo_set and np.all(out[h] >= x[h])
