"""Pins of the oracle's componentwise boundary search (section 3.4): the
worked illustration of fig. x1x2_find_ref, closed forms on series and
parallel systems, minimality against brute-force reference sets, the
multi-state level structure, and two independent routes to the system
function (table and BFS)."""
import numpy as np

import oracle
import workloads as WL
from test_oracle_pins import _bridge, _golden_worked, _graph


def _table_from_minimal(minimal, n, K):
    """Coherent Phi: 1 iff x dominates one of the given minimal states."""
    idx = np.arange(K ** n)
    states = np.stack([(idx // K ** i) % K for i in range(n)], axis=1)
    above = np.zeros(idx.size, dtype=bool)
    for m in minimal:
        above |= np.all(states >= np.array(m), axis=1)
    return above.astype(np.uint8), states


def test_worked_illustration():
    """Fig. x1x2_find_ref: from the unclassified (2,0), raising X1 reaches
    Phi = 1 at (4,0), so X1 stays at 3; raising X2 reaches Phi = 1 at (3,2),
    so X2 stays at 1: the new lower reference state is (3,1), found with the
    first evaluation on the sample and four more along the way."""
    d = _golden_worked()
    M = d["M"]
    minimal = d["upper"] + d["phi_one"]
    table, states = _table_from_minimal(minimal, 2, M)
    # The coherent system built from the stated survival points must agree with
    # every value the text states, and keep the printed lower state below it.
    for x in d["phi_zero"] + d["lower"]:
        assert table[x[0] + M * x[1]] == 0
    for x in d["phi_one"]:
        assert table[x[0] + M * x[1]] == 1
    out, side, evals = oracle.boundary_table(table, 2, M, d["boundary_from"][0])
    assert tuple(out[0]) == d["boundary_result"][0]
    assert side[0] == 0
    assert evals == 5


def test_series_and_parallel_closed_forms():
    """Series: a failure sample keeps only its highest-index failed edge
    failed (raising the others in index order cannot connect s and t until the
    last one); a survival sample is already the unique path.  Parallel: a
    survival sample keeps only its highest-index working edge; a failure
    sample is the all-failed state."""
    n = 9
    series = _graph(n + 1, [(i, i + 1) for i in range(n)], 0, n)
    parallel = _graph(2, [(0, 1)] * n, 0, 1)
    rng = np.random.default_rng(21)
    for _ in range(40):
        x = (rng.random(n) < 0.6).astype(np.uint8)
        out, side, _ = oracle.boundary_st(series, x)
        if x.all():
            assert side[0] == 1 and out[0].tolist() == [1] * n
        else:
            last = int(np.nonzero(x == 0)[0].max())
            want = np.ones(n, np.uint8)
            want[last] = 0
            assert side[0] == 0 and out[0].tolist() == want.tolist()
        out, side, _ = oracle.boundary_st(parallel, x)
        if not x.any():
            assert side[0] == 0 and out[0].tolist() == [0] * n
        else:
            last = int(np.nonzero(x == 1)[0].max())
            want = np.zeros(n, np.uint8)
            want[last] = 1
            assert side[0] == 1 and out[0].tolist() == want.tolist()


def test_results_are_boundary_states_on_tiny():
    """Every search result on the 20-edge graph is a minimal cut / path state
    of the brute-force reference sets, on the side of its start, and lies
    above (failure) or below (survival) the start."""
    c = WL.configs.tiny(N=10)
    n = c["n"]
    table = oracle.phi_table_st(c["graph"])
    lo, up = oracle.reference_sets(table, n, 2)
    lo_set, up_set = set(map(bytes, lo)), set(map(bytes, up))
    rng = np.random.default_rng(22)
    x = (rng.random((400, n)) < rng.uniform(0.2, 0.9, (400, 1))).astype(np.uint8)
    out, side, _ = oracle.boundary_st(c["graph"], x)
    for h in range(x.shape[0]):
        phi = oracle.phi_st(c["graph"], x[h])
        assert side[h] == phi
        if phi:
            assert bytes(out[h]) in up_set and np.all(out[h] <= x[h])
        else:
            assert bytes(out[h]) in lo_set and np.all(out[h] >= x[h])
    # Two routes to Phi (table lookup, BFS) give the same searches.
    out_t, side_t, _ = oracle.boundary_table(table, n, 2, x)
    np.testing.assert_array_equal(out_t, out)
    np.testing.assert_array_equal(side_t, side)


def test_multistate_levels_on_the_bridge():
    """K = 3 bridge, levels 1 and 2, every one of the 3^5 start states: the
    result is in the brute-force reference sets of that level, and since Phi
    depends only on which edges reach the level, failure results hold each
    edge at level-1 or K-1 and survival results at 0 or the level."""
    g = _bridge()
    K = 3
    idx = np.arange(K ** 5)
    states = np.stack([(idx // K ** i) % K for i in range(5)], axis=1).astype(np.uint8)
    for level in (1, 2):
        table = oracle.phi_table_st(g, K=K, level=level)
        lo, up = oracle.reference_sets(table, 5, K, level=1)
        lo_set, up_set = set(map(bytes, lo)), set(map(bytes, up))
        out, side, _ = oracle.boundary_st(g, states, K=K, level=level)
        out_t, side_t, _ = oracle.boundary_table(table, 5, K, states)
        np.testing.assert_array_equal(out_t, out)
        np.testing.assert_array_equal(side_t, side)
        for h in range(states.shape[0]):
            assert side[h] == table[h]
            if side[h]:
                assert bytes(out[h]) in up_set
                assert set(out[h].tolist()) <= {0, level}
            else:
                assert bytes(out[h]) in lo_set
                assert set(out[h].tolist()) <= {level - 1, K - 1}


def test_stage1_loop_on_tiny():
    """The oracle's Stage-1 loop from empty reference sets on the 20-edge
    graph: every row it finds is a brute-force boundary state of its side,
    the sets grow until a fresh sample set has no unclassified sample, and
    picks = 1 (the paper's one search per iteration) finds one new row per
    iteration until then."""
    c = WL.configs.tiny(N=10)
    n = c["n"]
    table = oracle.phi_table_st(c["graph"])
    lo_all, up_all = oracle.reference_sets(table, n, 2)
    lo_set, up_set = set(map(bytes, lo_all)), set(map(bytes, up_all))
    p = WL.configs.binary_model(c["p"][:, 1] * 0.9)
    lo, up, info = oracle.stage1(c["graph"], p, N=3000, picks=16, eps_u=1e-9, max_rows=10_000,
                                 max_iters=60, seed=3)
    assert info["p_u"] == 0.0 and info["iterations"] < 60
    assert len(lo) + len(up) + info["duplicates"] == info["searches"]
    assert set(map(bytes, lo)) <= lo_set and set(map(bytes, up)) <= up_set
    assert len(set(map(bytes, lo))) == len(lo) and len(set(map(bytes, up))) == len(up)
    # The grown sets are valid: no state is labelled against its Phi.
    idx = np.arange(1 << n, dtype=np.uint64)
    states = ((idx[:, None] >> np.arange(n, dtype=np.uint64)) & np.uint64(1)).astype(np.uint8)
    flags, _, _ = oracle.classify(lo, up, states, mode=1)
    assert not np.any((flags & 1) & (table == 1)) and not np.any((flags & 2) & (table == 0))
    lo1, up1, info1 = oracle.stage1(c["graph"], p, N=3000, picks=1, eps_u=1e-9, max_rows=10_000,
                                    max_iters=8, seed=3)
    assert info1["searches"] == 7 and info1["duplicates"] == 0 and len(lo1) + len(up1) == 7
    # max_rows caps the total, and the loop stops once it is reached.
    lo2, up2, info2 = oracle.stage1(c["graph"], p, N=3000, picks=16, eps_u=0.0, max_rows=5,
                                    max_iters=60, seed=3)
    assert len(lo2) + len(up2) == 5 and info2["iterations"] == 2
