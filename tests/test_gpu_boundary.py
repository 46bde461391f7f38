"""GPU parity of the componentwise boundary search (section 3.4): the rows and
sides from rsr_boundary_search must equal the oracle's search (which
evaluates the system function at every single step) bit for bit, on the
same seeded samples; plus the edge cases of the pick list."""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_17066_amd as R
import workloads as WL

pytestmark = pytest.mark.gpu


def _search(ctx, graph, p, K, level, seed, N, picks):
    m = R.Model(ctx, p)
    xs = R.rsr_sample(ctx, m, seed, 0, 0, N)
    system = R.System(ctx, graph, K=K, level=level)
    d_picks = torch.tensor(picks, dtype=torch.int64, device=ctx.device)
    rows, side = R.rsr_boundary_search(ctx, system, xs, N, d_picks)
    torch.cuda.synchronize()
    states = oracle.sample(p, seed, 0, 0, N)
    want_rows, want_side, _ = oracle.boundary_st(graph, states[picks], K=K, level=level)
    return rows.cpu().numpy(), side.cpu().numpy(), want_rows, want_side


@pytest.mark.parametrize("case", ["tiny", "graph2", "large"])
def test_boundary_binary_matches_oracle(rsr_ctx, case):
    rng = np.random.default_rng(31)
    if case == "tiny":
        c = WL.configs.tiny(N=10)
        graph, p, N, n_pick = c["graph"], c["p"], 3000, 3000
        # push the survival probabilities down so both sides are common
        p = WL.configs.binary_model(p[:, 1] * 0.85)
    elif case == "graph2":
        c = WL.configs.graph2(N=1, R_U=10, R_L=10)
        graph, p, N, n_pick = c["graph"], c["p"], 4096, 700
    else:
        sd = WL.configs.batched(n_scen=1, N=1, graphs=[7], ref_scale=1e-5)
        graph = sd["systems"][0]["graph"]
        p, N, n_pick = sd["jobs"][0]["p"], 512, 24
    picks = rng.choice(N, size=n_pick, replace=n_pick > N // 2).astype(np.int64)
    rows, side, want_rows, want_side = _search(rsr_ctx, graph, p, 2, 1, 77, N, picks)
    print(case, "upper picks:", int(side.sum()), "of", n_pick)
    if case != "large":
        assert 0 < side.sum() < n_pick
    np.testing.assert_array_equal(side, want_side)
    np.testing.assert_array_equal(rows, want_rows)


@pytest.mark.parametrize("level", [1, 2])
def test_boundary_multistate_matches_oracle(rsr_ctx, level):
    c = WL.configs.multi(N=1, R_per_level=4)
    N = 2048
    picks = np.arange(0, N, 7, dtype=np.int64)
    rows, side, want_rows, want_side = _search(rsr_ctx, c["graph"], c["p"], 3, level, 91, N, picks)
    print("level", level, "upper picks:", int(side.sum()), "of", picks.size)
    np.testing.assert_array_equal(side, want_side)
    np.testing.assert_array_equal(rows, want_rows)
    lo_vals = {level - 1, 2}
    up_vals = {0, level}
    for r, s in zip(rows, side):
        assert set(np.unique(r).tolist()) <= (up_vals if s else lo_vals)


def test_boundary_pick_edge_cases(rsr_ctx):
    c = WL.configs.tiny(N=10)
    N = 100
    m = R.Model(rsr_ctx, c["p"])
    xs = R.rsr_sample(rsr_ctx, m, 5, 0, 0, N)
    system = R.System(rsr_ctx, c["graph"])
    # n_pick = 0 is a no-op
    empty = torch.empty(0, dtype=torch.int64, device=rsr_ctx.device)
    rows, side = R.rsr_boundary_search(rsr_ctx, system, xs, N, empty)
    assert rows.shape == (0, c["n"]) and side.shape == (0,)
    # out-of-range indices are reported in side and leave their row alone;
    # repeated indices give repeated rows
    picks = torch.tensor([3, -1, N, 3, N - 1], dtype=torch.int64, device=rsr_ctx.device)
    rows = torch.full((5, c["n"]), 0xAB, dtype=torch.uint8, device=rsr_ctx.device)
    side = torch.zeros(5, dtype=torch.uint8, device=rsr_ctx.device)
    R.rsr_boundary_search(rsr_ctx, system, xs, N, picks, rows=rows, side=side)
    torch.cuda.synchronize()
    r, s = rows.cpu().numpy(), side.cpu().numpy()
    assert s[1] == 0xFF and s[2] == 0xFF
    assert np.all(r[1] == 0xAB) and np.all(r[2] == 0xAB)
    np.testing.assert_array_equal(r[0], r[3])
    states = oracle.sample(c["p"], 5, 0, 0, N)
    want, want_side, _ = oracle.boundary_st(c["graph"], states[[3, N - 1]])
    np.testing.assert_array_equal(r[[0, 4]], want)
    np.testing.assert_array_equal(s[[0, 4]], want_side)
    with pytest.raises(R.RSRError):
        R.rsr_boundary_search(rsr_ctx, system, xs, 0, picks)


@pytest.mark.parametrize("case", ["tiny", "graph2", "multi"])
def test_stage1_loop_matches_oracle(rsr_ctx, case):
    """rsr_stage1 against the oracle's loop: the same rows in the same order,
    the same iteration count, unclassified fraction, searches and
    duplicates."""
    K, level, lower0, upper0 = 2, 1, None, None
    if case == "tiny":
        c = WL.configs.tiny(N=10)
        graph, p = c["graph"], WL.configs.binary_model(c["p"][:, 1] * 0.9)
        N, picks, iters, max_rows = 3000, 16, 40, 10_000
    elif case == "graph2":
        c = WL.configs.graph2(N=1, R_U=40, R_L=40)
        graph, p = c["graph"], c["p"]
        N, picks, iters, max_rows = 20_000, 64, 4, 10_000
        lower0, upper0 = c["lower"], c["upper"]      # start from given rows
    else:
        c = WL.configs.multi(N=1, R_per_level=4)
        graph, p, K, level = c["graph"], c["p"], 3, 2
        N, picks, iters, max_rows = 10_000, 32, 3, 70
    m = R.Model(rsr_ctx, p)
    system = R.System(rsr_ctx, graph, K=K, level=level)
    lo, up, info = R.stage1(rsr_ctx, m, system, N, picks, 1e-9, max_rows, iters, 17,
                            lower0=lower0, upper0=upper0)
    wlo, wup, winfo = oracle.stage1(graph, p, N, picks, 1e-9, max_rows, iters, 17, K=K,
                                    level=level, lower0=lower0, upper0=upper0)
    print(case, info)
    for key in ("iterations", "p_u", "searches", "duplicates"):
        assert info[key] == winfo[key], key
    np.testing.assert_array_equal(lo, wlo)
    np.testing.assert_array_equal(up, wup)
    assert info["searches"] > 0
