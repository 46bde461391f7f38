"""GPU parity of the single-OD maximum-flow system (multi-state capacities,
target flow >= d): evaluation, boundary search (d-minimal path and cut
vectors), the Stage-2 path with brute-force reference sets and the Stage-1
loop, all against the oracle on the same seeded samples."""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_17066_amd as R
import workloads as WL

pytestmark = pytest.mark.gpu


def _cases():
    rng = np.random.default_rng(81)
    tiny = WL.configs.tiny(N=10)["graph"]
    multi = WL.configs.multi(N=1, R_per_level=4)
    grid = WL.graphs.grid(3, 3)
    return {
        "tiny_K4": (tiny, rng.dirichlet([1.0, 1.5, 2.0, 3.0], size=20), 4),
        "graph2_K3": (multi["graph"], multi["p"], 3),
        "grid_K3": (grid, rng.dirichlet([1.0, 2.0, 4.0], size=12), 3),
    }


@pytest.mark.parametrize("case", ["tiny_K4", "graph2_K3", "grid_K3"])
@pytest.mark.parametrize("demand", [1, 2, 4])
def test_flow_eval_matches_oracle(rsr_ctx, case, demand):
    graph, p, K = _cases()[case]
    N = 3000
    m = R.Model(rsr_ctx, p)
    xs = R.rsr_sample(rsr_ctx, m, 5, 0, 0, N)
    system = R.System(rsr_ctx, graph, K=K, level=demand, kind="flow")
    Y = R.rsr_eval_unknown(rsr_ctx, system, xs, N, None, which=R.RSR_ALL)
    torch.cuda.synchronize()
    x = oracle.sample(p, 5, 0, 0, N)
    want, _ = oracle.eval_unknown_flow(graph, x, None, which=1, demand=demand)
    print(case, demand, "P(flow >= d) =", want.mean())
    np.testing.assert_array_equal(Y.cpu().numpy(), want)


@pytest.mark.parametrize("case,demand,n_pick", [("tiny_K4", 2, 500), ("tiny_K4", 3, 500),
                                                ("grid_K3", 2, 500), ("graph2_K3", 2, 64)])
def test_flow_boundary_matches_oracle(rsr_ctx, case, demand, n_pick):
    graph, p, K = _cases()[case]
    N = 2048
    m = R.Model(rsr_ctx, p)
    xs = R.rsr_sample(rsr_ctx, m, 8, 0, 0, N)
    system = R.System(rsr_ctx, graph, K=K, level=demand, kind="flow")
    picks = np.random.default_rng(82).choice(N, size=n_pick, replace=False).astype(np.int64)
    rows, side = R.rsr_boundary_search(rsr_ctx, system, xs, N,
                                       torch.tensor(picks, device=rsr_ctx.device))
    torch.cuda.synchronize()
    x = oracle.sample(p, 8, 0, 0, N)
    want_rows, want_side, _ = oracle.boundary_flow(graph, x[picks], K, demand)
    print(case, demand, "survival picks:", int(want_side.sum()), "of", n_pick)
    assert 0 < want_side.sum() < n_pick
    np.testing.assert_array_equal(side.cpu().numpy(), want_side)
    np.testing.assert_array_equal(rows.cpu().numpy(), want_rows)


@pytest.mark.parametrize("demand", [1, 2, 3])
def test_flow_stage2_path_matches_oracle(rsr_ctx, demand):
    """2 x 3 grid (7 edges) with capacities 0..3: half of the complete
    d-minimal path / cut vectors from brute force over 4^7 states; labels,
    evaluations, estimate and gradient counts equal the oracle's."""
    graph = WL.graphs.grid(2, 3)
    K, n, N = 4, 7, 40_000
    p = np.random.default_rng(83).dirichlet([1.0, 1.5, 2.0, 3.0], size=n)
    table = oracle.maxflow_table(graph, K)
    lo, up = oracle.reference_sets(table, n, K, level=demand)
    lo, up = lo[::2], up[::2]
    m = R.Model(rsr_ctx, p)
    refs = R.Refs(rsr_ctx, n, K, lo, up)
    system = R.System(rsr_ctx, graph, K=K, level=demand, kind="flow")
    est, buf = R.stage2(rsr_ctx, m, refs, system, N, 9)
    _, counts = R.rsr_grad(rsr_ctx, m, buf.samples, buf.Y, N, want_counts=True)
    torch.cuda.synchronize()
    x = oracle.sample(p, 9, 0, 0, N)
    flags, _, _ = oracle.classify(lo, up, x, mode=0)
    Y, _ = oracle.eval_unknown_flow(graph, x, flags, demand=demand)
    cnt = oracle.counts(flags, Y)
    want = oracle.estimate(cnt)
    np.testing.assert_array_equal(buf.flags.cpu().numpy(), flags)
    np.testing.assert_array_equal(buf.Y.cpu().numpy(), Y)
    assert est["P"] == want[3] and est["n_u"] == int(cnt[2])
    assert 0 < est["n_u"] < N
    wcounts, _ = oracle.grad(p, x, Y)
    np.testing.assert_array_equal(counts.cpu().numpy().astype(np.uint64), wcounts)


@pytest.mark.parametrize("demand", [1, 2])
def test_flow_stage1_loop_matches_oracle(rsr_ctx, demand):
    graph, p, K = _cases()["grid_K3"]
    m = R.Model(rsr_ctx, p)
    system = R.System(rsr_ctx, graph, K=K, level=demand, kind="flow")
    lo, up, info = R.stage1(rsr_ctx, m, system, 3000, 16, 1e-9, 10_000, 8, 29)
    wlo, wup, winfo = oracle.stage1(graph, p, 3000, 16, 1e-9, 10_000, 8, 29, K=K, level=demand,
                                    kind="flow")
    print(demand, info)
    for key in ("iterations", "p_u", "searches", "duplicates"):
        assert info[key] == winfo[key], key
    np.testing.assert_array_equal(lo, wlo)
    np.testing.assert_array_equal(up, wup)
