"""GPU property tests on random coherent systems: s-t connectivity of random
multigraphs with K = 2 or 3 states at every level, random state
probabilities, random subsets of the complete reference sets (either side
may be empty) and a random sample count.  Through the C ABI, the whole
Stage-2 path (sample, LABEL classify, evaluate the unclassified samples,
estimate, gradient) equals the oracle: flags, Y and counts exactly, the
estimate bit for bit, the gradient within 1e-5 relative; COUNT mode in
every form gives the oracle's flags and match counts, and LABEL mode in
every form (the persistent cascade included) its flags."""
import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
import paper_2604_17066_amd as R
from strategies import st_systems

pytestmark = pytest.mark.gpu

GRAD_RTOL = 1e-5
SETTINGS = settings(max_examples=60, deadline=None, derandomize=True, database=None,
                    suppress_health_check=[HealthCheck.too_slow, HealthCheck.filter_too_much])


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _refs(graph, K, level, seed, keep_l, keep_u):
    n = graph["edge_u"].size
    table = oracle.phi_table_st(graph, K=K, level=level)
    lo, up = oracle.reference_sets(table, n, K, level=1)
    rng = np.random.default_rng(seed + 1)
    lo = np.ascontiguousarray(lo[rng.random(len(lo)) < keep_l])
    up = np.ascontiguousarray(up[rng.random(len(up)) < keep_u])
    return lo, up


@SETTINGS
@given(st_systems(), st.floats(0.0, 1.0), st.floats(0.0, 1.0), st.integers(1, 5000))
def test_random_systems_full_path(rsr_ctx, sysd, keep_l, keep_u, N):
    graph, K, level, p, seed = sysd
    n = graph["edge_u"].size
    lo, up = _refs(graph, K, level, seed, keep_l, keep_u)
    print(f"K={K} level={level} n={n} rows={len(lo)}+{len(up)} N={N} seed={seed}", flush=True)
    m = R.Model(rsr_ctx, p)
    refs = R.Refs(rsr_ctx, n, K, lo, up)
    sysm = R.System(rsr_ctx, graph, K=K, level=level)
    est, buf = R.stage2(rsr_ctx, m, refs, sysm, N, seed, stream_id=5)
    G, counts = R.rsr_grad(rsr_ctx, m, buf.samples, buf.Y, N, want_counts=True)
    x = oracle.sample(p, seed, 5, 0, N)
    fl, _, _ = oracle.classify(lo, up, x, mode=0)
    Y, nev = oracle.eval_unknown(graph, x, fl, which=0, level=level)
    cnt = oracle.counts(fl, Y)
    oest = oracle.estimate(cnt)
    c, Gref = oracle.grad(p, x, Y)
    np.testing.assert_array_equal(_np(buf.flags), fl)
    np.testing.assert_array_equal(_np(buf.Y), Y)
    assert int(_np(buf.n_eval)[0]) == nev
    for k, name in enumerate(oracle.COUNT_NAMES):
        assert est[name] == int(cnt[k]), name
    for k, name in enumerate(oracle.EST_NAMES):
        assert est[name] == oest[k] or (np.isinf(est[name]) and np.isinf(oest[k])), name
    np.testing.assert_array_equal(_np(counts).view(np.uint64), c)
    G = _np(G).astype(np.float64)
    nz = Gref != 0
    assert np.all(np.abs(G[nz] - Gref[nz]) <= GRAD_RTOL * np.abs(Gref[nz]))
    assert np.all(G[~nz] == 0.0)


@SETTINGS
@given(st_systems(min_edges=6), st.floats(0.0, 1.0), st.floats(0.0, 1.0), st.integers(1, 5000))
def test_random_systems_every_form(rsr_ctx, sysd, keep_l, keep_u, N):
    graph, K, level, p, seed = sysd
    n = graph["edge_u"].size
    lo, up = _refs(graph, K, level, seed, keep_l, keep_u)
    print(f"K={K} level={level} n={n} rows={len(lo)}+{len(up)} N={N} seed={seed}", flush=True)
    m = R.Model(rsr_ctx, p)
    refs = R.Refs(rsr_ctx, n, K, lo, up)
    assert refs.consistent
    xs = R.rsr_sample(rsr_ctx, m, seed, 0, 0, N)
    x = oracle.sample(p, seed, 0, 0, N)
    ol, _, _ = oracle.classify(lo, up, x, mode=0)
    oc, mL, mU = oracle.classify(lo, up, x, mode=1)
    for form in (R.RSR_POPCOUNT, R.RSR_MFMA, R.RSR_MFMA_FP4, R.RSR_AUTO):
        fc, mt = R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_COUNT, form, want_match=True)
        mt = _np(mt).view(np.uint32)
        np.testing.assert_array_equal(_np(fc), oc, err_msg=f"COUNT flags, form {form}")
        np.testing.assert_array_equal(mt[:, 0], mL, err_msg=f"lower matches, form {form}")
        np.testing.assert_array_equal(mt[:, 1], mU, err_msg=f"upper matches, form {form}")
    for form in (R.RSR_POPCOUNT, R.RSR_MFMA, R.RSR_MFMA_FP4, R.RSR_AUTO, R.RSR_PERSIST):
        fl = R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_LABEL, form)
        np.testing.assert_array_equal(_np(fl), ol, err_msg=f"LABEL flags, form {form}")


@st.composite
def st_plans(draw):
    """One to three random systems (each with its own K and level), one to
    three jobs per system with their own probabilities, seeds and sample
    counts (1 to 4000), and random subsets of the reference rows."""
    systems = []
    for _ in range(draw(st.integers(1, 3))):
        sysd = draw(st_systems(max_states=1 << 12))
        keep = (draw(st.floats(0.0, 1.0)), draw(st.floats(0.0, 1.0)))
        jobs = [(draw(st.integers(0, 2**31 - 1)), draw(st.integers(1, 4000)))
                for _ in range(draw(st.integers(1, 3)))]
        systems.append((sysd, keep, jobs))
    return systems


@settings(max_examples=20, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.filter_too_much])
@given(st_plans())
def test_random_plans_equal_the_plain_path(rsr_ctx, plan_d):
    """A plan over random systems and jobs (segments of different widths, K
    and levels in one captured graph): every job's flags, Y and estimate
    equal the plain one-job path's, and its flags the oracle's."""
    jobs, plain = [], []
    for (graph, K, level, p0, seed), (keep_l, keep_u), job_list in plan_d:
        n = graph["edge_u"].size
        lo, up = _refs(graph, K, level, seed, keep_l, keep_u)
        refs = R.Refs(rsr_ctx, n, K, lo, up)
        sysm = R.System(rsr_ctx, graph, K=K, level=level)
        for jseed, N in job_list:
            rng = np.random.default_rng(jseed)
            p = rng.uniform(0.05, 1.0, (n, K))
            p /= p.sum(axis=1, keepdims=True)
            m = R.Model(rsr_ctx, np.ascontiguousarray(p))
            jobs.append({"model": m, "refs": refs, "system": sysm, "seed": jseed, "N": N,
                         "buffers": R.Buffers(rsr_ctx, n, K, N), "grad": True})
            plain.append((lo, up, p, graph, level))
    print(f"plan: {len(plan_d)} systems, {len(jobs)} jobs, N = {[jb['N'] for jb in jobs]}", flush=True)
    plan = R.Plan(rsr_ctx, jobs, tune=False)
    plan.run()
    est, _ = plan.results()
    for k, (jb, (lo, up, p, graph, level)) in enumerate(zip(jobs, plain)):
        N = jb["N"]
        pe, pb = R.stage2(rsr_ctx, jb["model"], jb["refs"], jb["system"], N, jb["seed"])
        b = jb["buffers"]
        np.testing.assert_array_equal(_np(b.flags), _np(pb.flags), err_msg=f"job {k}")
        np.testing.assert_array_equal(_np(b.Y), _np(pb.Y), err_msg=f"job {k}")
        assert est[k]["P"] == pe["P"] and est[k]["n_u"] == pe["n_u"], k
        x = oracle.sample(p, jb["seed"], 0, 0, N)
        fl, _, _ = oracle.classify(lo, up, x, mode=0)
        np.testing.assert_array_equal(_np(b.flags), fl, err_msg=f"job {k} against the oracle")
    plan.close()


@SETTINGS
@given(st_systems(max_states=1 << 12), st.sampled_from(("global", "flow")), st.integers(1, 3),
       st.floats(0.0, 1.0), st.floats(0.0, 1.0), st.integers(1, 3000))
def test_random_global_and_flow_systems(rsr_ctx, sysd, kind, d, keep_l, keep_u, N):
    """The other system kinds on random multigraphs: global connectivity
    (K = 2, level 1 or 2) and maximum s-t flow >= d (capacities 0..K-1, d =
    1..3), reference rows from the brute-force state tables; the Stage-2
    path's flags, Y and counts equal the oracle's."""
    graph, K, _, p, seed = sysd
    n = graph["edge_u"].size
    rng = np.random.default_rng(seed + 3)
    if kind == "global":
        K, level = 2, 1 + (d - 1) % 2
        p = rng.uniform(0.05, 1.0, (n, 2))
        p = np.ascontiguousarray(p / p.sum(axis=1, keepdims=True))
        table = oracle.state_table_global(graph, 2)
        sysm = R.System(rsr_ctx, graph, level=level, kind="global")
    else:
        level = d
        table = oracle.maxflow_table(graph, K)
        sysm = R.System(rsr_ctx, graph, K=K, level=level, kind="flow")
    lo, up = oracle.reference_sets(table, n, K, level=level)
    lo = np.ascontiguousarray(lo[rng.random(len(lo)) < keep_l])
    up = np.ascontiguousarray(up[rng.random(len(up)) < keep_u])
    print(f"{kind} K={K} level={level} n={n} rows={len(lo)}+{len(up)} N={N} seed={seed}", flush=True)
    m = R.Model(rsr_ctx, p)
    refs = R.Refs(rsr_ctx, n, K, lo, up)
    est, buf = R.stage2(rsr_ctx, m, refs, sysm, N, seed)
    x = oracle.sample(p, seed, 0, 0, N)
    fl, _, _ = oracle.classify(lo, up, x, mode=0)
    if kind == "global":
        Y, nev = oracle.eval_unknown_global(graph, x, fl, which=0, level=level)
    else:
        Y, nev = oracle.eval_unknown_flow(graph, x, fl, which=0, demand=level)
    np.testing.assert_array_equal(_np(buf.flags), fl)
    np.testing.assert_array_equal(_np(buf.Y), Y)
    assert int(_np(buf.n_eval)[0]) == nev
    cnt = oracle.counts(fl, Y)
    for k, name in enumerate(oracle.COUNT_NAMES):
        assert est[name] == int(cnt[k]), name


@SETTINGS
@given(st_systems(max_states=1 << 12), st.sampled_from(("st", "global", "flow")), st.integers(1, 3),
       st.integers(1, 2000), st.integers(1, 256))
def test_random_boundary_searches(rsr_ctx, sysd, kind, d, N, n_pick):
    """The componentwise boundary search (section 3.4) on random multigraphs
    of every system kind, from random picks (repeats allowed): rows and sides
    equal the oracle's search, which evaluates the system function at every
    single step."""
    graph, K, level, p, seed = sysd
    n = graph["edge_u"].size
    rng = np.random.default_rng(seed + 5)
    if kind == "global":
        K, level = 2, 1 + (d - 1) % 2
        p = rng.uniform(0.05, 1.0, (n, 2))
        p = np.ascontiguousarray(p / p.sum(axis=1, keepdims=True))
        sysm = R.System(rsr_ctx, graph, level=level, kind="global")
    elif kind == "flow":
        level = d
        sysm = R.System(rsr_ctx, graph, K=K, level=level, kind="flow")
    else:
        sysm = R.System(rsr_ctx, graph, K=K, level=level)
    picks = rng.integers(0, N, n_pick).astype(np.int64)
    print(f"{kind} K={K} level={level} n={n} N={N} picks={n_pick} seed={seed}", flush=True)
    m = R.Model(rsr_ctx, p)
    xs = R.rsr_sample(rsr_ctx, m, seed, 0, 0, N)
    rows, side = R.rsr_boundary_search(rsr_ctx, sysm, xs, N,
                                       torch.tensor(picks, dtype=torch.int64, device=rsr_ctx.device))
    x = oracle.sample(p, seed, 0, 0, N)[picks]
    if kind == "global":
        want_rows, want_side, _ = oracle.boundary_global(graph, x, K=2, level=level)
    elif kind == "flow":
        want_rows, want_side, _ = oracle.boundary_flow(graph, x, K, level)
    else:
        want_rows, want_side, _ = oracle.boundary_st(graph, x, K=K, level=level)
    np.testing.assert_array_equal(_np(side), want_side)
    np.testing.assert_array_equal(_np(rows), want_rows)


@settings(max_examples=25, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.filter_too_much])
@given(st_systems(max_states=1 << 12), st.sampled_from(("st", "global", "flow")), st.integers(1, 3),
       st.integers(64, 3000), st.integers(1, 48), st.integers(2, 400), st.integers(1, 12))
def test_random_stage1_loops(rsr_ctx, sysd, kind, d, N, picks, max_rows, iters):
    """The Stage-1 loop (section 3.5) on random multigraphs of every system
    kind, from empty reference sets: the same rows in the same order, the same
    iteration count, unclassified fraction, searches and duplicates as the
    oracle's loop."""
    graph, K, level, p, seed = sysd
    n = graph["edge_u"].size
    rng = np.random.default_rng(seed + 7)
    if kind == "global":
        K, level = 2, 1 + (d - 1) % 2
        p = rng.uniform(0.05, 1.0, (n, 2))
        p = np.ascontiguousarray(p / p.sum(axis=1, keepdims=True))
        sysm = R.System(rsr_ctx, graph, level=level, kind="global")
    elif kind == "flow":
        level = d
        sysm = R.System(rsr_ctx, graph, K=K, level=level, kind="flow")
    else:
        sysm = R.System(rsr_ctx, graph, K=K, level=level)
    print(f"{kind} K={K} level={level} n={n} N={N} picks={picks} rows<={max_rows} iters={iters}",
          flush=True)
    m = R.Model(rsr_ctx, p)
    lo, up, info = R.stage1(rsr_ctx, m, sysm, N, picks, 1e-9, max_rows, iters, seed)
    wlo, wup, winfo = oracle.stage1(graph, p, N, picks, 1e-9, max_rows, iters, seed, K=K,
                                    level=level, kind=kind)
    for key in ("iterations", "p_u", "searches", "duplicates"):
        assert info[key] == winfo[key], key
    np.testing.assert_array_equal(lo, wlo)
    np.testing.assert_array_equal(up, wup)
