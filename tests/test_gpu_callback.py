"""GPU tests of a system function given as a host callback
(RSR_SYS_HOST_CALLBACK): Stage-2 evaluation, the boundary search and the
Stage-1 loop must give exactly what the built-in s-t connectivity system and
the oracle give for the same Phi, with Phi called only on the samples the
reference states leave unclassified."""
import numpy as np
import pytest
import torch

import oracle
import paper_2604_17066_amd as R
import workloads as WL

pytestmark = pytest.mark.gpu


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


class CountingPhi:
    """s-t connectivity of a graph at a level, by the oracle's BFS, counting
    calls and recording the states it was called with."""

    def __init__(self, graph, level=1):
        self.graph, self.level, self.calls = graph, level, 0
        self.seen = []

    def __call__(self, x):
        self.calls += 1
        self.seen.append(x.copy())
        # The callback returns the system state S; Phi = [S >= level] with level 1
        # in the library, so return Phi of the requested level directly.
        return oracle.phi_st(self.graph, x, level=self.level)


@pytest.mark.parametrize("which", [R.RSR_UNKNOWN_ONLY, R.RSR_ALL])
def test_callback_eval_equals_builtin_and_oracle(rsr_ctx, which):
    cfg = WL.configs.graph2(N=30_000)
    N, n = cfg["N"], cfg["n"]
    lower, upper = cfg["lower"][:300], cfg["upper"][:300]
    refs = R.Refs(rsr_ctx, n, 2, lower, upper)
    model = R.Model(rsr_ctx, cfg["p"])
    phi = CountingPhi(cfg["graph"])
    cb = R.System(rsr_ctx, None, K=2, level=1, kind="callback", phi=phi, n=n)
    builtin = R.System(rsr_ctx, cfg["graph"])
    xs = R.rsr_sample(rsr_ctx, model, cfg["seed"], 0, 0, N)
    flags = R.rsr_classify(rsr_ctx, refs, xs, N)
    n_ev = torch.zeros(1, dtype=torch.int64, device="cuda")
    Y_cb = R.rsr_eval_unknown(rsr_ctx, cb, xs, N, flags, which=which, n_evaluated=n_ev)
    Y_bi = R.rsr_eval_unknown(rsr_ctx, builtin, xs, N, flags, which=which)
    np.testing.assert_array_equal(_np(Y_cb), _np(Y_bi))
    x = oracle.sample(cfg["p"], cfg["seed"], 0, 0, N)
    fl, _, _ = oracle.classify(lower, upper, x, mode=0)
    np.testing.assert_array_equal(_np(flags), fl)
    Y, nev = oracle.eval_unknown(cfg["graph"], x, fl, which=1 if which == R.RSR_ALL else 0)
    np.testing.assert_array_equal(_np(Y_cb), Y)
    # Phi ran exactly on the samples that needed it, in index order.
    expect = N if which == R.RSR_ALL else int((fl == 0).sum())
    assert phi.calls == expect == int(_np(n_ev)[0])
    todo = np.arange(N) if which == R.RSR_ALL else np.nonzero(fl == 0)[0]
    np.testing.assert_array_equal(np.array(phi.seen).reshape(-1, n), x[todo])


def test_callback_multistate_level(rsr_ctx):
    """K = 3 states: the callback returns the bottleneck level S and the system
    compares it with `level`."""
    cfg = WL.configs.multi(N=5_000, R_per_level=400)
    n, N = cfg["n"], cfg["N"]
    g = cfg["graph"]

    def bottleneck(x):
        return 2 if oracle.phi_st(g, x, level=2) else (1 if oracle.phi_st(g, x, level=1) else 0)

    model = R.Model(rsr_ctx, cfg["p"])
    xs = R.rsr_sample(rsr_ctx, model, cfg["seed"], 0, 0, N)
    x = oracle.sample(cfg["p"], cfg["seed"], 0, 0, N)
    for level in (1, 2):
        lv = cfg["levels"][level]
        refs = R.Refs(rsr_ctx, n, 3, lv["lower"], lv["upper"])
        cb = R.System(rsr_ctx, None, K=3, level=level, kind="callback", phi=bottleneck, n=n)
        flags = R.rsr_classify(rsr_ctx, refs, xs, N)
        Y = R.rsr_eval_unknown(rsr_ctx, cb, xs, N, flags)
        fl, _, _ = oracle.classify(lv["lower"], lv["upper"], x, mode=0)
        Yo, _ = oracle.eval_unknown(g, x, fl, level=level)
        np.testing.assert_array_equal(_np(Y), Yo)


def test_callback_boundary_search_equals_oracle(rsr_ctx):
    cfg = WL.configs.tiny(N=4_000)
    n = cfg["n"]
    model = R.Model(rsr_ctx, cfg["p"])
    xs = R.rsr_sample(rsr_ctx, model, 5, 0, 0, cfg["N"])
    cb = R.System(rsr_ctx, None, K=2, level=1, kind="callback",
                  phi=lambda x: oracle.phi_st(cfg["graph"], x), n=n)
    builtin = R.System(rsr_ctx, cfg["graph"])
    picks = torch.tensor([0, 7, 3999, -1, 4000, 123, 2500], dtype=torch.int64, device="cuda")
    rows0 = torch.full((picks.numel(), n), 9, dtype=torch.uint8, device="cuda")
    rows_cb, side_cb = R.rsr_boundary_search(rsr_ctx, cb, xs, cfg["N"], picks, rows=rows0.clone())
    rows_bi, side_bi = R.rsr_boundary_search(rsr_ctx, builtin, xs, cfg["N"], picks,
                                             rows=rows0.clone())
    sc, sb = _np(side_cb), _np(side_bi)
    np.testing.assert_array_equal(sc, sb)
    assert sc[3] == 0xFF and sc[4] == 0xFF
    rc, rb = _np(rows_cb), _np(rows_bi)
    np.testing.assert_array_equal(rc, rb)
    assert np.all(rc[3] == 9) and np.all(rc[4] == 9)      # invalid picks: rows untouched
    valid = [0, 1, 2, 5, 6]
    idx = _np(picks)[valid].astype(np.uint64)
    x = oracle.sample_at(cfg["p"], 5, 0, idx)
    rows_o, side_o, _ = oracle.boundary_st(cfg["graph"], x)
    np.testing.assert_array_equal(rc[valid], rows_o)
    np.testing.assert_array_equal(sc[valid], side_o)


def test_callback_stage1_equals_builtin(rsr_ctx):
    cfg = WL.configs.tiny(N=10)
    model = R.Model(rsr_ctx, cfg["p"])
    cb = R.System(rsr_ctx, None, K=2, level=1, kind="callback",
                  phi=lambda x: oracle.phi_st(cfg["graph"], x), n=cfg["n"])
    builtin = R.System(rsr_ctx, cfg["graph"])
    a = R.stage1(rsr_ctx, model, cb, 5_000, 8, 1e-4, 400, 12, 3)
    b = R.stage1(rsr_ctx, model, builtin, 5_000, 8, 1e-4, 400, 12, 3)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    assert a[2] == b[2]


def test_callback_negative_state_is_an_error_and_context_survives(rsr_ctx):
    cfg = WL.configs.tiny(N=2_000)
    n = cfg["n"]
    model = R.Model(rsr_ctx, cfg["p"])
    refs = R.Refs(rsr_ctx, n, 2, cfg["lower"][:2], cfg["upper"][:2])
    bad = R.System(rsr_ctx, None, K=2, level=1, kind="callback", phi=lambda x: -1, n=n)
    xs = R.rsr_sample(rsr_ctx, model, 1, 0, 0, cfg["N"])
    flags = R.rsr_classify(rsr_ctx, refs, xs, cfg["N"])
    with pytest.raises(R.RSRError) as ei:
        R.rsr_eval_unknown(rsr_ctx, bad, xs, cfg["N"], flags)
    assert ei.value.status == R.RSR_EINVAL
    # A Python exception inside phi is reported the same way.
    def boom(x):
        raise ValueError("no")
    bad2 = R.System(rsr_ctx, None, K=2, level=1, kind="callback", phi=boom, n=n)
    with pytest.raises(R.RSRError):
        R.rsr_eval_unknown(rsr_ctx, bad2, xs, cfg["N"], flags)
    good = R.System(rsr_ctx, None, K=2, level=1, kind="callback",
                    phi=lambda x: oracle.phi_st(cfg["graph"], x), n=n)
    Y = R.rsr_eval_unknown(rsr_ctx, good, xs, cfg["N"], flags)
    x = oracle.sample(cfg["p"], 1, 0, 0, cfg["N"])
    fl, _, _ = oracle.classify(cfg["lower"][:2], cfg["upper"][:2], x, mode=0)
    Yo, _ = oracle.eval_unknown(cfg["graph"], x, fl)
    np.testing.assert_array_equal(_np(Y), Yo)


def test_callback_system_rejected_by_plans(rsr_ctx):
    cfg = WL.configs.tiny(N=1_000)
    n = cfg["n"]
    refs = R.Refs(rsr_ctx, n, 2, cfg["lower"], cfg["upper"])
    cb = R.System(rsr_ctx, None, K=2, level=1, kind="callback", phi=lambda x: 1, n=n)
    jobs = [{"model": R.Model(rsr_ctx, cfg["p"]), "refs": refs, "system": cb, "seed": 1,
             "N": 1000, "buffers": R.Buffers(rsr_ctx, n, 2, 1000)}]
    with pytest.raises(R.RSRError) as ei:
        R.Plan(rsr_ctx, jobs, tune=False)
    assert ei.value.status == R.RSR_EUNSUPPORTED
