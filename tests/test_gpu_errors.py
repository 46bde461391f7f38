"""GPU tests of the error paths of the C ABI: every entry point rejects
invalid arguments with RSR_EINVAL (or RSR_EUNSUPPORTED for requests outside
the build's limits) before launching anything, leaves a message, and the
context stays usable; allocation failures injected with rsr_debug_fail_alloc
surface as RSR_ENOMEM, release what was allocated and leave the context
usable (the hot path afterwards still equals the oracle)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2604_17066_amd as R
import workloads as WL
from paper_2604_17066_amd import _abi as A

pytestmark = pytest.mark.gpu

P = R.api._ptr


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _check_path_still_exact(ctx):
    """A small full pass (sample, classify, evaluate, estimate, gradient)
    against the oracle."""
    cfg = WL.configs.tiny(N=8_000)
    lower, upper = cfg["lower"][:-3], cfg["upper"][:-10]
    model = R.Model(ctx, cfg["p"])
    refs = R.Refs(ctx, cfg["n"], 2, lower, upper)
    system = R.System(ctx, cfg["graph"])
    est, buf = R.stage2(ctx, model, refs, system, cfg["N"], cfg["seed"])
    x = oracle.sample(cfg["p"], cfg["seed"], 0, 0, cfg["N"])
    fl, _, _ = oracle.classify(lower, upper, x, mode=0)
    Y, _ = oracle.eval_unknown(cfg["graph"], x, fl)
    oest = oracle.estimate(oracle.counts(fl, Y))
    np.testing.assert_array_equal(_np(buf.flags), fl)
    np.testing.assert_array_equal(_np(buf.Y), Y)
    assert est["P"] == oest[3]


def _err(ctx):
    raw = A.lib().rsr_last_error(ctx.h)
    return raw.decode() if raw else ""


@pytest.fixture
def setup(rsr_ctx):
    cfg = WL.configs.tiny(N=1_000)
    n = cfg["n"]
    model = R.Model(rsr_ctx, cfg["p"])
    refs = R.Refs(rsr_ctx, n, 2, cfg["lower"], cfg["upper"])
    system = R.System(rsr_ctx, cfg["graph"])
    buf = R.Buffers(rsr_ctx, n, 2, cfg["N"])
    R.stage2(rsr_ctx, model, refs, system, cfg["N"], 1, buffers=buf)
    return cfg, model, refs, system, buf


def test_einval_per_entry_point(rsr_ctx, setup):
    cfg, model, refs, system, buf = setup
    lib, h, N, n = A.lib(), rsr_ctx.h, cfg["N"], cfg["n"]
    x, f, Y, G = P(buf.samples), P(buf.flags), P(buf.Y), P(buf.G)
    out = ctypes.c_void_p()
    p = np.ascontiguousarray(cfg["p"])
    bad_p = p.copy()
    bad_p[0] = [0.5, 0.6]
    rows = np.zeros((2, n), dtype=np.uint8)
    bad_rows = rows.copy()
    bad_rows[1, 3] = 2                      # a state >= K
    eu = np.ascontiguousarray(cfg["graph"]["edge_u"], dtype=np.int32)
    ev = np.ascontiguousarray(cfg["graph"]["edge_v"], dtype=np.int32)
    i32p = ctypes.POINTER(ctypes.c_int32)

    def desc(**kw):
        d = dict(kind=A.RSR_SYS_ST_CONNECTIVITY, n_nodes=cfg["graph"]["n_nodes"], n_edges=n, K=2,
                 edge_u=eu.ctypes.data_as(i32p), edge_v=ev.ctypes.data_as(i32p),
                 source=cfg["graph"]["source"], sink=cfg["graph"]["sink"], level=1)
        d.update(kw)
        return A.rsr_system_desc(**d)

    picks = torch.zeros(4, dtype=torch.int64, device="cuda")
    rows_d = torch.empty((4, n), dtype=torch.uint8, device="cuda")
    side_d = torch.empty(4, dtype=torch.uint8, device="cuda")
    est = A.rsr_estimate_t()
    I = torch.empty(n, dtype=torch.float32, device="cuda")
    lo = np.zeros((8, n), dtype=np.uint8)
    prm = A.rsr_stage1_params(1000, 4, 1e-3, 8, 3, 1)
    res = A.rsr_stage1_result()
    cases = {
        "rsr_model_create: row sum": lib.rsr_model_create(h, n, 2, bad_p.ctypes.data, ctypes.byref(out)),
        "rsr_model_create: K=1": lib.rsr_model_create(h, n, 1, p.ctypes.data, ctypes.byref(out)),
        "rsr_model_update: row sum": lib.rsr_model_update(model.h, bad_p.ctypes.data),
        "rsr_refs_create: state >= K": lib.rsr_refs_create(h, n, 2, bad_rows.ctypes.data, 2, None, 0,
                                                           ctypes.byref(out)),
        "rsr_refs_create: NULL rows": lib.rsr_refs_create(h, n, 2, None, 2, None, 0, ctypes.byref(out)),
        "rsr_refs_create: negative R": lib.rsr_refs_create(h, n, 2, None, -1, None, 0, ctypes.byref(out)),
        "rsr_system_create: source = sink": lib.rsr_system_create(h, ctypes.byref(desc(sink=cfg["graph"]["source"])),
                                                                  ctypes.byref(out)),
        "rsr_system_create: level": lib.rsr_system_create(h, ctypes.byref(desc(level=2)), ctypes.byref(out)),
        "rsr_system_create: kind": lib.rsr_system_create(h, ctypes.byref(desc(kind=9)), ctypes.byref(out)),
        "rsr_system_create: no phi": lib.rsr_system_create(h, ctypes.byref(desc(kind=A.RSR_SYS_HOST_CALLBACK)),
                                                           ctypes.byref(out)),
        "rsr_sample: N=0": lib.rsr_sample(h, model.h, 1, 0, 0, 0, x),
        "rsr_sample: NULL": lib.rsr_sample(h, model.h, 1, 0, 0, N, None),
        "rsr_classify: mode": lib.rsr_classify(h, refs.h, x, N, 7, 0, f, None),
        "rsr_classify: form": lib.rsr_classify(h, refs.h, x, N, 0, 9, f, None),
        "rsr_classify: N<0": lib.rsr_classify(h, refs.h, x, -5, 0, 0, f, None),
        "rsr_eval_unknown: which": lib.rsr_eval_unknown(h, system.h, x, N, f, 5, Y, None),
        "rsr_eval_unknown: no flags": lib.rsr_eval_unknown(h, system.h, x, N, None, 0, Y, None),
        "rsr_estimate: N=0": lib.rsr_estimate(h, f, Y, 0, ctypes.byref(est)),
        "rsr_estimate: NULL out": lib.rsr_estimate(h, f, Y, N, None),
        "rsr_grad: NULL G": lib.rsr_grad(h, model.h, x, Y, N, None, None),
        "rsr_importance: N=0": lib.rsr_importance(h, model.h, x, Y, 0, P(I)),
        "rsr_boundary_search: n_pick<0": lib.rsr_boundary_search(h, system.h, x, N, P(picks), -1,
                                                                  P(rows_d), P(side_d)),
        "rsr_boundary_search: N": lib.rsr_boundary_search(h, system.h, x, 0, P(picks), 4, P(rows_d),
                                                          P(side_d)),
        "rsr_stage1: cap": lib.rsr_stage1(h, model.h, system.h, ctypes.byref(prm), None, 0, None, 0,
                                          lo.ctypes.data, 2, lo.ctypes.data, 2, ctypes.byref(res)),
        "rsr_plan_create: no jobs": lib.rsr_plan_create(h, None, 0, None, ctypes.byref(out)),
    }
    for name, st in cases.items():
        assert st == A.RSR_EINVAL, f"{name}: status {st}"
        assert _err(rsr_ctx), name
    # rsr_importance needs K = 2.
    m3 = R.Model(rsr_ctx, np.full((4, 3), 1.0 / 3.0))
    x3 = R.rsr_sample(rsr_ctx, m3, 1, 0, 0, 64)
    Y3 = torch.zeros(64, dtype=torch.uint8, device="cuda")
    assert lib.rsr_importance(h, m3.h, P(x3), P(Y3), 64, P(I)) == A.RSR_EINVAL
    # Requests beyond the build's limits.
    big = np.full((5000, 2), 0.5)
    assert lib.rsr_model_create(h, 5000, 2, big.ctypes.data, ctypes.byref(out)) == A.RSR_EUNSUPPORTED
    # The persistent cascade takes LABEL mode on consistent rows only.
    assert lib.rsr_classify(h, refs.h, x, N, A.RSR_COUNT, A.RSR_PERSIST, f, None) == A.RSR_EUNSUPPORTED
    assert "persistent" in _err(rsr_ctx)
    both = R.Refs(rsr_ctx, n, 2, np.ones((1, n), np.uint8), np.zeros((1, n), np.uint8))
    assert not both.consistent
    assert lib.rsr_classify(h, both.h, x, N, A.RSR_LABEL, A.RSR_PERSIST, f, None) == A.RSR_EUNSUPPORTED
    assert lib.rsr_classify(h, refs.h, x, N, 0, R.RSR_MFMA, f, None) == A.RSR_OK
    assert lib.rsr_classify(h, refs.h, x, N, A.RSR_LABEL, A.RSR_PERSIST, f, None) == A.RSR_OK
    _check_path_still_exact(rsr_ctx)


def test_plan_results_rejects_null_and_context_survives(rsr_ctx, setup):
    cfg, model, refs, system, buf = setup
    plan = R.Plan(rsr_ctx, [{"model": model, "refs": refs, "system": system, "seed": 3,
                             "N": cfg["N"], "buffers": buf}], tune=False)
    assert A.lib().rsr_plan_results(plan.h, None, None) == A.RSR_EINVAL
    plan.run()
    est, _ = plan.results()
    assert est[0]["N"] == cfg["N"]
    plan.close()
    _check_path_still_exact(rsr_ctx)


@pytest.mark.parametrize("target", ["model", "refs", "system", "ctx", "plan", "classify",
                                    "stage1", "callback"])
def test_injected_enomem_leaves_context_usable(rsr_ctx, target):
    """Arms the allocation failure at every allocation the call makes in turn
    (0, 1, 2, ... successful ones first) until the call succeeds; each failure
    must be RSR_ENOMEM with a message, and the library must work afterwards."""
    lib = A.lib()
    cfg = WL.configs.tiny(N=3_000)
    n = cfg["n"]
    p = np.ascontiguousarray(cfg["p"])
    graph = cfg["graph"]
    def attempt():
        if target == "model":
            R.Model(rsr_ctx, p).close()
        elif target == "refs":
            R.Refs(rsr_ctx, n, 2, cfg["lower"], cfg["upper"]).close()
        elif target == "system":
            R.System(rsr_ctx, graph).close()
        elif target == "ctx":
            R.Context(0).close()
        elif target == "plan":
            model = R.Model(rsr_ctx, p)
            refs = R.Refs(rsr_ctx, n, 2, cfg["lower"], cfg["upper"])
            system = R.System(rsr_ctx, graph)
            buf = R.Buffers(rsr_ctx, n, 2, 3000)
            R.Plan(rsr_ctx, [{"model": model, "refs": refs, "system": system, "seed": 1,
                              "N": 3000, "buffers": buf}], tune=False).close()
        elif target == "classify":
            # A fresh context grows its cascade workspace on the first LABEL call.
            c2 = R.Context(0)
            handles = []
            try:
                model = R.Model(c2, p)
                refs = R.Refs(c2, n, 2, cfg["lower"], cfg["upper"])
                handles += [model, refs]
                xs = R.rsr_sample(c2, model, 1, 0, 0, 3000)
                lib.rsr_debug_fail_alloc(armed[0])
                try:
                    R.rsr_classify(c2, refs, xs, 3000)
                finally:
                    lib.rsr_debug_fail_alloc(-1)
                torch.cuda.synchronize()
            finally:
                # Handles are destroyed before their context.
                for hd in handles:
                    hd.close()
                c2.close()
        elif target == "stage1":
            model = R.Model(rsr_ctx, p)
            system = R.System(rsr_ctx, graph)
            R.stage1(rsr_ctx, model, system, 2_000, 4, 1e-4, 60, 3, 1)
        elif target == "callback":
            # A fresh context grows its list and callback staging on first use.
            c2 = R.Context(0)
            handles = []
            try:
                model = R.Model(c2, p)
                refs = R.Refs(c2, n, 2, cfg["lower"][:1], cfg["upper"][:1])
                cb = R.System(c2, None, K=2, level=1, kind="callback",
                              phi=lambda x: oracle.phi_st(graph, x), n=n)
                handles += [model, refs, cb]
                xs = R.rsr_sample(c2, model, 2, 0, 0, 3000)
                fl = R.rsr_classify(c2, refs, xs, 3000)
                lib.rsr_debug_fail_alloc(armed[0])
                try:
                    R.rsr_eval_unknown(c2, cb, xs, 3000, fl)
                finally:
                    lib.rsr_debug_fail_alloc(-1)
                torch.cuda.synchronize()
            finally:
                for hd in handles:
                    hd.close()
                c2.close()

    armed = [0]
    failures = 0
    for k in range(64):
        armed[0] = k
        if target not in ("classify", "callback"):
            lib.rsr_debug_fail_alloc(k)
        try:
            attempt()
            ok = True
        except R.RSRError as e:
            ok = False
            assert e.status == A.RSR_ENOMEM, f"allocation {k}: {e}"
            assert str(e).split(":", 1)[1].strip(), f"allocation {k}: no message"
            failures += 1
        finally:
            lib.rsr_debug_fail_alloc(-1)
        torch.cuda.synchronize()
        if ok:
            break
    assert ok and failures >= 1, (target, failures)
    _check_path_still_exact(rsr_ctx)


def test_persistent_barrier_timeout_is_reported(rsr_ctx):
    """The persistent cascade's grid barriers wait with a time limit.  Forced
    to zero from the host (rsr_debug_barrier_timeout), a block that would
    wait gives up at once and sets the error flag, every launch still ends,
    and the next rsr_estimate reports RSR_EHIP; with the default limit
    restored, the same classification equals the oracle."""
    cfg = WL.configs.batched(n_scen=1, N=1, graphs=[5], ref_scale=1.0)
    sd = cfg["systems"][0]
    n, p = sd["n"], cfg["jobs"][0]["p"]
    N = 100_000
    model = R.Model(rsr_ctx, p)
    xs = R.rsr_sample(rsr_ctx, model, 7, 0, 0, N)
    refs = R.Refs(rsr_ctx, n, 2, sd["lower"], sd["upper"])
    lib = A.lib()
    try:
        assert lib.rsr_debug_barrier_timeout(0) == A.RSR_OK
        fl = R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_LABEL, R.RSR_PERSIST)
        with pytest.raises(R.RSRError) as ei:
            R.rsr_estimate(rsr_ctx, fl, None, N)
        assert ei.value.status == A.RSR_EHIP
        assert "timed out" in str(ei.value)
    finally:
        lib.rsr_debug_barrier_timeout(-1)
    fl = R.rsr_classify(rsr_ctx, refs, xs, N, R.RSR_LABEL, R.RSR_PERSIST)
    est = R.rsr_estimate(rsr_ctx, fl, None, N)
    idx = np.unique(np.concatenate([np.arange(0, N, 211), [N - 1]]))
    x = oracle.sample_at(p, 7, 0, idx.astype(np.uint64))
    want, _, _ = oracle.classify(sd["lower"], sd["upper"], x, mode=0)
    np.testing.assert_array_equal(_np(fl)[idx], want)
    assert est["n_L"] + est["n_U"] + est["n_u"] == N
